"""ctypes binding of the C ABI in include/fewha.h (argument marshalling only).

Device memory and streams come from PyTorch; every computation runs in the HIP kernels of
libfewha.so.  There is no fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfewha.so")

FEWHA_ABI_VERSION = 3
FEWHA_MAX_LEVELS = 10
FEWHA_E_BREAKDOWN = 5
FLAG_BREAKDOWN, FLAG_TOL_UNMET, FLAG_WS_REJECTED, FLAG_BAD_RHS = 1, 2, 4, 8
FEWHA_FP64, FEWHA_FP32_OP_FP64_RED = 0, 1
FEWHA_RECYCLE_PAPER, FEWHA_RECYCLE_GALERKIN = 0, 1
PIECE_WINV, PIECE_WINVT, PIECE_A, PIECE_AT = 0, 1, 2, 3
STATUS = {0: "FEWHA_OK", 1: "FEWHA_E_INVAL", 2: "FEWHA_E_NOMEM", 3: "FEWHA_E_HIP", 4: "FEWHA_E_NOT_SPD",
          5: "FEWHA_E_BREAKDOWN", 6: "FEWHA_E_STATE"}

EXPORTS = ["fewha_workspace_size", "fewha_setup", "fewha_workspace_size_batch", "fewha_setup_batch",
           "fewha_instances", "fewha_frame_iterations", "fewha_sizes", "fewha_apply_A", "fewha_rhs",
           "fewha_solve_aug", "fewha_apply_A_noalloc", "fewha_reset", "fewha_apply_piece", "fewha_get_vector", "fewha_state_size",
           "fewha_get_state", "fewha_set_state", "fewha_use_graphs", "fewha_profile", "fewha_profile_read",
           "fewha_kernel_name", "fewha_time_kernel", "fewha_wavelet_steps", "fewha_get_tuning", "fewha_set_tuning",
           "fewha_autotune", "fewha_destroy", "fewha_last_error",
           "fewha_unet_workspace_size", "fewha_unet_setup", "fewha_unet_num_params", "fewha_unet_num_nodes",
           "fewha_unet_set_params", "fewha_unet_get_params", "fewha_unet_forward", "fewha_unet_backward",
           "fewha_unet_adam_step", "fewha_unet_get_grads", "fewha_unet_destroy", "fewha_unet_last_error",
           "fewha_unet_groups", "fewha_solve_aug_ws", "fewha_warmstart_input",
           "fewha_loop_workspace_size", "fewha_loop_setup", "fewha_loop_num_actuators", "fewha_loop_step",
           "fewha_loop_piece", "fewha_loop_get_commands", "fewha_loop_set_commands", "fewha_loop_destroy", "fewha_loop_last_error"]
LOOP_DM_SLOPES, LOOP_FIT = 0, 1
UNET_MAX_GROUPS = 8


class fewha_layer(C.Structure):
    _fields_ = [("height", C.c_double), ("weight", C.c_double), ("spacing", C.c_double),
                ("origin_x", C.c_double), ("origin_y", C.c_double), ("n", C.c_int32), ("levels", C.c_int32)]


class fewha_wfs(C.Structure):
    _fields_ = [("n_sub", C.c_int32), ("pad_", C.c_int32), ("subap", C.c_double), ("theta_x", C.c_double),
                ("theta_y", C.c_double), ("lgs_height", C.c_double), ("slope_weight", C.POINTER(C.c_double)),
                ("cross_weight", C.POINTER(C.c_double)), ("tt_filter", C.c_int32), ("pad2_", C.c_int32)]


class fewha_config(C.Structure):
    _fields_ = [("abi_version", C.c_int32), ("n_layers", C.c_int32), ("layers", C.POINTER(fewha_layer)),
                ("n_wfs", C.c_int32), ("pad_", C.c_int32), ("wfs", C.POINTER(fewha_wfs)),
                ("alpha", C.c_double), ("r0", C.c_double), ("L0", C.c_double),
                ("prior_diag", C.POINTER(C.c_double)), ("precond_inv", C.POINTER(C.c_double)),
                ("max_iter", C.c_int32), ("recycle_k", C.c_int32), ("recycle_mode", C.c_int32),
                ("project_all", C.c_int32), ("rel_tol", C.c_double), ("precision", C.c_int32),
                ("block_elems", C.c_int32), ("pad2_", C.c_int32), ("level_weight", C.POINTER(C.c_double))]


class fewha_solve_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("recycle_used", C.c_int32), ("dropped", C.c_int32),
                ("flags", C.c_int32), ("rel_res", C.c_double)]


class fewha_unet_config(C.Structure):
    _fields_ = [("abi_version", C.c_int32), ("n_groups", C.c_int32), ("images", C.c_int32 * 8),
                ("size", C.c_int32 * 8), ("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float)]


class fewha_warmstart(C.Structure):
    _fields_ = [("scale_c", C.c_float), ("scale_r", C.c_float), ("scale_out", C.c_float)]


class fewha_tuning(C.Structure):
    _fields_ = [("syn_tile", C.c_int32), ("gather_rows", C.c_int32), ("reserved", C.c_int32 * 6)]


class fewha_dm(C.Structure):
    _fields_ = [("height", C.c_double), ("spacing", C.c_double), ("origin_x", C.c_double), ("origin_y", C.c_double),
                ("n", C.c_int32), ("pad_", C.c_int32)]


class fewha_loop_config(C.Structure):
    _fields_ = [("abi_version", C.c_int32), ("n_dm", C.c_int32), ("dms", C.POINTER(fewha_dm)), ("gain", C.c_double),
                ("closed", C.c_int32), ("fit_iter", C.c_int32), ("n_dirs", C.c_int32), ("n_pts", C.c_int32),
                ("dirs", C.POINTER(C.c_double)), ("pupil_d", C.c_double), ("obstruction", C.c_double)]


class FewhaError(RuntimeError):
    pass


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libfewha.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FewhaError(f"{path} is missing: build it with paper_2011_06842_amd.build.build()")
    lib = C.CDLL(path)
    vp, st = C.c_void_p, C.c_int
    sig = {
        "fewha_workspace_size": ([C.POINTER(fewha_config), C.POINTER(C.c_size_t)], st),
        "fewha_setup": ([C.POINTER(fewha_config), vp, C.c_size_t, vp, C.POINTER(vp)], st),
        "fewha_workspace_size_batch": ([C.POINTER(fewha_config), C.c_int32, C.POINTER(C.c_size_t)], st),
        "fewha_setup_batch": ([C.POINTER(fewha_config), C.c_int32, vp, C.c_size_t, vp, C.POINTER(vp)], st),
        "fewha_instances": ([vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.c_int32, C.POINTER(C.c_int32)], st),
        "fewha_frame_iterations": ([vp, C.POINTER(C.c_int32)], st),
        "fewha_sizes": ([vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)], st),
        "fewha_apply_A": ([vp, vp, vp, vp], st),
        "fewha_apply_A_noalloc": ([vp, vp, vp, vp], st),
        "fewha_rhs": ([vp, vp, vp, vp], st),
        "fewha_solve_aug": ([vp, vp, vp, vp, vp], st),
        "fewha_reset": ([vp], st),
        "fewha_apply_piece": ([vp, C.c_int32, vp, vp, vp], st),
        "fewha_get_vector": ([vp, C.c_int32, vp, vp], st),
        "fewha_state_size": ([vp, C.POINTER(C.c_size_t)], st),
        "fewha_get_state": ([vp, vp, vp], st),
        "fewha_set_state": ([vp, vp, vp], st),
        "fewha_use_graphs": ([vp, C.c_int32], st),
        "fewha_profile": ([vp, C.c_int32], st),
        "fewha_profile_read": ([vp, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32, C.POINTER(C.c_int32)], st),
        "fewha_kernel_name": ([C.c_int32], C.c_char_p),
        "fewha_time_kernel": ([vp, C.c_int32, C.c_int32, C.c_int32, vp, C.POINTER(C.c_float)], st),
        "fewha_wavelet_steps": ([vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int32)], st),
        "fewha_get_tuning": ([vp, C.POINTER(fewha_tuning)], st),
        "fewha_set_tuning": ([vp, C.POINTER(fewha_tuning)], st),
        "fewha_autotune": ([vp, C.c_int32, vp, C.POINTER(fewha_tuning), C.POINTER(C.c_float), C.c_int32,
                            C.POINTER(C.c_int32)], st),
        "fewha_destroy": ([vp], st),
        "fewha_last_error": ([vp], C.c_char_p),
        "fewha_unet_workspace_size": ([C.POINTER(fewha_unet_config), C.POINTER(C.c_size_t)], st),
        "fewha_unet_setup": ([C.POINTER(fewha_unet_config), vp, C.c_size_t, vp, C.POINTER(vp)], st),
        "fewha_unet_num_params": ([vp, C.POINTER(C.c_int64)], st),
        "fewha_unet_num_nodes": ([vp, C.POINTER(C.c_int64)], st),
        "fewha_unet_set_params": ([vp, vp, vp], st),
        "fewha_unet_get_params": ([vp, vp, vp], st),
        "fewha_unet_forward": ([vp, vp, vp, vp], st),
        "fewha_unet_backward": ([vp, vp, vp, vp, vp], st),
        "fewha_unet_adam_step": ([vp, vp], st),
        "fewha_unet_get_grads": ([vp, vp, vp], st),
        "fewha_unet_destroy": ([vp], st),
        "fewha_unet_last_error": ([vp], C.c_char_p),
        "fewha_unet_groups": ([vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)], st),
        "fewha_solve_aug_ws": ([vp, vp, C.POINTER(fewha_warmstart), vp, vp, vp, vp], st),
        "fewha_warmstart_input": ([vp, C.POINTER(fewha_warmstart), vp, vp, vp, vp], st),
        "fewha_loop_workspace_size": ([vp, C.POINTER(fewha_loop_config), C.POINTER(C.c_size_t)], st),
        "fewha_loop_setup": ([vp, C.POINTER(fewha_loop_config), vp, C.c_size_t, vp, C.POINTER(vp)], st),
        "fewha_loop_num_actuators": ([vp, C.POINTER(C.c_int64)], st),
        "fewha_loop_step": ([vp, vp, vp, vp, vp], st),
        "fewha_loop_piece": ([vp, C.c_int32, vp, vp, vp], st),
        "fewha_loop_get_commands": ([vp, C.c_int32, vp, vp], st),
        "fewha_loop_set_commands": ([vp, vp, vp, vp, vp], st),
        "fewha_loop_destroy": ([vp], st),
        "fewha_loop_last_error": ([vp], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(status: int, ctx=None):
    if status != 0:
        msg = _lib.fewha_last_error(ctx).decode() if _lib is not None else ""
        raise FewhaError(f"{STATUS.get(status, status)}: {msg}")


def _ptr(t) -> int:
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def make_config(spec, prior_diag=None, precond_inv=None, keep=None):
    """fewha_config from any object with the attributes of a system description (layers with
    height/weight/spacing/origin_x/origin_y/n/levels; wfs with n_sub/subap/theta_x/theta_y/
    lgs_height/weight, optionally cross_weight/tt_filter; alpha, r0, L0, max_iter, recycle_k, recycle_mode, project_all,
    precision, optionally block_elems and level_weight).  `keep` collects the host arrays that must outlive the
    setup call."""
    keep = [] if keep is None else keep
    L, G = len(spec.layers), len(spec.wfs)
    layers = (fewha_layer * L)()
    for i, l in enumerate(spec.layers):
        layers[i] = fewha_layer(l.height, l.weight, l.spacing, l.origin_x, l.origin_y, l.n, l.levels)
    wfs = (fewha_wfs * G)()
    for i, w in enumerate(spec.wfs):
        if w.weight is None:
            raise FewhaError(f"sensor {i}: slope weights are not set")
        wt = np.ascontiguousarray(w.weight, dtype=np.float64)
        keep.append(wt)
        cw = getattr(w, "cross_weight", None)
        cwp = None
        if cw is not None:
            cw = np.ascontiguousarray(cw, dtype=np.float64)
            keep.append(cw)
            cwp = cw.ctypes.data_as(C.POINTER(C.c_double))
        wfs[i] = fewha_wfs(w.n_sub, 0, w.subap, w.theta_x, w.theta_y, w.lgs_height,
                           wt.ctypes.data_as(C.POINTER(C.c_double)), cwp, int(bool(getattr(w, "tt_filter", False))), 0)
    keep += [layers, wfs]

    def dptr(a):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=np.float64)
        keep.append(a)
        return a.ctypes.data_as(C.POINTER(C.c_double))

    cfg = fewha_config()
    cfg.abi_version = FEWHA_ABI_VERSION
    cfg.n_layers, cfg.layers = L, layers
    cfg.n_wfs, cfg.wfs = G, wfs
    cfg.alpha, cfg.r0, cfg.L0 = spec.alpha, spec.r0, spec.L0
    cfg.prior_diag = dptr(prior_diag)
    cfg.precond_inv = dptr(precond_inv)
    cfg.max_iter = spec.max_iter
    cfg.recycle_k = spec.recycle_k
    cfg.recycle_mode = FEWHA_RECYCLE_PAPER if spec.recycle_mode == "paper" else FEWHA_RECYCLE_GALERKIN
    cfg.project_all = int(bool(spec.project_all))
    cfg.rel_tol = float(getattr(spec, "rel_tol", 0.0) or 0.0)
    cfg.precision = FEWHA_FP64 if spec.precision == "fp64" else FEWHA_FP32_OP_FP64_RED
    cfg.block_elems = int(getattr(spec, "block_elems", 0) or 0)
    lw = getattr(spec, "level_weight", None)
    if lw is not None:
        w = np.ones(FEWHA_MAX_LEVELS + 1)
        w[:len(lw)] = lw
        cfg.level_weight = dptr(w)
    return cfg


def _configs(specs, prior_diag, precond_inv, keep):
    """Array of fewha_config for one system description or a list of them (a batch)."""
    batch = isinstance(specs, (list, tuple))
    specs = list(specs) if batch else [specs]
    pd = prior_diag if batch and prior_diag is not None else [prior_diag] * len(specs)
    pj = precond_inv if batch and precond_inv is not None else [precond_inv] * len(specs)
    arr = (fewha_config * len(specs))()
    for i, sp in enumerate(specs):
        arr[i] = make_config(sp, prior_diag=pd[i], precond_inv=pj[i], keep=keep)
    return arr, specs


def fewha_workspace_size(spec, prior_diag=None, precond_inv=None) -> int:
    """Workspace bytes of one system description or of a batch (a list of them)."""
    lib = load_library()
    keep = []
    arr, specs = _configs(spec, prior_diag, precond_inv, keep)
    n = C.c_size_t()
    _check(lib.fewha_workspace_size_batch(arr, len(specs), C.byref(n)))
    return n.value


class FewhaContext:
    """One solver context: owns its workspace tensor; calls mirror the C ABI names.  `spec` is
    one system description or a list of them (a batch of independent instances, solved
    together; vectors are then the concatenation over instances, see `coeff_offsets` and
    `slope_offsets`)."""

    def __init__(self, spec, device="cuda", prior_diag=None, precond_inv=None, stream=None):
        import torch
        self.lib = load_library()
        keep = []
        arr, specs = _configs(spec, prior_diag, precond_inv, keep)
        nb = len(specs)
        n = C.c_size_t()
        _check(self.lib.fewha_workspace_size_batch(arr, nb, C.byref(n)))
        self.workspace = torch.empty(n.value + 256, dtype=torch.uint8, device=device)
        base = _ptr(self.workspace)
        off = (-base) % 256
        self._ws_ptr = base + off
        ctx = C.c_void_p()
        _check(self.lib.fewha_setup_batch(arr, nb, C.c_void_p(self._ws_ptr), n.value, C.c_void_p(_stream(stream)),
                                          C.byref(ctx)))
        self.ctx = ctx
        self.dtype = torch.float64 if specs[0].precision == "fp64" else torch.float32
        self.device = device
        Nc, Sc = C.c_int64(), C.c_int64()
        _check(self.lib.fewha_sizes(self.ctx, C.byref(Nc), C.byref(Sc)), self.ctx)
        self.N, self.S = Nc.value, Sc.value
        co = (C.c_int64 * (nb + 1))()
        so = (C.c_int64 * (nb + 1))()
        cnt = C.c_int32()
        _check(self.lib.fewha_instances(self.ctx, co, so, nb + 1, C.byref(cnt)), self.ctx)
        self.B = cnt.value
        self.coeff_offsets = [co[i] for i in range(nb + 1)]
        self.slope_offsets = [so[i] for i in range(nb + 1)]
        self.breakdown_reports = []   # messages of FEWHA_E_BREAKDOWN returned by frame calls

    # -- helpers
    def _vec(self, n):
        import torch
        return torch.empty(n, dtype=self.dtype, device=self.device)

    def _in(self, t, n):
        if t.dtype != self.dtype or t.numel() != n or not t.is_contiguous() or not t.is_cuda:
            raise FewhaError(f"expected a contiguous {self.dtype} device tensor of {n} elements")
        return t

    # -- C ABI calls
    def fewha_apply_A(self, x, y=None, stream=None):
        x = self._in(x, self.N)
        y = self._vec(self.N) if y is None else self._in(y, self.N)
        _check(self.lib.fewha_apply_A(self.ctx, _ptr(x), _ptr(y), _stream(stream)), self.ctx)
        return y

    def fewha_apply_A_noalloc(self, x, y, stream=None):
        """y = M x with the library's static scratch array (see include/fewha.h); y is given."""
        x = self._in(x, self.N)
        y = self._in(y, self.N)
        _check(self.lib.fewha_apply_A_noalloc(self.ctx, _ptr(x), _ptr(y), _stream(stream)), self.ctx)
        return y

    def fewha_rhs(self, s, b=None, stream=None):
        s = self._in(s, self.S)
        b = self._vec(self.N) if b is None else self._in(b, self.N)
        _check(self.lib.fewha_rhs(self.ctx, _ptr(s), _ptr(b), _stream(stream)), self.ctx)
        return b

    def fewha_solve_aug(self, s, c=None, info=None, stream=None):
        """One frame; returns c (device tensor).  `info`, if given, is a uint8 device tensor
        (:meth:`new_info`) that receives one fewha_solve_info per instance (decode with
        :func:`decode_info`)."""
        s = self._in(s, self.S)
        c = self._vec(self.N) if c is None else self._in(c, self.N)
        ip = _ptr(info) if info is not None else None
        self._frame_status(self.lib.fewha_solve_aug(self.ctx, _ptr(s), _ptr(c), ip, _stream(stream)))
        return c

    def _frame_status(self, st):
        """FEWHA_E_BREAKDOWN from a frame call reports an earlier frame's breakdown (this call's
        frame was enqueued): it is recorded in `breakdown_reports`, not raised."""
        if st == FEWHA_E_BREAKDOWN:
            self.breakdown_reports.append(self.lib.fewha_last_error(self.ctx).decode())
        else:
            _check(st, self.ctx)

    def fewha_solve_aug_ws(self, net, scales, s, c=None, info=None, stream=None):
        """One frame warm-started by the U-Net `net` (UNetContext); scales = (scale_c,
        scale_r, scale_out).  Returns c (device tensor)."""
        s = self._in(s, self.S)
        c = self._vec(self.N) if c is None else self._in(c, self.N)
        ws = fewha_warmstart(*[float(v) for v in scales])
        ip = _ptr(info) if info is not None else None
        self._frame_status(self.lib.fewha_solve_aug_ws(self.ctx, net.net, C.byref(ws), _ptr(s), _ptr(c), ip,
                                                        _stream(stream)))
        return c

    def fewha_warmstart_input(self, scales, c, s, out=None, stream=None):
        """Network input (N, 4) FP32 device tensor of the warm start for slopes `s` after
        coefficients `c` (see include/fewha_unet.h); scales = (scale_c, scale_r[, scale_out])."""
        import torch
        c = self._in(c, self.N)
        s = self._in(s, self.S)
        out = torch.empty((self.N, 4), dtype=torch.float32, device=self.device) if out is None else out
        sc = list(scales) + [1.0] * (3 - len(scales))
        ws = fewha_warmstart(*[float(v) for v in sc])
        _check(self.lib.fewha_warmstart_input(self.ctx, C.byref(ws), _ptr(c), _ptr(s), _ptr(out), _stream(stream)),
               self.ctx)
        return out

    def fewha_frame_iterations(self) -> int:
        n = C.c_int32()
        _check(self.lib.fewha_frame_iterations(self.ctx, C.byref(n)), self.ctx)
        return n.value

    def fewha_reset(self):
        _check(self.lib.fewha_reset(self.ctx), self.ctx)

    def fewha_apply_piece(self, piece, x, stream=None):
        n_in = self.S if piece == PIECE_AT else self.N
        n_out = self.S if piece == PIECE_A else self.N
        x = self._in(x, n_in)
        y = self._vec(n_out)
        _check(self.lib.fewha_apply_piece(self.ctx, piece, _ptr(x), _ptr(y), _stream(stream)), self.ctx)
        return y

    def fewha_get_vector(self, which, stream=None):
        y = self._vec(self.N)
        _check(self.lib.fewha_get_vector(self.ctx, which, _ptr(y), _stream(stream)), self.ctx)
        return y

    def fewha_state_size(self):
        n = C.c_size_t()
        _check(self.lib.fewha_state_size(self.ctx, C.byref(n)), self.ctx)
        return n.value

    def fewha_get_state(self, stream=None):
        import torch
        buf = torch.empty(self.fewha_state_size(), dtype=torch.uint8, device=self.device)
        _check(self.lib.fewha_get_state(self.ctx, _ptr(buf), _stream(stream)), self.ctx)
        return buf

    def fewha_set_state(self, buf, stream=None):
        _check(self.lib.fewha_set_state(self.ctx, _ptr(buf), _stream(stream)), self.ctx)

    def fewha_use_graphs(self, enable=True):
        _check(self.lib.fewha_use_graphs(self.ctx, int(bool(enable))), self.ctx)

    def fewha_profile(self, enable=True):
        _check(self.lib.fewha_profile(self.ctx, int(bool(enable))), self.ctx)

    def fewha_profile_read(self) -> dict:
        """{kernel: (total ms, launches)} accumulated since fewha_profile(True)."""
        n = 32
        ms = (C.c_double * n)()
        ln = (C.c_int64 * n)()
        cnt = C.c_int32()
        _check(self.lib.fewha_profile_read(self.ctx, ms, ln, n, C.byref(cnt)), self.ctx)
        return {self.lib.fewha_kernel_name(i).decode(): (ms[i], ln[i]) for i in range(cnt.value)}

    def fewha_time_kernel(self, kernel, step=0, reps=50, stream=None) -> float:
        """Mean duration in ms of one operator kernel (see include/fewha.h)."""
        ms = C.c_float()
        _check(self.lib.fewha_time_kernel(self.ctx, kernel, step, reps, _stream(stream), C.byref(ms)), self.ctx)
        return ms.value

    def fewha_get_tuning(self) -> dict:
        """Tile shapes in use: {"syn_tile": 16 | 32, "gather_rows": 1 | 4}."""
        t = fewha_tuning()
        _check(self.lib.fewha_get_tuning(self.ctx, C.byref(t)), self.ctx)
        return {"syn_tile": t.syn_tile, "gather_rows": t.gather_rows}

    def fewha_set_tuning(self, syn_tile=0, gather_rows=None):
        t = fewha_tuning()
        t.syn_tile = int(syn_tile)
        t.gather_rows = int(self.fewha_get_tuning()["gather_rows"] if gather_rows is None else gather_rows)
        _check(self.lib.fewha_set_tuning(self.ctx, C.byref(t)), self.ctx)

    def fewha_autotune(self, reps=20, stream=None):
        """Times the tile-shape candidates on M x, keeps the fastest; returns (best, {candidate: ms})."""
        t = fewha_tuning()
        ms = (C.c_float * 6)()
        n = C.c_int32()
        _check(self.lib.fewha_autotune(self.ctx, int(reps), _stream(stream), C.byref(t), ms, 6, C.byref(n)), self.ctx)
        cands = [(16, 1), (16, 4), (32, 1), (32, 4), (64, 1), (64, 4)]
        return ({"syn_tile": t.syn_tile, "gather_rows": t.gather_rows},
                {f"syn{a}_rows{b}": float(ms[i]) for i, (a, b) in enumerate(cands[:n.value])})

    def fewha_wavelet_steps(self):
        """[(largest block, layer count)] of the tiled analysis launches (finest first)."""
        bs = (C.c_int32 * 16)()
        lc = (C.c_int32 * 16)()
        n = C.c_int32()
        _check(self.lib.fewha_wavelet_steps(self.ctx, bs, lc, 16, C.byref(n)), self.ctx)
        return [(bs[i], lc[i]) for i in range(n.value)]

    def fewha_destroy(self):
        if getattr(self, "ctx", None):
            self.lib.fewha_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.fewha_destroy()
        except Exception:
            pass

    def new_info(self):
        import torch
        return torch.zeros(C.sizeof(fewha_solve_info) * self.B, dtype=torch.uint8, device=self.device)


def decode_info(info_tensor):
    """dict of one fewha_solve_info, or a list of them for a batch."""
    raw = bytes(info_tensor.cpu().numpy().tobytes())
    sz = C.sizeof(fewha_solve_info)
    out = []
    for i in range(len(raw) // sz):
        s = fewha_solve_info.from_buffer_copy(raw[i * sz:(i + 1) * sz])
        out.append({"iters": s.iters, "recycle_used": s.recycle_used, "dropped": s.dropped, "flags": s.flags,
                    "rel_res": s.rel_res})
    return out[0] if len(out) == 1 else out


def _ucheck(status: int, net=None):
    if status != 0:
        msg = _lib.fewha_unet_last_error(net).decode() if _lib is not None else ""
        raise FewhaError(f"{STATUS.get(status, status)}: {msg}")


class UNetContext:
    """The warm-start U-Net (include/fewha_unet.h): `groups` is a list of (images, size) of
    square images; inputs are (nodes, 4) FP32, outputs (nodes,) FP32, groups in order."""

    def __init__(self, groups, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, device="cuda", stream=None):
        import torch
        self.lib = load_library()
        cfg = fewha_unet_config()
        cfg.abi_version = FEWHA_ABI_VERSION
        cfg.n_groups = len(groups)
        for g, (n, sz) in enumerate(groups):
            cfg.images[g] = n
            cfg.size[g] = sz
        cfg.lr, cfg.beta1, cfg.beta2, cfg.eps = lr, beta1, beta2, eps
        nbytes = C.c_size_t()
        _ucheck(self.lib.fewha_unet_workspace_size(C.byref(cfg), C.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=device)
        base = _ptr(self.workspace)
        net = C.c_void_p()
        _ucheck(self.lib.fewha_unet_setup(C.byref(cfg), C.c_void_p(base + (-base) % 256), nbytes.value,
                                          C.c_void_p(_stream(stream)), C.byref(net)))
        self.net = net
        self.device = device
        self.groups = list(groups)
        n = C.c_int64()
        _ucheck(self.lib.fewha_unet_num_params(self.net, C.byref(n)), self.net)
        self.n_params = n.value
        _ucheck(self.lib.fewha_unet_num_nodes(self.net, C.byref(n)), self.net)
        self.nodes = n.value

    def _f32(self, t, n):
        import torch
        if t.dtype != torch.float32 or t.numel() != n or not t.is_contiguous() or not t.is_cuda:
            raise FewhaError(f"expected a contiguous float32 device tensor of {n} elements")
        return t

    def set_params(self, params, stream=None):
        _ucheck(self.lib.fewha_unet_set_params(self.net, _ptr(self._f32(params, self.n_params)), _stream(stream)),
                self.net)

    def get_params(self, stream=None):
        import torch
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        _ucheck(self.lib.fewha_unet_get_params(self.net, _ptr(out), _stream(stream)), self.net)
        return out

    def forward(self, x, out=None, stream=None):
        import torch
        x = self._f32(x, 4 * self.nodes)
        out = torch.empty(self.nodes, dtype=torch.float32, device=self.device) if out is None else out
        _ucheck(self.lib.fewha_unet_forward(self.net, _ptr(x), _ptr(self._f32(out, self.nodes)), _stream(stream)),
                self.net)
        return out

    def backward(self, x, target, loss=None, stream=None):
        import torch
        loss = torch.zeros(1, dtype=torch.float32, device=self.device) if loss is None else loss
        _ucheck(self.lib.fewha_unet_backward(self.net, _ptr(self._f32(x, 4 * self.nodes)),
                                             _ptr(self._f32(target, self.nodes)), _ptr(loss), _stream(stream)),
                self.net)
        return loss

    def adam_step(self, stream=None):
        _ucheck(self.lib.fewha_unet_adam_step(self.net, _stream(stream)), self.net)

    def get_grads(self, stream=None):
        import torch
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        _ucheck(self.lib.fewha_unet_get_grads(self.net, _ptr(out), _stream(stream)), self.net)
        return out

    def destroy(self):
        if getattr(self, "net", None):
            self.lib.fewha_unet_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class LoopContext:
    """Closed-loop wrapper (include/fewha_loop.h) around a single-instance FewhaContext `ctx`:
    `dms` is a list of (height, n, spacing[, origin_x, origin_y]); fit_iter 0 = direct fitting,
    else that many CG iterations over the fitting directions `dirs` [(theta_x, theta_y)] on an
    n_pts x n_pts pupil grid of diameter pupil_d and obstruction ratio `obstruction`."""

    def __init__(self, ctx, dms, gain=0.4, closed=True, fit_iter=0, dirs=(), n_pts=0, pupil_d=0.0,
                 obstruction=0.0, stream=None):
        import torch
        self.lib = load_library()
        self.ctx = ctx
        arr = (fewha_dm * len(dms))()
        for i, d in enumerate(dms):
            d = tuple(d) + (0.0, 0.0)[len(d) - 3:] if len(d) < 5 else tuple(d)
            arr[i] = fewha_dm(float(d[0]), float(d[2]), float(d[3]), float(d[4]), int(d[1]), 0)
        dv = np.ascontiguousarray(np.asarray(dirs, dtype=np.float64).reshape(-1))
        cfg = fewha_loop_config()
        cfg.abi_version, cfg.n_dm, cfg.dms = FEWHA_ABI_VERSION, len(dms), arr
        cfg.gain, cfg.closed, cfg.fit_iter = float(gain), int(bool(closed)), int(fit_iter)
        cfg.n_dirs, cfg.n_pts = len(dv) // 2, int(n_pts)
        cfg.dirs = dv.ctypes.data_as(C.POINTER(C.c_double)) if dv.size else None
        cfg.pupil_d, cfg.obstruction = float(pupil_d), float(obstruction)
        self._keep = (arr, dv)
        n = C.c_size_t()
        self._lcheck(self.lib.fewha_loop_workspace_size(ctx.ctx, C.byref(cfg), C.byref(n)), None)
        self.workspace = torch.empty(n.value + 256, dtype=torch.uint8, device=ctx.device)
        base = _ptr(self.workspace)
        lp = C.c_void_p()
        self._lcheck(self.lib.fewha_loop_setup(ctx.ctx, C.byref(cfg), C.c_void_p(base + (-base) % 256), n.value,
                                               C.c_void_p(_stream(stream)), C.byref(lp)), None)
        self.loop = lp
        na = C.c_int64()
        self._lcheck(self.lib.fewha_loop_num_actuators(self.loop, C.byref(na)))
        self.n_act = na.value

    def _lcheck(self, st, use_loop=True):
        if st != 0:
            msg = self.lib.fewha_loop_last_error(self.loop if use_loop else None).decode()
            raise FewhaError(f"{STATUS.get(st, st)}: {msg}")

    def _vec(self, n):
        import torch
        return torch.empty(n, dtype=self.ctx.dtype, device=self.ctx.device)

    def step(self, s, a=None, info=None, stream=None):
        """One frame of Alg. 3; returns the new commands (device tensor)."""
        s = self.ctx._in(s, self.ctx.S)
        a = self._vec(self.n_act) if a is None else self.ctx._in(a, self.n_act)
        ip = _ptr(info) if info is not None else None
        st = self.lib.fewha_loop_step(self.loop, _ptr(s), _ptr(a), ip, _stream(stream))
        self.ctx._frame_status(st)
        return a

    def piece(self, which, x, stream=None):
        n_in = self.n_act if which == LOOP_DM_SLOPES else self.ctx.N
        n_out = self.ctx.S if which == LOOP_DM_SLOPES else self.n_act
        x = self.ctx._in(x, n_in)
        y = self._vec(n_out)
        self._lcheck(self.lib.fewha_loop_piece(self.loop, which, _ptr(x), _ptr(y), _stream(stream)))
        return y

    def get_commands(self, which, stream=None):
        y = self._vec(self.n_act)
        self._lcheck(self.lib.fewha_loop_get_commands(self.loop, which, _ptr(y), _stream(stream)))
        return y

    def set_commands(self, prev=None, cur=None, fit=None, stream=None):
        args = [None if t is None else _ptr(self.ctx._in(t, self.n_act)) for t in (prev, cur, fit)]
        self._lcheck(self.lib.fewha_loop_set_commands(self.loop, *args, _stream(stream)))

    def destroy(self):
        if getattr(self, "loop", None):
            self.lib.fewha_loop_destroy(self.loop)
            self.loop = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
