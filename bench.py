#!/usr/bin/env python3
"""Frame-solve benchmark of the augmented wavelet reconstructor on one MI355X.

Workload: the ELT-scale MCAO system (39 m, 28 % obstruction, 6 laser guide stars at 45
arcsec and 90 km with 84x84 Shack-Hartmann subapertures, 9 layers 0-20 km on a 256^2
ground grid and 128^2 grids above, periodic db3 over 6 levels, 6 PCG iterations per
frame, 10 recycled directions, FP32 operator with FP64 reductions) on a seeded synthetic
frozen-flow von Karman sequence with SNR-10 slope noise.  A step is one frame: right-hand
side, residual update, Galerkin projection, augmented PCG (Alg. 3 with Alg. 2).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--cpu-frames F] [--no-cpu-baseline]

Prints one JSON line.  `value` is operator applications per second of the whole frame
solve (6 per frame), with the slopes already resident in device memory.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "augmented-PCG frame latency p50/p99 (ms) + operator applies/s, % HBM roofline"
HBM_PEAK_GBS = 8000.0
# vector-instruction issue peak: 256 CUs x 4 SIMDs x 2.4 GHz, one wave64 instruction per SIMD
# every 4 cycles (16 lanes wide); in wave-instructions per second
VALU_PEAK_INST_S = 256 * 4 * 2.4e9 / 4
SEED = 20201112


COARSE_BLOCK = 64      # largest wavelet block a single workgroup transforms in LDS
# operator kernels in the library's profiler numbering (see include/fewha.h)
OP_KERNELS = ["idwt_coarse", "idwt_step", "data_term", "adj_gather", "dwt_step", "dwt_coarse"]
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_2011_06842_amd", "csrc")


def log(msg):
    """Progress of the legs on stderr (stdout carries the one JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def coarse_sizes(spec):
    """Per layer: side of the top-left block the coarse kernels transform in LDS (0 if none)."""
    out = []
    for l in spec.layers:
        lc = 1
        while (l.n >> (lc - 1)) > COARSE_BLOCK:
            lc += 1
        out.append(l.n >> (lc - 1) if l.levels >= lc else 0)
    return out


def op_kernel_bytes(name, step, spec, steps, N, S, V, e):
    """Algorithmic HBM bytes of one launch of an operator kernel inside M x: every operand it
    must read or write once (x, the prior and the slope weights included), intermediates
    between kernels counted once at each side, nothing counted twice within a kernel."""
    if name == "idwt_coarse":     # coarse coefficients in, coarse image (or LL band) out
        return sum(2 * b * b for b in coarse_sizes(spec)) * e
    if name == "dwt_coarse":      # LL band in; coefficients out; prior and x in
        return sum(4 * b * b for b in coarse_sizes(spec)) * e
    nb, nl = steps[step] if step is not None else (0, 0)
    if name == "idwt_step":       # LL band + 3 detail bands in, next LL band (or image) out
        return 2 * nb * nb * nl * e
    if name == "dwt_step":        # image/LL in; 3 detail bands + LL out; prior and x of the details in
        return 3.5 * nb * nb * nl * e
    if name == "data_term":       # layer images in, slope weights in, sensor nodes out
        return (N + S + V) * e
    if name == "adj_gather":      # sensor nodes in, layer images out
        return (V + N) * e
    raise ValueError(name)


def frame_kernel_bytes(name, N, S, V, e, m, it, mp):
    """Algorithmic bytes of one steady-state frame's launches of a solver kernel (m recycled
    directions, it iterations, mp directions projected in the loop)."""
    if name == "slopes_adj":      # slopes and weights in, sensor nodes out
        return (2 * S + V) * e
    if name == "residual":        # b, b_prev, r in; r, b_prev out
        return 5 * N * e
    if name == "gram":            # m U, m Q, r, J^-1 in
        return (2 * m + 2) * N * e
    if name == "galerkin_apply":  # c, r, J^-1, m U, m Q in; c, r, p_0 out
        return (6 + 2 * m) * N * e
    if name == "init_dir":        # r, J^-1 in; p_0 out (no recycled directions)
        return 3 * N * e
    if name == "update1":         # p, q, c, r, J^-1 (+ U, Q of the projection) in; c, r, z out; last: no z
        return ((it - 1) * (8 + 2 * mp) + 6) * N * e
    if name == "update2":         # z, p (+ U of the projection) in; next p out
        return (it - 1) * (3 + mp) * N * e
    return 0.0


def source_sha256():
    """Hash of the library's sources: counter figures stay valid only while it matches."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".cpp", ".h")):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def pmc_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` in `workload` ("single" or "batched") from the
    committed counter summaries, or None."""
    return pmc_value(kernel, workload, "traffic_bytes_per_launch")


def pmc_value(kernel, workload, key):
    """Value `key` of `kernel` in `workload` ("single" or "batched") from the committed counter
    summaries (profiles/*_pmc.md, blocks of "- key: value" lines starting at "- kernel:"), or
    None when none matches or the sources changed since."""
    import glob
    sha = source_sha256()
    for path in sorted(glob.glob(os.path.join(PROFILES, "*_pmc.md"))):
        with open(path) as f:
            lines = f.read().splitlines()
        blocks, cur = [], None
        for line in lines:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                k, v = k.strip(), v.strip().strip("`")
                if k == "kernel":
                    cur = {}
                    blocks.append(cur)
                if cur is not None:
                    cur[k] = v
        for blk in blocks:
            if (blk.get("kernel") == kernel and blk.get("workload") == workload and blk.get("source_sha256") == sha
                    and key in blk):
                try:
                    return float(blk[key])
                except ValueError:
                    return None
    return None


def copy_probe(mib):
    """A plain device-to-device copy of known size, run under the memory counters to scale
    FETCH_SIZE / WRITE_SIZE to bytes."""
    import torch
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": 4 * n, "launches": 5}), flush=True)
    return 0


def run_batch(args, dev):
    """Throughput form: B independent instances of the ELT geometry in one context (one frame
    advances all of them).  Instance i reads the slope stream of atmosphere i mod A at a time
    offset, so that every instance sees its own frames; all share the noise weights, hence
    one exact Jacobi preconditioner, passed explicitly to the later contexts of the tuner."""
    import numpy as np
    import torch

    import synth
    import paper_2011_06842_amd as fw

    B = args.batch
    A = min(4, B)
    stride = 2
    tune_warm, tune_steps = 3, max(3, args.batch_steps // 4)
    F = max(args.batch_warmup + args.batch_steps, tune_warm + tune_steps)
    need = F + stride * ((B + A - 1) // A)
    base = synth.config_elt_mcao(precision="fp32")
    t0 = time.perf_counter()
    specs_a, seqs = [], []
    for a in range(A):
        sp = base.copy()
        seqs.append(synth.make_sequence(sp, need, seed=SEED + 1 + a).astype(np.float32))
        specs_a.append(sp)
    spec = specs_a[0]
    specs = [spec] * B
    S1 = seqs[0].shape[1]
    frames = torch.empty((F, B * S1), dtype=torch.float32)
    for i in range(B):
        o = stride * (i // A)
        frames[:, i * S1:(i + 1) * S1] = torch.from_numpy(seqs[i % A][o:o + F])
    frames = frames.to(dev)
    t_gen = time.perf_counter() - t0
    log(f"batched leg: {B} instances, slopes generated in {t_gen:.1f} s")
    it, m = spec.max_iter, spec.recycle_k
    mp = 1

    def timed(ctx, warm, steps):
        c = torch.empty(ctx.N, dtype=torch.float32, device=dev)
        for t in range(warm):
            ctx.fewha_solve_aug(frames[t], c)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        w0 = time.perf_counter()
        ev[0].record()
        for k in range(steps):
            ctx.fewha_solve_aug(frames[warm + k], c)
            ev[k + 1].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        return wall, np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])

    # tuner: elements per vector workgroup (fixes the reduction order of every instance)
    t0 = time.perf_counter()
    tune = {}
    jinv = None
    for be in args.block_elems:
        sp = spec.copy()
        sp.block_elems = be
        ctx = fw.FewhaContext([sp] * B, device=dev, precond_inv=jinv)
        if jinv is None:
            j = ctx.fewha_get_vector(1).double().cpu().numpy()
            n1 = ctx.coeff_offsets[1]
            jinv = [j[:n1]] * B
        wall, fm = timed(ctx, tune_warm, tune_steps)
        tune[be] = float(np.median(fm))
        log(f"batched leg: block_elems {be}: frame {tune[be]:.3f} ms")
        del ctx
        torch.cuda.empty_cache()
    best = min(tune, key=tune.get)
    t_setup = time.perf_counter() - t0
    sp = spec.copy()
    sp.block_elems = best
    ctx = fw.FewhaContext([sp] * B, device=dev, precond_inv=jinv)
    wall, fm = timed(ctx, args.batch_warmup, args.batch_steps)
    log(f"batched leg: timed {args.batch_steps} frames, p50 {np.median(fm):.3f} ms")
    N, S = ctx.N, ctx.S
    V = B * sum((w.n_sub + 1) ** 2 for w in spec.wfs)

    # per-kernel profile of further frames (synchronous per launch, outside the timed region)
    ctx.fewha_profile(True)
    P = 3
    for t in range(P):
        ctx.fewha_solve_aug(frames[t])
    prof = ctx.fewha_profile_read()
    ctx.fewha_profile(False)
    steps = ctx.fewha_wavelet_steps()
    e = 4
    kern = {}
    for name, (ms, nl) in prof.items():
        if not nl:
            continue
        if name in OP_KERNELS:
            if name.endswith("_step"):
                b = sum(op_kernel_bytes(name, k, spec, steps, N, S, V, e) for k in range(len(steps)))
                b *= (nl / P) / len(steps)
            else:
                b = op_kernel_bytes(name, None, spec, steps, N, S, V, e) * (B if "coarse" in name else 1)
                b *= nl / P
        else:
            b = frame_kernel_bytes(name, N, S, V, e, m, it, mp)
        ms_f = ms / P
        kern[name] = {"ms_per_frame": round(ms_f, 4), "launches_per_frame": nl / P,
                      "GB_s": round(b / (ms_f * 1e-3) / 1e9, 1) if b else None}
        # vector-instruction issue rate: counted instructions per launch (committed counter
        # summary) over the duration measured here
        vi = pmc_value(name, "batched", "valu_insts_per_launch")
        if vi:
            rate = vi * (nl / P) / (ms_f * 1e-3)
            kern[name]["valu_Ginst_s"] = round(rate / 1e9, 1)
            kern[name]["valu_frac"] = round(rate / VALU_PEAK_INST_S, 4)
    dom = max((k for k in kern if kern[k]["GB_s"]), key=lambda k: kern[k]["ms_per_frame"])
    ach = kern[dom]["GB_s"]
    # the dominant operator kernel against the roofline that bounds it (HBM or vector issue)
    opk = max((k for k in kern if k in OP_KERNELS), key=lambda k: kern[k]["ms_per_frame"])
    ko = kern[opk]
    hbm_frac = ko["GB_s"] / HBM_PEAK_GBS if ko["GB_s"] else 0.0
    if ko.get("valu_frac") is not None and ko["valu_frac"] > hbm_frac:
        op_roof = {"bound": "valu", "kernel": opk, "achieved": ko["valu_Ginst_s"],
                   "peak": round(VALU_PEAK_INST_S / 1e9, 1), "unit": "G wave-instructions/s",
                   "frac": ko["valu_frac"], "hbm_frac": round(hbm_frac, 4)}
    else:
        op_roof = {"bound": "hbm", "kernel": opk, "achieved": ko["GB_s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                   "frac": round(hbm_frac, 4), "valu_frac": ko.get("valu_frac")}
    return {
        "workload": f"elt_mcao_fp32_x{B}_instances",
        "instances": B,
        "applies_per_s": round(B * it * args.batch_steps / wall, 1),
        "frame_ms_p50": round(float(np.percentile(fm, 50)), 4),
        "frame_ms_p99": round(float(np.percentile(fm, 99)), 4),
        "instance_frames_per_s": round(B * args.batch_steps / wall, 1),
        "steps": args.batch_steps, "warmup": args.batch_warmup,
        "block_elems": best, "tuner_frame_ms": {str(k): round(v, 4) for k, v in tune.items()},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": pmc_traffic(dom, "batched"),
                     "share_of_frame": round(kern[dom]["ms_per_frame"] / float(np.median(fm)), 3)},
        "operator_roofline": op_roof,
        "kernels": dict(sorted(kern.items(), key=lambda kv: -kv[1]["ms_per_frame"])),
        "input": f"{A} seeded atmospheres, instance i reads atmosphere i mod {A} from frame {stride} (i div {A})",
        "input_generation_s": round(t_gen, 1), "setup_and_tuning_s": round(t_setup, 1),
    }


def _ragged_instance(args):
    """One seeded random instance and its slope sequence (runs in a worker process)."""
    seed, frames = args
    import numpy as np
    import synth
    rng = np.random.default_rng(seed)
    sp = synth.config_random_instance(rng, precision="fp32")
    seq = synth.make_sequence(sp, frames, seed=seed + 1).astype(np.float32)
    return sp, seq


def run_ragged(args, dev):
    """Ragged batch: independent random instances (telescope 8-39 m, 20-84 subapertures, 3-9
    layers, 1-6 NGS/LGS, grids up to 256^2), FP32 operator, every instance stopping at its own
    first ||r|| <= 1e-4 ||b|| (cap 200) on the device; the frame is one graph replay."""
    import numpy as np
    import torch
    from concurrent.futures import ProcessPoolExecutor

    import paper_2011_06842_amd as fw

    B = args.ragged
    F = args.ragged_warmup + args.ragged_steps
    t0 = time.perf_counter()
    workers = max(1, min(16, os.cpu_count() or 1, B))
    with ProcessPoolExecutor(max_workers=workers) as ex:
        pairs = list(ex.map(_ragged_instance, [(SEED + 1000 + 7 * i, F) for i in range(B)]))
    specs = [p[0] for p in pairs]
    t_gen = time.perf_counter() - t0
    log(f"ragged leg: {B} instances, slopes generated in {t_gen:.1f} s ({workers} processes)")
    frames = torch.from_numpy(np.concatenate([p[1] for p in pairs], axis=1)).to(dev)
    t0 = time.perf_counter()
    ctx = fw.FewhaContext(specs, device=dev)
    t_setup = time.perf_counter() - t0
    c = torch.empty(ctx.N, dtype=torch.float32, device=dev)
    info = ctx.new_info()
    for t in range(args.ragged_warmup):
        ctx.fewha_solve_aug(frames[t], c, info)
    torch.cuda.synchronize()
    ms, iters, firsts, unmet = [], [], [], 0
    w0 = time.perf_counter()
    for k in range(args.ragged_steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.fewha_solve_aug(frames[args.ragged_warmup + k], c, info)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
        inf = fw.decode_info(info)
        iters.append(max(x["iters"] for x in inf))
        firsts += [x["iters"] for x in inf]
        unmet += sum(1 for x in inf if x["flags"] & 2)
    wall = time.perf_counter() - w0
    log(f"ragged leg: {args.ragged_steps} frames, p50 {np.median(ms):.2f} ms, longest instance "
        f"{np.mean(iters):.1f} iterations, mean {np.mean(firsts):.1f}")
    sizes = [synth_n(sp) for sp in specs]
    return {
        "workload": f"ragged_random_fp32_x{B}_tol1e-4",
        "instances": B, "coefficients": int(ctx.N), "coefficients_min_max": [min(sizes), max(sizes)],
        "applies_per_s": round(sum(firsts) / wall, 1),
        "frame_ms_p50": round(float(np.percentile(ms, 50)), 3),
        "frame_ms_p99": round(float(np.percentile(ms, 99)), 3),
        "longest_instance_iterations_mean": round(float(np.mean(iters)), 2),
        "iterations_enqueued_per_frame": int(specs[0].max_iter),
        "instance_iterations_to_tol_mean": round(float(np.mean(firsts)), 2),
        "instance_iterations_to_tol_max": int(max(firsts)),
        "tolerance_unmet_instance_frames": unmet,
        "steps": args.ragged_steps, "warmup": args.ragged_warmup,
        "input_generation_s": round(t_gen, 1), "setup_s": round(t_setup, 1),
        "note": "each instance stops at its first crossing (its kernels return at once afterwards); "
                "applies/s counts the applies instances performed",
    }


UNET_CONVS = [(32, 32, 0), (32, 32, 0), (32, 64, 1), (64, 64, 1), (64, 128, 2), (128, 128, 2), (128, 256, 3),
              (256, 256, 3), (384, 128, 2), (128, 128, 2), (192, 64, 1), (64, 64, 1), (96, 32, 0), (32, 32, 0)]
BF16_PEAK_TFS = 2500.0


def unet_forward_flops(groups):
    """Matrix-core flops the forward pass executes (padded input channels included)."""
    f = 0
    for n, size in groups:
        for cin, cout, lev in UNET_CONVS:
            f += 2 * n * (size >> lev) ** 2 * 9 * cin * cout
    return f


def run_unet(args, dev):
    """U-Net on one ELT frame (a 256^2 ground layer and eight 128^2 layers): forward and one
    training step (forward, backward, Adam), timed with HIP events on the context's stream."""
    import numpy as np
    import torch

    import paper_2011_06842_amd as fw
    from paper_2011_06842_amd import warmstart as W

    groups = [(1, 256), (8, 128)]
    net = fw.UNetContext(groups, device=dev)
    rng = np.random.default_rng(SEED)
    # He-normal weights plus symmetric noise on every parameter (nonzero biases and head, so
    # every layer carries gradient, with a finite loss)
    noise = torch.from_numpy((0.02 * rng.standard_normal(net.n_params)).astype(np.float32)).to(dev)
    net.set_params(W.init_params(net.n_params, None, SEED, dev) + noise)
    x = torch.from_numpy(rng.standard_normal(4 * net.nodes).astype(np.float32)).to(dev)
    t = torch.from_numpy(rng.standard_normal(net.nodes).astype(np.float32)).to(dev)
    out = torch.empty(net.nodes, dtype=torch.float32, device=dev)
    for _ in range(3):
        net.forward(x, out)
    torch.cuda.synchronize()
    R = args.unet_reps
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(R):
        net.forward(x, out)
    e1.record()
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / R
    loss0 = float(net.backward(x, t).cpu()[0])
    net.adam_step()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(R):
        net.backward(x, t)
        net.adam_step()
    e1.record()
    torch.cuda.synchronize()
    train_ms = e0.elapsed_time(e1) / R
    ff = unet_forward_flops(groups)
    ach = ff / (fwd_ms * 1e-3) / 1e12
    log(f"U-Net: forward {fwd_ms:.3f} ms ({ach:.1f} TFLOP/s), training step {train_ms:.3f} ms")
    return {
        "workload": "unet_4level_32-256ch_elt_frame (1x256^2 + 8x128^2 images)",
        "params": net.n_params, "forward_ms": round(fwd_ms, 4), "train_step_ms": round(train_ms, 4),
        "forward_gflop": round(ff / 1e9, 2), "train_step_gflop": round(3 * ff / 1e9, 2),
        "roofline": {"bound": "mfma", "kernel": "forward (all layers)", "achieved": round(ach, 2),
                     "peak": BF16_PEAK_TFS, "unit": "TFLOP/s", "frac": round(ach / BF16_PEAK_TFS, 4),
                     "traffic": None},
        "train_tflops": round(3 * ff / (train_ms * 1e-3) / 1e12, 2),
        "first_step_loss": round(loss0, 6),
    }


def _elt_sequence(arg):
    """(calibrated ELT spec, FP32 slope sequence) of one seed (process-pool worker)."""
    import numpy as np
    import synth
    seed, frames = arg
    sp = synth.config_elt_mcao(seed=seed)
    return sp, synth.make_sequence(sp, frames, seed=seed + 7).astype(np.float32)


def run_warmstart(args, dev):
    """Plain, learned-warm-start and batched augmented PCG on the ELT system at equal final
    residual (every frame iterated to ||r|| <= 1e-3 ||b||, cap 200).  The network is trained
    here on converged solves (256 iterations) of seeded training sequences with their own
    winds, the epoch kept is the one with the lowest loss on a validation sequence, and all
    three forms run on a held-out evaluation sequence (the batch adds further sequences)."""
    import numpy as np
    import torch
    from concurrent.futures import ProcessPoolExecutor

    import paper_2011_06842_amd as fw
    from paper_2011_06842_amd import warmstart as W

    tol, cap, F = 1e-3, 200, args.ws_frames
    nt, B = args.ws_train, args.ws_batch
    t0 = time.perf_counter()
    seeds = [SEED + 300 + 11 * i for i in range(nt + 1 + B)]   # training, validation, evaluation + batch
    with ProcessPoolExecutor(max_workers=max(1, min(16, os.cpu_count() or 1, len(seeds)))) as ex:
        seqs = list(ex.map(_elt_sequence, [(sd, F) for sd in seeds]))
    t_gen = time.perf_counter() - t0
    log(f"warm start: {len(seqs)} ELT sequences of {F} frames generated in {t_gen:.1f} s")
    base = seqs[0][0]
    spec = base.copy(rel_tol=tol, max_iter=cap)
    truth = base.copy(rel_tol=1e-6, max_iter=256)
    t0 = time.perf_counter()
    xs, ys = [], []
    for _, sq in seqs[:nt + 1]:
        x, y = W.collect(spec, fw.FewhaContext(spec, device=dev), fw.FewhaContext(truth, device=dev), sq, dev)
        xs.append(x)
        ys.append(y)
    x, y = np.concatenate(xs[:nt]), np.concatenate(ys[:nt])
    scales = W.scales_of(x, y)
    xn, yn = W.normalise(x, y, scales)
    xv, yv = W.normalise(xs[nt], ys[nt], scales)
    del xs, ys, x, y
    t_collect = time.perf_counter() - t0

    def val_loss(params):
        net = W.inference_net(spec, params, dev)
        out = torch.empty(net.nodes, dtype=torch.float32, device=dev)
        err = 0.0
        for i in range(xv.shape[0]):
            net.forward(torch.from_numpy(W._group_major(spec, xv[i:i + 1], 4)).to(dev), out)
            err += float(np.mean((out.cpu().numpy() - W._group_major(spec, yv[i:i + 1], 1)) ** 2))
        return err / xv.shape[0]

    t0 = time.perf_counter()
    params, hist, best = None, [], (float("inf"), None, -1)
    for ep in range(args.ws_epochs):
        params, losses = W.train(spec, xn, yn, batch=2, epochs=1, lr=1e-3, seed=ep, params=params, device=dev)
        vl = val_loss(params)
        hist.append((round(float(np.mean(losses)), 4), round(vl, 4)))
        if vl < best[0]:
            best = (vl, params.clone(), ep)
    t_train = time.perf_counter() - t0
    log(f"warm start: {xn.shape[0]} samples, {args.ws_epochs} epochs in {t_train:.1f} s, "
        f"best validation loss {best[0]:.3f} (epoch {best[2]})")
    net = W.inference_net(spec, best[1], dev)

    evals = seqs[nt + 1:]
    res = {}
    for name in ("plain", "warm"):
        ctx = fw.FewhaContext(spec, device=dev)
        info = ctx.new_info()
        ms, its, acc = [], [], 0
        for t in range(F):
            s = torch.from_numpy(evals[0][1][t]).to(dev)
            torch.cuda.synchronize()
            w0 = time.perf_counter()
            if name == "plain":
                ctx.fewha_solve_aug(s, info=info)
            else:
                ctx.fewha_solve_aug_ws(net, scales, s, info=info)
            torch.cuda.synchronize()
            dt = 1000 * (time.perf_counter() - w0)
            g = fw.decode_info(info)
            if g["flags"] & 2:
                raise RuntimeError(f"{name} frame {t}: tolerance not met within {cap} iterations")
            if t >= 2:
                ms.append(dt)
                its.append(g["iters"])
                acc += 0 if g["flags"] & 4 else 1
        res[name] = {"iterations_to_tol_mean": round(float(np.mean(its)), 2),
                     "frame_ms_p50": round(float(np.percentile(ms, 50)), 3),
                     "frame_ms_p99": round(float(np.percentile(ms, 99)), 3)}
        if name == "warm":
            res[name]["correction_accepted"] = f"{acc}/{len(its)}"
    # batched: the evaluation sequence and B - 1 further ones in one lock-step batch
    bspecs = [sp.copy(rel_tol=tol, max_iter=cap) for sp, _ in evals]
    bctx = fw.FewhaContext(bspecs, device=dev)
    frames = torch.from_numpy(np.concatenate([sq for _, sq in evals], axis=1)).to(dev)
    c = torch.empty(bctx.N, dtype=torch.float32, device=dev)
    info = bctx.new_info()
    ms, its = [], []
    for t in range(F):
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        bctx.fewha_solve_aug(frames[t], c, info)
        torch.cuda.synchronize()
        dt = 1000 * (time.perf_counter() - w0)
        if t >= 2:
            ms.append(dt)
            its.append(float(np.mean([x["iters"] for x in fw.decode_info(info)])))
    res["batched"] = {"instances": len(evals), "iterations_to_tol_mean": round(float(np.mean(its)), 2),
                      "batch_frame_ms_p50": round(float(np.percentile(ms, 50)), 3),
                      "batch_frame_ms_p99": round(float(np.percentile(ms, 99)), 3),
                      "per_instance_ms_p50": round(float(np.percentile(ms, 50)) / len(evals), 3)}
    log(f"warm start: iterations plain {res['plain']['iterations_to_tol_mean']}, warm "
        f"{res['warm']['iterations_to_tol_mean']}; p99 plain {res['plain']['frame_ms_p99']} ms, warm "
        f"{res['warm']['frame_ms_p99']} ms, batch of {len(evals)} {res['batched']['batch_frame_ms_p99']} ms")
    return {"workload": f"elt_mcao_fp32 tolerance {tol:g} (cap {cap}); train {nt} x {F - 1} transitions, "
                        f"validate 1, evaluate 1 sequence (frames 2..{F - 1} timed)",
            "truth": "256 iterations of augmented PCG (rel_tol 1e-6 cap) per training frame",
            "loss_train_validation_per_epoch": hist, "epoch_kept": best[2],
            "generate_s": round(t_gen, 1), "collect_s": round(t_collect, 1), "train_s": round(t_train, 1),
            **res, "timing": "host wall clock per frame (each synchronised)"}


def synth_n(spec):
    return int(sum(l.n * l.n for l in spec.layers))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-frames", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-frames", type=int, default=20)
    ap.add_argument("--kernel-reps", type=int, default=100)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB")
    ap.add_argument("--batch", type=int, default=64, help="instances of the batched leg (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--batch-warmup", type=int, default=5)
    ap.add_argument("--block-elems", type=lambda v: [int(x) for x in v.split(",")], default=[384, 2048, 8192])
    ap.add_argument("--ragged", type=int, default=64, help="instances of the ragged tolerance leg (0: skip)")
    ap.add_argument("--ragged-steps", type=int, default=8)
    ap.add_argument("--ragged-warmup", type=int, default=2)
    ap.add_argument("--unet", type=int, default=1, help="U-Net timing leg (0: skip)")
    ap.add_argument("--unet-reps", type=int, default=10)
    ap.add_argument("--warmstart", type=int, default=1, help="warm-start comparison leg (0: skip)")
    ap.add_argument("--ws-frames", type=int, default=40, help="frames per warm-start sequence")
    ap.add_argument("--ws-train", type=int, default=6, help="training sequences of the warm start")
    ap.add_argument("--ws-epochs", type=int, default=12)
    ap.add_argument("--ws-batch", type=int, default=8, help="instances of the batched form")
    args = ap.parse_args(argv)
    if args.copy_probe:
        return copy_probe(args.copy_probe)
    if args.gpus != 1:
        print("bench.py measures one MI355X: the frame solve runs on a single GPU and the library has no "
              "multi-GPU path (--gpus must be 1)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import synth
    import paper_2011_06842_amd as fw

    dev = "cuda:0"
    spec = synth.config_elt_mcao(precision="fp32")
    F = args.warmup + args.steps
    t_gen = time.perf_counter()
    seq64 = synth.make_sequence(spec, F, seed=SEED)
    t_gen = time.perf_counter() - t_gen
    seq32 = seq64.astype(np.float32)
    log(f"single instance: {F} frames generated in {t_gen:.1f} s")
    slopes = torch.from_numpy(seq32).to(dev)                  # resident in HBM before timing
    ctx = fw.FewhaContext(spec, device=dev)
    N, S = ctx.N, ctx.S
    V = sum((w.n_sub + 1) ** 2 for w in spec.wfs)
    c = torch.empty(N, dtype=torch.float32, device=dev)
    info = ctx.new_info()

    for t in range(args.warmup):
        ctx.fewha_solve_aug(slopes[t], c, info)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(args.steps):
        ctx.fewha_solve_aug(slopes[args.warmup + k], c, info)
        ev[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    frame_ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)])
    last_info = fw.decode_info(info)
    it = spec.max_iter
    applies_per_s = it * args.steps / wall

    # operator alone (pure M applications, same stream)
    x = torch.randn(N, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    for _ in range(10):
        ctx.fewha_apply_A(x, y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    R = 200
    e0.record()
    for _ in range(R):
        ctx.fewha_apply_A(x, y)
    e1.record()
    torch.cuda.synchronize()
    op_ms = e0.elapsed_time(e1) / R
    log(f"single instance: frame p50 {np.median(frame_ms):.4f} ms, apply {1000 * op_ms:.1f} us")

    # per-kernel durations from HIP events around every launch of a fresh run of the same
    # frames (profiling synchronises per call, so it runs outside the timed region)
    pctx = fw.FewhaContext(spec, device=dev)
    pc = torch.empty_like(c)
    for t in range(args.warmup):
        pctx.fewha_solve_aug(slopes[t], pc)
    pctx.fewha_profile(True)
    P = min(args.profile_frames, args.steps)
    for t in range(P):
        pctx.fewha_solve_aug(slopes[args.warmup + t], pc)
    prof = pctx.fewha_profile_read()
    pctx.fewha_profile(False)
    kernels = {name: {"ms_per_frame": ms / P, "launches_per_frame": nl / P, "avg_launch_us": 1000 * ms / nl}
               for name, (ms, nl) in prof.items() if nl}

    # operator kernels one at a time: R launches with the frame's own arguments, captured in
    # one graph and replayed between two HIP events on the context's stream
    steps = ctx.fewha_wavelet_steps()
    e = 4
    opk = {}
    for kid, name in enumerate(OP_KERNELS):
        for st in (range(len(steps)) if name.endswith("_step") else [None]):
            us = 1000 * ctx.fewha_time_kernel(kid, st or 0, args.kernel_reps)
            b = op_kernel_bytes(name, st, spec, steps, N, S, V, e)
            key = name if st is None else f"{name}[{steps[st][0]}x{steps[st][0]} x{steps[st][1]}]"
            opk[key] = {"kernel": name, "avg_us": round(us, 3), "bytes": b, "GB_s": round(b / us * 1e-3, 1)}
    # dominant operator kernel: largest time per frame (timed duration x launches per frame,
    # a tiled kernel's launches spread evenly over its levels)
    for v in opk.values():
        nst = len(steps) if v["kernel"].endswith("_step") else 1
        v["us_per_frame"] = round(v["avg_us"] * kernels.get(v["kernel"], {}).get("launches_per_frame", 0) / nst, 2)
    per_kernel = {}
    for v in opk.values():
        per_kernel[v["kernel"]] = per_kernel.get(v["kernel"], 0.0) + v["us_per_frame"]
    dom = max(per_kernel, key=per_kernel.get)
    dk = max((k for k, v in opk.items() if v["kernel"] == dom), key=lambda k: opk[k]["avg_us"])
    d = opk[dk]
    achieved = d["bytes"] / (d["avg_us"] * 1e-6) / 1e9
    roofline = {"bound": "hbm", "kernel": dk, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": pmc_traffic(dk, "single"),
                "bytes_per_launch": d["bytes"], "avg_launch_us": d["avg_us"],
                "share_of_frame": round(per_kernel[dom] * 1e-3 / float(np.median(frame_ms)), 3)}

    out = {
        "metric": METRIC,
        "value": round(applies_per_s, 1),
        "unit": "applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000 * wall / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "elt_mcao_fp32_single_instance", "telescope_m": spec.D,
                   "lgs": len(spec.wfs), "n_sub": spec.wfs[0].n_sub,
                   "layers": [l.n for l in spec.layers], "wavelet_levels": spec.layers[0].levels,
                   "pcg_iters": it, "recycle_k": spec.recycle_k, "recycle_mode": spec.recycle_mode,
                   "N": N, "S": S, "reductions": "f64", "frames_generated": F,
                   "input": "seeded frozen-flow von Karman screens, SNR-10 slope noise"},
        "frame_ms_p50": round(float(np.percentile(frame_ms, 50)), 4),
        "frame_ms_p99": round(float(np.percentile(frame_ms, 99)), 4),
        "frames_per_s": round(args.steps / wall, 1),
        "operator_apply_ms": round(op_ms, 4),
        "operator_applies_per_s_alone": round(1000.0 / op_ms, 1),
        "last_frame_rel_res": last_info["rel_res"],
        "roofline": roofline,
        "kernels": {k: {kk: round(vv, 4) for kk, vv in v.items()}
                    for k, v in sorted(kernels.items(), key=lambda kv: -kv[1]["ms_per_frame"])},
        "operator_kernels": opk,
        "paper_context": "CPU aug. FEWHA MCAO 1.9 ms/frame on 12 Haswell cores (different system size)",
    }

    log("single instance: kernel profile and per-kernel timing done")
    if not args.no_cpu_baseline:
        from threadpoolctl import threadpool_limits
        from oracle import AugmentedReconstructor, OracleSystem
        nf = max(1, min(args.cpu_frames, F))
        with threadpool_limits(limits=1):
            sysm = OracleSystem(spec)
            ref = AugmentedReconstructor(sysm)
            t0 = time.perf_counter()
            refs = [ref.solve(seq32[t].astype(np.float64))[0] for t in range(nf)]
            cpu_wall = time.perf_counter() - t0
        # the GPU on the same frames from a fresh context, against the FP64 oracle
        vctx = fw.FewhaContext(spec, device=dev)
        errs = []
        for t in range(nf):
            g = vctx.fewha_solve_aug(slopes[t]).double().cpu().numpy()
            errs.append(float(np.linalg.norm(g - refs[t]) / np.linalg.norm(refs[t])))
        out["cpu_baseline"] = {"value": round(it * nf / cpu_wall, 3), "unit": "applies/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"first {nf} frames of the same sequence (FP64 NumPy oracle, "
                                         f"{1000 * cpu_wall / nf:.1f} ms/frame incl. the first frame's extra apply)"}
        # free-running: both sides carry their own residual from frame 0 (FP32 rounding
        # differences accumulate slowly; the per-frame bound applies from an identical state)
        out["rel_err_vs_oracle_free_running"] = {"frames": nf, "max": max(errs), "last": errs[-1]}
    out["input_generation_s"] = round(t_gen, 2)
    if args.batch > 0:
        del ctx, pctx
        torch.cuda.empty_cache()
        out["batched"] = run_batch(args, dev)
        torch.cuda.empty_cache()
    if args.ragged > 0:
        out["ragged"] = run_ragged(args, dev)
        torch.cuda.empty_cache()
    if args.unet:
        out["unet"] = run_unet(args, dev)
        torch.cuda.empty_cache()
    if args.warmstart:
        out["warmstart"] = run_warmstart(args, dev)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
