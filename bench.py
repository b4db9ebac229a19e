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


COARSE_BLOCK = 32      # analysis levels whose block fits this side run in one workgroup's LDS
# operator kernels in the library's profiler numbering (see include/fewha.h)
OP_KERNELS = ["idwt", "data_term", "adj_gather", "dwt_tiles", "dwt_coarse"]
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_2011_06842_amd", "csrc")


def log(msg):
    """Progress of the legs on stderr (stdout carries the one JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def ana_segments(n, levels, kmax):
    """Tiled analysis levels of a layer: (group, first level, count), as the library plans them
    (groups of kmax block sizes above the coarse block, one launch each, finest first)."""
    out = []
    lc = 1
    while (n >> (lc - 1)) > COARSE_BLOCK:
        lc += 1
    for lev in range(1, min(levels, lc - 1) + 1):
        g = ((n >> (lev - 1)).bit_length() - 1 - (COARSE_BLOCK.bit_length() - 1) - 1) // kmax
        if out and out[-1][0] == g:
            out[-1][2] += 1
        else:
            out.append([g, lev, 1])
    return out, lc


def op_kernel_bytes(name, step, spec, steps, N, S, V, e):
    """Algorithmic HBM bytes of one launch of an operator kernel inside M x: every operand it
    must read or write once (x, the prior and the slope weights included), intermediates
    between kernels counted once at each side, nothing counted twice within a kernel."""
    kmax = 2 if spec.precision == "fp64" else 3
    if name == "idwt":            # coefficients in, images out
        return 2 * N * e
    if name == "data_term":       # layer images in, slope weights in, sensor nodes out
        return (N + S + V) * e
    if name == "adj_gather":      # sensor nodes in, layer images out
        return (V + N) * e
    groups = sorted({sg[0] for l in spec.layers for sg in ana_segments(l.n, l.levels, kmax)[0]}, reverse=True)
    total = 0
    for l in spec.layers:
        segs, lc = ana_segments(l.n, l.levels, kmax)
        if name == "dwt_coarse":  # LL block (or image) in; coefficients, prior and x of the block
            total += 4 * (l.n >> (lc - 1)) ** 2 if l.levels >= lc else 0
            continue
        for g, l1, k in segs:     # input window of the launch; 3 bands per level (+ prior, x)
            if g != groups[step]:
                continue
            nb_in = l.n >> (l1 - 1)
            total += nb_in * nb_in
            for j in range(k):
                m = nb_in >> (j + 1)
                total += 3 * m * m * 3
            m = nb_in >> k
            total += m * m * (3 if l1 + k - 1 == l.levels else 1)
    return total * e


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
    summaries (profiles/*_pmc.md), or None."""
    return _profile_block_value("*_pmc.md", kernel, workload, key)


def _profile_block_value(pattern, kernel, workload, key):
    """Value `key` from the committed summaries matching `pattern` (blocks of "- key: value"
    lines starting at "- kernel:"), or None when none matches or the sources changed since."""
    import glob
    sha = source_sha256()
    for path in sorted(glob.glob(os.path.join(PROFILES, pattern))):
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


BATCH_ATMOSPHERES, BATCH_STRIDE = 4, 2


def batch_frames_needed(args):
    """Frames of each atmosphere the batched leg reads."""
    B = args.batch
    A = min(BATCH_ATMOSPHERES, B)
    F = max(args.batch_warmup + args.batch_steps, 3 + max(3, args.batch_steps // 4))
    return F + BATCH_STRIDE * ((B + A - 1) // A)


def run_batch(args, dev, atmos, t_gen):
    """Throughput form: B independent instances of the ELT geometry in one context (one frame
    advances all of them).  Instance i reads the slope stream of atmosphere i mod A (`atmos`: A
    (spec, sequence) pairs of seeded ELT atmospheres) at a time offset, so that every instance
    sees its own frames; all share the noise weights, hence one exact Jacobi preconditioner,
    passed explicitly to the later contexts of the tuner."""
    import numpy as np
    import torch

    import paper_2011_06842_amd as fw

    B = args.batch
    A = min(BATCH_ATMOSPHERES, B)
    stride = BATCH_STRIDE
    tune_warm, tune_steps = 3, max(3, args.batch_steps // 4)
    F = max(args.batch_warmup + args.batch_steps, tune_warm + tune_steps)
    seqs = [a[1] for a in atmos]
    spec = atmos[0][0]
    specs = [spec] * B
    S1 = seqs[0].shape[1]
    frames = torch.empty((F, B * S1), dtype=torch.float32)
    for i in range(B):
        o = stride * (i // A)
        frames[:, i * S1:(i + 1) * S1] = torch.from_numpy(seqs[i % A][o:o + F])
    frames = frames.to(dev)
    log(f"batched leg: {B} instances")
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
    tuned, tune_ms = choose_tiles(ctx, args.batch_tuning, 5)
    log(f"batched leg: autotuner chose {tuned}")
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
            if name == "dwt_tiles":
                b = B * sum(op_kernel_bytes(name, k, spec, steps, N, S, V, e) for k in range(len(steps)))
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
        "autotuner": {"chosen": tuned, "apply_ms_per_candidate": {k: round(v, 4) for k, v in tune_ms.items()}},
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


def ragged_inputs(ex, args):
    """Seeded random instances of the ragged leg and their slope sequences (process pool)."""
    F = args.ragged_warmup + args.ragged_steps
    return list(ex.map(_ragged_instance, [(SEED + 1000 + 7 * i, F) for i in range(args.ragged)]))


def run_ragged(args, dev, pairs, t_gen):
    """Ragged batch: independent random instances (telescope 8-39 m, 20-84 subapertures, 3-9
    layers, 1-6 NGS/LGS, grids up to 256^2), FP32 operator, every instance stopping at its own
    first ||r|| <= 1e-4 ||b|| (cap 200) on the device; the frame is one graph replay."""
    import numpy as np
    import torch

    import paper_2011_06842_amd as fw

    B = args.ragged
    specs = [p[0] for p in pairs]
    log(f"ragged leg: {B} instances")
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


def warmstart_inputs(ex, args):
    """ELT sequences of the warm-start leg: training, validation, evaluation and batch."""
    seeds = [SEED + 300 + 11 * i for i in range(args.ws_train + 1 + args.ws_batch)]
    return list(ex.map(_elt_sequence, [(sd, args.ws_frames) for sd in seeds]))


def run_warmstart(args, dev, seqs, t_gen):
    """Plain, learned-warm-start and batched augmented PCG on the ELT system at equal final
    residual (every frame iterated to ||r|| <= 1e-3 ||b||, cap 200).  The network is trained
    here on converged solves (256 iterations) of seeded training sequences with their own
    winds, the epoch kept is the one with the lowest loss on a validation sequence, and all
    three forms run on a held-out evaluation sequence (the batch adds further sequences)."""
    import numpy as np
    import torch

    import paper_2011_06842_amd as fw
    from paper_2011_06842_amd import warmstart as W

    tol, cap, F = 1e-3, 200, args.ws_frames
    nt, B = args.ws_train, args.ws_batch
    log(f"warm start: {len(seqs)} ELT sequences of {F} frames")
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


# ---------------------------------------------------------------- inputs and CPU baselines

def host_cpu_info():
    """Host CPU: model name, logical CPUs, and the CPUs this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return {"model": model, "nproc": os.cpu_count(), "affinity": avail}


def pool_size():
    """Worker processes for input generation and the all-core baseline (at most 16)."""
    return max(1, min(16, host_cpu_info()["affinity"]))


def make_config(name):
    import synth
    if name == "elt":
        return synth.config_elt_mcao(precision="fp32")
    if name == "full":
        return synth.config_elt_lgs_noise(precision="fp32")
    if name == "small":
        return synth.config_small()
    raise ValueError(name)


def _seq_chunk(arg):
    """(calibrated spec, frames start..start+n-1) of one configuration (pool worker; every frame
    depends on its index and the seed only, so chunks concatenate to the serial sequence)."""
    import numpy as np
    import synth
    name, seed, start, n = arg
    sp = make_config(name)
    seq = synth.make_sequence(sp, n, seed=seed, start=start)
    return sp, seq.astype(np.float32 if sp.precision == "fp32" else np.float64)


def gen_sequence(ex, name, seed, frames, chunk=25):
    import numpy as np
    parts = list(ex.map(_seq_chunk, [(name, seed, s, min(chunk, frames - s)) for s in range(0, frames, chunk)]))
    return parts[0][0], np.concatenate([p[1] for p in parts])


_BARRIER = None


def _set_barrier(b):
    global _BARRIER
    _BARRIER = b


def _oracle_run(arg):
    """The FP64 oracle on consecutive frames in one thread: (setup s, per-frame s, solutions).
    `perturb` > 0 multiplies every output of M (each operator application) by
    (1 + perturb * N(0, 1)) (seeded): the method's own sensitivity to one rounding of that
    relative size per operator output.  `sync` waits for the other workers of an all-core run
    after setup."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import AugmentedReconstructor, OracleSystem
    spec, seq, keep, perturb, sync = arg
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        rec = AugmentedReconstructor(OracleSystem(spec))
        setup = time.perf_counter() - t0
        rng = np.random.default_rng(SEED + 5)
        if perturb:
            exact = rec.apply_M
            rec.apply_M = lambda x: (lambda y: y * (1.0 + perturb * rng.standard_normal(y.size)))(exact(x))
        if sync:
            _BARRIER.wait(timeout=900)
        ts, sols = [], []
        for t in range(len(seq)):
            s = np.asarray(seq[t], dtype=np.float64)
            w0 = time.perf_counter()
            c, _ = rec.solve(s)
            ts.append(time.perf_counter() - w0)
            if keep:
                sols.append(c)
    return setup, ts, sols


def _oracle_loop_run(arg):
    """The FP64 closed-loop oracle of the full ELT loop on consecutive open-loop frames: the
    commands after every frame (the measured slopes are the open-loop ones minus the oracle's
    own DM slopes of a^(i-1), rounded to the slope precision)."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    import synth
    from oracle import AugmentedReconstructor, OracleSystem
    from oracle.closed_loop import ClosedLoopOracle, DmSpec
    spec, seq, n_pts, fit_iter, gain = arg
    with threadpool_limits(limits=1):
        ref = ClosedLoopOracle(AugmentedReconstructor(OracleSystem(spec)), [DmSpec(*d) for d in synth.elt_mcao_dms()],
                               gain=gain, closed=True, fit_dirs=synth.mcao_fit_directions(), n_pts=n_pts,
                               fit_iter=fit_iter)
        out, ts = [], []
        for t in range(len(seq)):
            s = (np.asarray(seq[t], dtype=np.float64) - ref.dm_slopes(ref.a_prev)).astype(seq.dtype).astype(np.float64)
            w0 = time.perf_counter()
            a, _ = ref.step(s)
            ts.append(time.perf_counter() - w0)
            out.append(a.copy())
    return out, ts


def frame_stats(ts_s, it):
    import numpy as np
    ms = 1000.0 * np.asarray(ts_s)
    return {"frame_ms_p50": round(float(np.percentile(ms, 50)), 3),
            "frame_ms_p99": round(float(np.percentile(ms, 99)), 3),
            "applies_per_s": round(it * len(ms) / float(ms.sum() * 1e-3), 3), "frames": int(len(ms))}


def cpu_baselines(spec, seq, n_single, n_all, workers):
    """Single-thread and all-core figures of the FP64 oracle on the first frames of `seq`:
    one process (one BLAS/NumPy thread) for the single-thread figure and its solutions, one
    more with every operator output perturbed at FP32 rounding size (2^-24) and, for an FP64
    configuration, one at FP64 rounding size (2^-52), then `workers` processes each
    solving the same frames concurrently after a common start (aggregate applies/s over the
    span from the common start to the last finish)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    ctx = mp.get_context("fork")
    it = spec.max_iter
    sizes = [24] + ([52] if spec.precision == "fp64" else [])
    with ProcessPoolExecutor(max_workers=1 + len(sizes), mp_context=ctx) as ex:
        f1 = ex.submit(_oracle_run, (spec, seq[:n_single], True, 0.0, False))
        fp = {e: ex.submit(_oracle_run, (spec, seq[:n_single], True, 2.0 ** -e, False)) for e in sizes}
        setup1, ts1, sols = f1.result()
        sols_p = {e: f.result()[2] for e, f in fp.items()}
    barrier = ctx.Barrier(workers)
    with ProcessPoolExecutor(max_workers=workers, mp_context=ctx, initializer=_set_barrier,
                             initargs=(barrier,)) as ex:
        res = list(ex.map(_oracle_run, [(spec, seq[:n_all], False, 0.0, True)] * workers))
    # every worker starts its frames when the last one has finished setup: the span is the
    # longest worker's loop
    span = max(sum(r[1]) for r in res)
    all_ts = [t for r in res for t in r[1]]
    single = frame_stats(ts1, it)
    allc = frame_stats(all_ts, it)
    allc["applies_per_s"] = round(it * len(all_ts) / span, 3)
    single["setup_s"] = round(setup1, 2)
    return single, allc, sols, sols_p


# ---------------------------------------------------------------- GPU legs

def choose_tiles(ctx, spec_tuning, reps):
    """The autotuner's tile shapes, or the fixed ones `spec_tuning` names ("synS_rowsR"; for
    profiled runs, whose tracing overhead distorts the tuner's timings)."""
    if spec_tuning == "auto":
        return ctx.fewha_autotune(reps=reps)
    syn, rows = spec_tuning.replace("syn", "").split("_rows")
    ctx.fewha_set_tuning(int(syn), int(rows))
    return {"syn_tile": int(syn), "gather_rows": int(rows)}, {}


def time_frames(ctx, slopes, t0, n, c, info):
    """Frames t0..t0+n-1 (each a graph replay), one HIP event after each on the context's stream:
    (wall s, per-frame ms)."""
    import numpy as np
    import torch
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(n + 1)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev[0].record()
    for k in range(n):
        ctx.fewha_solve_aug(slopes[t0 + k], c, info)
        ev[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    return wall, np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(n)])


def kernel_stats_value(kernel, workload, key):
    """Value `key` of `kernel` in `workload` from the committed kernel-trace summaries
    (profiles/*_kernel_stats.md, same block format as the counter summaries), or None."""
    return _profile_block_value("*_kernel_stats.md", kernel, workload, key)


def run_small(args, dev, spec, seq):
    """The 8 m FP64 system (3 NGS, 40x40 subapertures, 3 layers on 64^2 grids, 4 levels, 10
    PCG iterations, k = 5): frame latency over the whole sequence and applies/s."""
    import numpy as np
    import torch
    import paper_2011_06842_amd as fw
    slopes = torch.from_numpy(seq).to(dev)
    ctx = fw.FewhaContext(spec, device=dev)
    c = torch.empty(ctx.N, dtype=torch.float64, device=dev)
    info = ctx.new_info()
    W = min(args.warmup, len(seq) // 10)
    time_frames(ctx, slopes, 0, W, c, info)
    wall, ms = time_frames(ctx, slopes, W, len(seq) - W, c, info)
    it = spec.max_iter
    return {"workload": "small_8m_3ngs_fp64_single_instance", "N": ctx.N, "S": ctx.S, "pcg_iters": it,
            "recycle_k": spec.recycle_k, "frames": len(seq) - W, "warmup": W,
            "frame_ms_p50": round(float(np.percentile(ms, 50)), 4),
            "frame_ms_p99": round(float(np.percentile(ms, 99)), 4),
            "applies_per_s": round(it * (len(seq) - W) / wall, 1)}


def run_full_loop(args, dev, spec, seq):
    """The full ELT loop (6 LGS + 3 low-order NGS, FP32 operator with FP64 reductions, the LGS
    noise model: elongated spots, LGS tip/tilt jitter filtered out of C_eta^-1): Alg. 3 in
    closed loop with the three MCAO DMs, least-squares fitting by 4 CG iterations over the
    5 x 5 science directions, gain 0.4, over the whole sequence.  The measured slopes of frame i
    are the open-loop ones minus the DM slopes of a^(i-1) (the telescope's part, computed
    outside the timed region); each loop step is bracketed by HIP events on the stream."""
    import numpy as np
    import torch
    import synth
    import paper_2011_06842_amd as fw
    ctx = fw.FewhaContext(spec, device=dev)
    loop = fw.LoopContext(ctx, synth.elt_mcao_dms(), gain=args.loop_gain, closed=True, fit_iter=args.loop_fit_iter,
                          dirs=synth.mcao_fit_directions(), n_pts=args.loop_pts, pupil_d=spec.D,
                          obstruction=spec.obstruction)
    slopes = torch.from_numpy(seq).to(dev)
    a_next = torch.zeros(loop.n_act, dtype=torch.float32, device=dev)
    info = ctx.new_info()
    n = len(seq)
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(n)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(n)]
    early = []
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for t in range(n):
        s = slopes[t] - loop.piece(fw.LOOP_DM_SLOPES, loop.get_commands(0))
        ev0[t].record()
        loop.step(s, a_next, info)
        ev1[t].record()
        if t < args.loop_check_frames:
            early.append(a_next.double().cpu().numpy())
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = np.array([ev0[t].elapsed_time(ev1[t]) for t in range(n)])
    W = min(args.warmup, n // 10)
    m = ms[W:]
    budget = 2.0
    return {"workload": "elt_full_loop_fp32 (6 LGS 84x84 with elongated spots and filtered tip/tilt + NGS 2x2, "
                        "1x1, 1x1; 3 DMs; CG fitting over 5x5 directions)", "N": ctx.N, "S": ctx.S, "actuators": loop.n_act,
            "frames": int(len(m)), "warmup": W, "fit_iter": args.loop_fit_iter, "fit_pupil_points": args.loop_pts,
            "loop_step_ms_p50": round(float(np.percentile(m, 50)), 4),
            "loop_step_ms_p99": round(float(np.percentile(m, 99)), 4),
            "loop_step_ms_max": round(float(m.max()), 4),
            "budget_ms": budget, "frames_over_budget": int((m > budget).sum()),
            "wall_s": round(wall, 2), "note": "HIP events around each loop step; the DM slopes that form the "
                                                "measured slopes run between steps"}, early


def run_single(args, dev, spec, seq):
    """ELT single instance: the timed frames (value), a longer latency pass, the event-timed
    kernel profile, the per-kernel timer and the per-frame algorithmic-bytes fraction."""
    import numpy as np
    import torch
    import paper_2011_06842_amd as fw
    slopes = torch.from_numpy(seq).to(dev)                  # resident in HBM before timing
    ctx = fw.FewhaContext(spec, device=dev)
    N, S = ctx.N, ctx.S
    V = sum((w.n_sub + 1) ** 2 for w in spec.wfs)
    c = torch.empty(N, dtype=torch.float32, device=dev)
    info = ctx.new_info()
    tuned, tune_ms = choose_tiles(ctx, args.tuning, args.kernel_reps)   # tile shapes (no result bit changes)
    log(f"single instance: autotuner chose {tuned} ({ {k: round(v * 1000, 2) for k, v in tune_ms.items()} } us per apply)")
    time_frames(ctx, slopes, 0, args.warmup, c, info)
    wall, frame_ms = time_frames(ctx, slopes, args.warmup, args.steps, c, info)
    last_info = fw.decode_info(info)
    it = spec.max_iter
    # latency pass: the rest of the sequence
    L0 = args.warmup + args.steps
    lat_wall, lat_ms = time_frames(ctx, slopes, L0, len(seq) - L0, c, info) if len(seq) > L0 else (wall, frame_ms)
    if len(seq) <= L0:
        lat_ms = frame_ms
    lat_all = np.concatenate([frame_ms, lat_ms]) if len(seq) > L0 else frame_ms

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
    log(f"single instance: frame p50 {np.median(lat_all):.4f} ms over {len(lat_all)} frames, apply {1000 * op_ms:.1f} us")

    # per-kernel durations from HIP events around every launch of a fresh run of the same
    # frames (profiling synchronises per call, so it runs outside the timed region)
    pctx = fw.FewhaContext(spec, device=dev)
    pctx.fewha_set_tuning(tuned["syn_tile"], tuned["gather_rows"])
    pc = torch.empty_like(c)
    for t in range(args.warmup):
        pctx.fewha_solve_aug(slopes[t], pc)
    pctx.fewha_profile(True)
    P = min(args.profile_frames, args.steps)
    for t in range(P):
        pctx.fewha_solve_aug(slopes[args.warmup + t], pc)
    prof = pctx.fewha_profile_read()
    pctx.fewha_profile(False)
    del pctx
    kernels = {name: {"ms_per_frame": ms / P, "launches_per_frame": nl / P, "avg_launch_us": 1000 * ms / nl}
               for name, (ms, nl) in prof.items() if nl}

    # operator kernels one at a time: R launches with the frame's own arguments, captured in
    # one graph and replayed between two HIP events on the context's stream
    steps = ctx.fewha_wavelet_steps()
    e = 4
    m, mp = spec.recycle_k, 1
    opk = {}
    for kid, name in enumerate(OP_KERNELS):
        for st in (range(len(steps)) if name == "dwt_tiles" else [None]):
            us = 1000 * ctx.fewha_time_kernel(kid, st or 0, args.kernel_reps)
            b = op_kernel_bytes(name, st, spec, steps, N, S, V, e)
            key = name if st is None else f"{name}[{steps[st][0]}x{steps[st][0]} x{steps[st][1]}]"
            opk[key] = {"kernel": name, "avg_us": round(us, 3), "bytes": b, "GB_s": round(b / us * 1e-3, 1)}
    # per kernel function: launches per frame (event profile), the timer's duration of each
    # launch shape, and the algorithmic bytes of the frame's launches (a tiled kernel's launches
    # spread evenly over its levels)
    per_kernel = {}
    for v in opk.values():
        k = v["kernel"]
        nst = len(steps) if k == "dwt_tiles" else 1
        nl = kernels.get(k, {}).get("launches_per_frame", 0) / nst
        pk = per_kernel.setdefault(k, {"us_per_frame": 0.0, "bytes_per_frame": 0.0, "launches_per_frame": 0.0})
        pk["us_per_frame"] += v["avg_us"] * nl
        pk["bytes_per_frame"] += v["bytes"] * nl
        pk["launches_per_frame"] += nl
        v["us_per_frame"] = round(v["avg_us"] * nl, 2)
    dom = max(per_kernel, key=lambda k: per_kernel[k]["us_per_frame"])
    d = per_kernel[dom]
    bpl = d["bytes_per_frame"] / d["launches_per_frame"]
    avg_us = d["us_per_frame"] / d["launches_per_frame"]
    achieved = bpl / (avg_us * 1e-6) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": pmc_traffic(dom, "single"),
                "bytes_per_launch": round(bpl, 1), "avg_launch_us": round(avg_us, 3),
                "launches_per_frame": d["launches_per_frame"],
                "duration_source": "HIP events around graph replays of the kernel's launches with the frame's "
                                   "arguments, weighted by their launches per frame",
                "share_of_frame": round(d["us_per_frame"] * 1e-3 / float(np.median(frame_ms)), 3)}
    rp = kernel_stats_value(dom, "single", "avg_launch_us")
    if rp:
        roofline["rocprof_avg_launch_us"] = rp
        roofline["frac_rocprof"] = round(bpl / (rp * 1e-6) / 1e9 / HBM_PEAK_GBS, 5)
    # the whole frame: algorithmic bytes of every launch over the frame time
    fb = sum(pk["bytes_per_frame"] for pk in per_kernel.values())
    for name, kv in kernels.items():
        if name not in OP_KERNELS:
            fb += frame_kernel_bytes(name, N, S, V, e, m, it, mp)
    p50 = float(np.median(lat_all))
    frame_frac = {"bytes_per_frame": round(fb), "frame_ms_p50": round(p50, 4),
                  "achieved_GB_s": round(fb / (p50 * 1e-3) / 1e9, 1),
                  "frac": round(fb / (p50 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    out = {
        "metric": METRIC,
        "value": round(it * args.steps / wall, 1),
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
                   "N": N, "S": S, "reductions": "f64", "frames_generated": len(seq),
                   "input": "seeded frozen-flow von Karman screens, SNR-10 slope noise"},
        "frame_ms_p50": round(float(np.percentile(lat_all, 50)), 4),
        "frame_ms_p99": round(float(np.percentile(lat_all, 99)), 4),
        "latency_frames": int(len(lat_all)),
        "timed_frames_ms_p50": round(float(np.percentile(frame_ms, 50)), 4),
        "frames_per_s": round(args.steps / wall, 1),
        "operator_apply_ms": round(op_ms, 4),
        "autotuner": {"chosen": tuned, "apply_us_per_candidate": {k: round(v * 1000, 2) for k, v in tune_ms.items()}},
        "operator_applies_per_s_alone": round(1000.0 / op_ms, 1),
        "last_frame_rel_res": last_info["rel_res"],
        "roofline": roofline,
        "frame_roofline": frame_frac,
        "kernel_launches_per_frame": round(sum(k["launches_per_frame"] for k in kernels.values()), 2),
        "kernels": {k: {kk: round(vv, 4) for kk, vv in v.items()}
                    for k, v in sorted(kernels.items(), key=lambda kv: -kv[1]["ms_per_frame"])},
        "operator_kernels": opk,
        "paper_context": "CPU aug. FEWHA MCAO 1.9 ms/frame on 12 Haswell cores (different system size)",
    }
    return out, ctx


def run_precond(args, dev, spec, seq):
    """Exact vs frequency-weighted ("modified") Jacobi preconditioner on the ELT system at
    tolerance 1e-3 (cap 200; the FP32 system does not reach 1e-4 within it): iterations to the
    tolerance per frame and frame time.  The weights
    (the two lowest-frequency groups, the coarsest details and the scaling coefficients, halved)
    are this library's choice; the paper gives none."""
    import numpy as np
    import torch
    import paper_2011_06842_amd as fw
    levels = spec.layers[0].levels
    lw = tuple([1.0] * (levels - 1) + [0.5, 0.5])
    F = min(args.precond_frames, len(seq))
    slopes = torch.from_numpy(seq[:F]).to(dev)
    out = {"workload": f"elt_mcao_fp32 tolerance 1e-3 (cap 200), {F} frames", "level_weight": lw}
    for name, w in (("exact", None), ("weighted", lw)):
        sp = spec.copy(rel_tol=1e-3, max_iter=200, level_weight=w)
        ctx = fw.FewhaContext(sp, device=dev)
        info = ctx.new_info()
        its, ms = [], []
        for t in range(F):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ctx.fewha_solve_aug(slopes[t], info=info)
            e1.record()
            torch.cuda.synchronize()
            g = fw.decode_info(info)
            its.append(g["iters"])
            ms.append(e0.elapsed_time(e1))
        out[name] = {"first_frame_iterations": its[0], "iterations_mean_after_first": round(float(np.mean(its[1:])), 2),
                     "frame_ms_p50_after_first": round(float(np.median(ms[1:])), 3)}
        del ctx
    log(f"preconditioner: iterations exact {out['exact']}, weighted {out['weighted']}")
    return out


def free_running_errors(spec, slopes_dev, sols, sols_p, dev):
    """A fresh GPU context over the frames the oracle solved: relative error of every frame's
    coefficients against the FP64 oracle, next to the oracle's own drift when every operator
    output is perturbed at FP32 rounding size and, for FP64, at FP64 rounding size (the method's
    sensitivity over the same frames).  `sols_p`: perturbed solutions by the exponent e of 2^-e."""
    import numpy as np
    import paper_2011_06842_amd as fw
    vctx = fw.FewhaContext(spec, device=dev)
    errs = []
    sens = {e: [] for e in sols_p}
    for t, ref in enumerate(sols):
        g = vctx.fewha_solve_aug(slopes_dev[t]).double().cpu().numpy()
        errs.append(float(np.linalg.norm(g - ref) / np.linalg.norm(ref)))
        for e, sp in sols_p.items():
            sens[e].append(float(np.linalg.norm(sp[t] - ref) / np.linalg.norm(ref)))
    out = {"frames": len(sols), "max": max(errs), "last": errs[-1], "per_frame": [float(f"{x:.3e}") for x in errs]}
    for e, v in sens.items():
        out[f"oracle_vs_oracle_with_M_outputs_perturbed_2^-{e}"] = [float(f"{x:.3e}") for x in v]
        out[f"oracle_vs_oracle_2^-{e}_max"] = max(v)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--tuning", default="auto",
                    help="single-instance tile shapes: auto (the autotuner) or synS_rowsR, e.g. syn16_rows1")
    ap.add_argument("--batch-tuning", default="auto", help="batched-leg tile shapes (as --tuning)")
    ap.add_argument("--latency-frames", type=int, default=2000,
                    help="frames of the single-instance sequence (timed frames first, the rest a latency pass)")
    ap.add_argument("--cpu-frames", type=int, default=20, help="frames of the single-thread oracle baseline")
    ap.add_argument("--cpu-frames-all", type=int, default=5, help="frames per process of the all-core baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-frames", type=int, default=20)
    ap.add_argument("--kernel-reps", type=int, default=100)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB")
    ap.add_argument("--small", type=int, default=1, help="8 m FP64 leg (0: skip)")
    ap.add_argument("--small-frames", type=int, default=2000)
    ap.add_argument("--loop", type=int, default=1, help="full ELT closed-loop leg (0: skip)")
    ap.add_argument("--loop-frames", type=int, default=2000)
    ap.add_argument("--loop-check-frames", type=int, default=5, help="loop frames compared with the oracle")
    ap.add_argument("--loop-fit-iter", type=int, default=4)
    ap.add_argument("--loop-pts", type=int, default=40)
    ap.add_argument("--loop-gain", type=float, default=0.4)
    ap.add_argument("--precond", type=int, default=1, help="exact vs frequency-weighted Jacobi leg (0: skip)")
    ap.add_argument("--precond-frames", type=int, default=20)
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

    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    import numpy as np

    # inputs and CPU baselines first, in forked processes, before anything touches the GPU
    workers = pool_size()
    F = max(args.warmup + args.steps, args.latency_frames)
    t0 = time.perf_counter()
    gen_s = {}
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("fork")) as ex:
        spec, seq = gen_sequence(ex, "elt", SEED, F)
        small = gen_sequence(ex, "small", SEED + 2, args.small_frames) if args.small else None
        full = gen_sequence(ex, "full", SEED + 3, args.loop_frames) if args.loop else None
        t1 = time.perf_counter()
        atmos = [gen_sequence(ex, "elt", SEED + 1 + a, batch_frames_needed(args))
                 for a in range(min(BATCH_ATMOSPHERES, args.batch))] if args.batch > 0 else None
        gen_s["batched"] = round(time.perf_counter() - t1, 1)
        t1 = time.perf_counter()
        ragged = ragged_inputs(ex, args) if args.ragged > 0 else None
        gen_s["ragged"] = round(time.perf_counter() - t1, 1)
        t1 = time.perf_counter()
        ws = warmstart_inputs(ex, args) if args.warmstart else None
        gen_s["warmstart"] = round(time.perf_counter() - t1, 1)
    t_gen = time.perf_counter() - t0
    log(f"inputs: {F} ELT frames{', small and full-loop sequences' if args.small or args.loop else ''} "
        f"generated in {t_gen:.1f} s ({workers} processes)")
    cpu = None
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        info = host_cpu_info()
        nf = max(1, min(args.cpu_frames, F))
        s1, sa, sols, sols_p = cpu_baselines(spec, seq, nf, max(1, args.cpu_frames_all), workers)
        cpu = {"elt": (s1, sa, sols, sols_p)}
        if args.small:
            nsm = min(len(small[1]), 2 * nf)
            cpu["small"] = cpu_baselines(small[0], small[1], nsm, max(1, nsm // 4), workers)
        loop_ref = None
        if args.loop and args.loop_check_frames:
            loop_ref = _oracle_loop_run((full[0], full[1][:args.loop_check_frames], args.loop_pts,
                                         args.loop_fit_iter, args.loop_gain))
        log(f"CPU baselines: {time.perf_counter() - t0:.1f} s on {info['model']} ({workers} processes)")

    import torch
    dev = "cuda:0"
    out, ctx = run_single(args, dev, spec, seq)
    slopes = torch.from_numpy(seq[:args.cpu_frames]).to(dev)
    log("single instance: kernel profile and per-kernel timer done")
    if cpu is not None:
        s1, sa, sols, sols_p = cpu["elt"]
        info = host_cpu_info()
        out["cpu_baseline"] = {
            "value": sa["applies_per_s"], "unit": "applies/s", "cores": workers, "kind": "oracle",
            "sample": f"first {sa['frames'] // workers} frames of the same ELT sequence solved by each of {workers} "
                      f"single-threaded processes of the FP64 NumPy oracle from a common start",
            "cpu_model": info["model"], "nproc": info["nproc"], "cpus_available": info["affinity"],
            "all_core": sa, "single_thread": {**s1, "sample": f"first {s1['frames']} frames, one process, one thread"}}
        out["rel_err_vs_oracle_free_running"] = free_running_errors(spec, slopes, sols, sols_p, dev)
    del ctx
    torch.cuda.empty_cache()
    out["input_generation_s"] = round(t_gen, 2)
    if args.small:
        out["small"] = run_small(args, dev, *small)
        if cpu is not None:
            s1, sa, sols, sols_p = cpu["small"]
            out["small"]["cpu_baseline"] = {"single_thread": s1, "all_core": {**sa, "cores": workers}}
            sl = torch.from_numpy(small[1][:len(sols)]).to(dev)
            out["small"]["rel_err_vs_oracle_free_running"] = free_running_errors(small[0], sl, sols, sols_p, dev)
        log(f"small FP64: frame p50 {out['small']['frame_ms_p50']} ms")
        torch.cuda.empty_cache()
    if args.loop:
        res, early = run_full_loop(args, dev, *full)
        if cpu is not None and loop_ref is not None:
            refs, ts = loop_ref
            res["rel_err_vs_oracle_commands"] = [float(f"{np.linalg.norm(a - r) / np.linalg.norm(r):.3e}")
                                                 for a, r in zip(early, refs)]
            res["oracle_loop_step_ms"] = round(1000 * float(np.median(ts)), 1)
        out["full_loop"] = res
        log(f"full ELT loop: step p50 {res['loop_step_ms_p50']} ms, p99 {res['loop_step_ms_p99']} ms")
        torch.cuda.empty_cache()
    if args.precond:
        out["preconditioner"] = run_precond(args, dev, spec, seq)
        torch.cuda.empty_cache()
    if args.batch > 0:
        out["batched"] = run_batch(args, dev, atmos, gen_s["batched"])
        torch.cuda.empty_cache()
    if args.ragged > 0:
        out["ragged"] = run_ragged(args, dev, ragged, gen_s["ragged"])
        torch.cuda.empty_cache()
    if args.unet:
        out["unet"] = run_unet(args, dev)
        torch.cuda.empty_cache()
    if args.warmstart:
        out["warmstart"] = run_warmstart(args, dev, ws, gen_s["warmstart"])
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
