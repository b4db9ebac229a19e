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
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "augmented-PCG frame latency p50/p99 (ms) + operator applies/s, % HBM roofline"
HBM_PEAK_GBS = 8000.0
SEED = 20201112


def family_bytes(fam: str, spec, N: int, S: int, V: int, e: int, m: int, it: int) -> float:
    """Algorithmic HBM bytes of one frame's launches of a kernel family: every operand the
    family must read or write once, intermediates between families included (they leave
    the kernel), nothing counted twice within a kernel."""
    apply_n = it                       # operator applications per frame (steady state)
    if fam == "idwt":        # coefficients in, nodal layers out
        return apply_n * 2 * N * e
    if fam == "dwt":         # nodal in, coefficients out; + x and alpha D for the prior (applies)
        return apply_n * 4 * N * e + 2 * N * e
    if fam == "data_term":   # nodal layers in, slope weights in, sensor nodes out
        return apply_n * (N + S + V) * e
    if fam == "adj_gather":  # sensor nodes in, layer nodes out (applies + right-hand side)
        return (apply_n + 1) * (V + N) * e
    if fam == "slopes_adj":  # slopes and weights in, sensor nodes out
        return (2 * S + V) * e
    if fam == "gram":        # m U, m Q, r
        return (2 * m + 1) * N * e
    if fam == "galerkin_apply":  # c, r, J^-1, m U, m Q in; c, r, z out
        return (3 + 2 * m + 3) * N * e
    if fam == "init_dir":    # z, r, m U in; p out
        return (2 + m + 1) * N * e
    if fam == "dot":
        return it * 2 * N * e
    if fam == "update1":     # p, q, c, r, J^-1, u_last, q_last in; c, r, z out
        return it * (7 + 3) * N * e
    if fam == "update2":     # z, p, u_last in; p out
        return (it - 1) * 4 * N * e
    if fam == "residual":    # b, b_prev, r in; r, b_prev out
        return 5 * N * e
    return 0.0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-frames", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-frames", type=int, default=20)
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py measures one MI355X: the frame solve runs on a single GPU and this build has no "
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

    # per-kernel-family durations from HIP events around every launch of a fresh run of the
    # same frames (profiling synchronises per call, so it runs outside the timed region)
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
    m = spec.recycle_k
    fams = {}
    for name, (ms, nl) in prof.items():
        if nl == 0:
            continue
        b = family_bytes(name, spec, N, S, V, 4, m, it)
        fams[name] = {"ms_per_frame": ms / P, "launches_per_frame": nl / P, "avg_launch_us": 1000 * ms / nl,
                      "bytes_per_launch": b / (nl / P) if b else None}
    dom = max((k for k in fams if fams[k]["bytes_per_launch"]), key=lambda k: fams[k]["ms_per_frame"])
    d = fams[dom]
    achieved = d["bytes_per_launch"] / (d["avg_launch_us"] * 1e-6) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                "bytes_per_launch": d["bytes_per_launch"], "avg_launch_us": round(d["avg_launch_us"], 3)}

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
        "kernels": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in sorted(fams.items(), key=lambda kv: -kv[1]["ms_per_frame"])},
        "paper_context": "CPU aug. FEWHA MCAO 1.9 ms/frame on 12 Haswell cores (different system size)",
    }

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
        out["rel_err_vs_oracle_max"] = max(errs)
    out["input_generation_s"] = round(t_gen, 2)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
