"""GPU (HIP, through the C ABI) versus the FP64 oracle, element by element on the same
seeded inputs.  Bars: relative error <= 1e-12 (operators) / 1e-10 (frames) in FP64 and
<= 5e-5 with the FP32 operator; bitwise for determinism and checkpoint/resume."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth
from oracle import AugmentedReconstructor, OracleSystem
import paper_2011_06842_amd as fw

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dtype)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def _calibrated(spec, frames, seed):
    seq = synth.make_sequence(spec, frames, seed=seed)
    return spec, seq


_CACHE = {}


def system(name, precision="fp64"):
    key = (name, precision)
    if key not in _CACHE:
        if name == "tiny":
            spec, seq = synth.config_tiny(), None
        elif name == "tiny_full_levels":
            spec, seq = synth.config_tiny(n=8, levels=3, n_sub=12), None
        elif name == "mixed":
            spec, seq = synth.config_mixed(), None
        elif name == "small":
            spec, seq = _calibrated(synth.config_small(), 12, seed=5)
        elif name == "elt":
            spec, seq = _calibrated(synth.config_elt_mcao(precision=precision), 8, seed=6)
        elif name == "elt_full":
            spec, seq = _calibrated(synth.config_elt_full(precision=precision), 6, seed=7)
        spec.precision = precision
        if seq is None:
            rng = np.random.default_rng(17)
            base = rng.standard_normal(synth.n_slopes(spec))
            seq = np.stack([base + 0.1 * t * rng.standard_normal(base.size) for t in range(8)])
            m = np.concatenate([np.concatenate([w.mask.ravel(), w.mask.ravel()]) for w in spec.wfs])
            seq = seq * m
        _CACHE[key] = (spec, seq, OracleSystem(spec))
    return _CACHE[key]


OPS_CASES = ["tiny", "tiny_full_levels", "mixed", "small", "elt"]


@pytest.mark.parametrize("name", OPS_CASES)
def test_operator_pieces_fp64(name):
    spec, seq, sysm = system(name)
    ctx = fw.FewhaContext(spec, device=DEV)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(sysm.N)
    s = rng.standard_normal(sysm.S)
    phis = sysm.W_inv(x)
    np.testing.assert_array_less(rel(host(ctx.fewha_apply_piece(fw.PIECE_WINV, dev(x, np.float64))),
                                     np.concatenate([p.ravel() for p in phis])), 1e-13)
    img = rng.standard_normal(sysm.N)
    np.testing.assert_array_less(rel(host(ctx.fewha_apply_piece(fw.PIECE_WINVT, dev(img, np.float64))),
                                     sysm.W_invT(sysm.split_layers(img))), 1e-13)
    np.testing.assert_array_less(rel(host(ctx.fewha_apply_piece(fw.PIECE_A, dev(img, np.float64))),
                                     sysm.A(sysm.split_layers(img))), 1e-13)
    np.testing.assert_array_less(rel(host(ctx.fewha_apply_piece(fw.PIECE_AT, dev(s, np.float64))),
                                     np.concatenate([p.ravel() for p in sysm.A_T(s)])), 1e-13)


@pytest.mark.parametrize("name", OPS_CASES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_prior_preconditioner_apply_and_rhs(name, precision):
    spec, seq, sysm = system(name, precision)
    ctx = fw.FewhaContext(spec, device=DEV)
    dt = np.float64 if precision == "fp64" else np.float32
    tol_vec = 1e-13 if precision == "fp64" else 2e-7
    tol_op = 1e-12 if precision == "fp64" else 2e-5
    D = sysm.prior()
    np.testing.assert_allclose(host(ctx.fewha_get_vector(0)), sysm.alpha * D, rtol=tol_vec)
    np.testing.assert_allclose(host(ctx.fewha_get_vector(1)), 1.0 / sysm.diag_M(D), rtol=tol_vec * 10)
    x = np.random.default_rng(2).standard_normal(sysm.N)
    y = host(ctx.fewha_apply_A(dev(x, dt)))
    assert rel(y, sysm.apply_M(x.astype(dt).astype(np.float64), D)) <= tol_op
    b = host(ctx.fewha_rhs(dev(seq[0], dt)))
    assert rel(b, sysm.rhs(seq[0].astype(dt).astype(np.float64))) <= tol_op


def _run_sequence(spec, seq, sysm, frames, ctx=None, **kw):
    dt = np.float64 if spec.precision == "fp64" else np.float32
    ctx = ctx or fw.FewhaContext(spec, device=DEV)
    ref = AugmentedReconstructor(sysm, **kw)
    info = ctx.new_info()
    errs, infos = [], []
    for t in range(frames):
        c_ref, i_ref = ref.solve(seq[t].astype(dt).astype(np.float64))
        c = host(ctx.fewha_solve_aug(dev(seq[t], dt), info=info))
        errs.append(rel(c, c_ref))
        gi = fw.decode_info(info)
        infos.append((gi, i_ref))
    return errs, infos


@pytest.mark.parametrize("name", ["tiny", "mixed", "small"])
@pytest.mark.parametrize("mode, project_all", [("galerkin", False), ("paper", False), ("galerkin", True)])
def test_frame_sequence_fp64(name, mode, project_all):
    spec, seq, sysm = system(name)
    spec = spec.copy(recycle_mode=mode, project_all=project_all)
    sysm = OracleSystem(spec)
    errs, infos = _run_sequence(spec, seq, sysm, len(seq))
    assert max(errs) <= 1e-10, errs
    for gi, ri in infos:
        assert gi["iters"] == ri["iters"] and gi["recycle_used"] == ri["recycle_used"]
        assert gi["dropped"] == ri["dropped"] and gi["flags"] == 0
        assert abs(gi["rel_res"] - ri["rel_res"]) <= 1e-9 * ri["rel_res"]


@pytest.mark.parametrize("mode, project_all", [("galerkin", False), ("paper", False), ("galerkin", True)])
def test_zero_frame_then_frames_fp64(mode, project_all):
    """An all-zero slope frame (b = 0, exact residual 0) returns c = 0; its zero curvature with
    a zero residual is exact convergence, not a breakdown; the zero directions it stores get
    zero coefficients, so the following frames are finite and match the oracle."""
    spec, seq, _ = system("small")
    spec = spec.copy(recycle_mode=mode, project_all=project_all)
    sysm = OracleSystem(spec)
    frames = np.concatenate([np.zeros_like(seq[:1]), seq[:4]])
    errs, infos = [], []
    ctx = fw.FewhaContext(spec, device=DEV)
    ref = AugmentedReconstructor(sysm)
    info = ctx.new_info()
    for t in range(frames.shape[0]):
        c_ref, i_ref = ref.solve(frames[t])
        c = host(ctx.fewha_solve_aug(dev(frames[t], np.float64), info=info))
        gi = fw.decode_info(info)
        if t == 0:
            np.testing.assert_array_equal(c, 0.0)
            assert gi["flags"] == 0 and gi["rel_res"] == 0.0 and i_ref["rel_res"] == 0.0 and i_ref["flags"] == 0
        else:
            assert np.all(np.isfinite(c)) and gi["flags"] == 0, (t, gi)
            errs.append(rel(c, c_ref))
    assert max(errs) <= 1e-10, errs


@pytest.mark.parametrize("mode", ["galerkin", "paper"])
def test_large_recycle_space_fp64(mode):
    """k = 20 recycled directions (20 iterations per frame, so that the PAPER mode, which
    recycles the previous frame's directions, also reaches 20): the Gram pass spans 2 x 2
    tiles of 16 (off-diagonal tiles load their own J^-1 Q rows).  Frames this long amplify
    rounding-order differences (the non-conjugate sequential projections of the PAPER mode
    most), so each frame's bar is 10 times the oracle's own deviation when the slopes are
    perturbed at 1e-15, and at least 1e-10."""
    spec, seq, _ = system("small")
    spec = spec.copy(recycle_k=20, max_iter=20, recycle_mode=mode)
    sysm = OracleSystem(spec)
    frames = 4
    errs, infos = _run_sequence(spec, seq, sysm, frames)
    a, b = AugmentedReconstructor(sysm), AugmentedReconstructor(sysm)
    rng = np.random.default_rng(0)
    for t in range(frames):
        ca, _ = a.solve(seq[t])
        cb, _ = b.solve(seq[t] * (1 + 1e-15 * rng.standard_normal(seq[t].shape)))
        assert errs[t] <= max(1e-10, 10 * rel(cb, ca)), (t, errs[t], rel(cb, ca))
    assert max(gi["recycle_used"] for gi, _ in infos) == 20
    for gi, ri in infos:
        assert gi["recycle_used"] == ri["recycle_used"] and gi["dropped"] == ri["dropped"]


@pytest.mark.parametrize("k", [1, 3, 4, 5, 7, 8, 11, 12, 15, 24, 32])
def test_recycle_dimensions_galerkin_fp64(k):
    """GALERKIN frames with k recycled directions across the Gram's forms: one 4x4 block
    diagonal (k <= 3), two (4 <= k <= 7) and three (8 <= k <= 11) of the small-block
    matrix-core form, the 16x16 tile (12 <= k <= 15) and 2 x 2 tiles (24, 32; the elimination's
    widest register blocking at 32).  As many iterations per frame as k,
    so the ring holds k directions from the second frame on; the same bar as the k = 20 test
    (10 times the oracle's own deviation under 1e-15 slope perturbations, at least 1e-10)."""
    spec, seq, _ = system("small")
    spec = spec.copy(recycle_k=k, max_iter=max(k, 4), recycle_mode="galerkin")
    sysm = OracleSystem(spec)
    frames = 4
    errs, infos = _run_sequence(spec, seq, sysm, frames)
    a, b = AugmentedReconstructor(sysm), AugmentedReconstructor(sysm)
    rng = np.random.default_rng(1)
    for t in range(frames):
        ca, _ = a.solve(seq[t])
        cb, _ = b.solve(seq[t] * (1 + 1e-15 * rng.standard_normal(seq[t].shape)))
        assert errs[t] <= max(1e-10, 10 * rel(cb, ca)), (t, errs[t], rel(cb, ca))
    assert max(gi["recycle_used"] for gi, _ in infos) == k
    for gi, ri in infos:
        assert gi["recycle_used"] == ri["recycle_used"] and gi["dropped"] == ri["dropped"] and gi["flags"] == 0


def test_plain_pcg_k0_fp64():
    spec, seq, sysm = system("small")
    spec = spec.copy(recycle_k=0)
    errs, _ = _run_sequence(spec, seq, OracleSystem(spec), 6)
    assert max(errs) <= 1e-10, errs


def test_frame_sequence_elt_fp32():
    spec, seq, sysm = system("elt", "fp32")
    errs, infos = _run_sequence(spec, seq, sysm, len(seq))
    assert max(errs) <= 5e-5, errs
    for gi, ri in infos:
        assert gi["recycle_used"] == ri["recycle_used"]


def test_frame_sequence_elt_fp64():
    spec, seq, sysm = system("elt", "fp64")
    errs, _ = _run_sequence(spec, seq, sysm, 4)
    assert max(errs) <= 1e-10, errs


@pytest.mark.parametrize("precision, tol", [("fp64", 1e-10), ("fp32", 5e-5)])
def test_frame_sequence_elt_full_loop(precision, tol):
    """The full ELT loop's system (6 LGS + one 2x2 and two 1x1 low-order NGS): frames from
    setup against the oracle."""
    spec, seq, sysm = system("elt_full", precision)
    errs, infos = _run_sequence(spec, seq, sysm, len(seq))
    assert max(errs) <= tol, errs
    for gi, ri in infos:
        assert gi["recycle_used"] == ri["recycle_used"] and gi["flags"] == 0


def test_reset_restarts_from_true_residual():
    spec, seq, sysm = system("small")
    ctx = fw.FewhaContext(spec, device=DEV)
    ref = AugmentedReconstructor(sysm)
    for t in range(6):
        if t == 3:
            ctx.fewha_reset()
            ref.reset()
        c_ref, _ = ref.solve(seq[t])
        c = host(ctx.fewha_solve_aug(dev(seq[t], np.float64)))
        assert rel(c, c_ref) <= 1e-10


def test_checkpoint_resume_and_determinism_bitwise():
    spec, seq, sysm = system("small")
    a = fw.FewhaContext(spec, device=DEV)
    outs = [host(a.fewha_solve_aug(dev(seq[t], np.float64))) for t in range(8)]
    b = fw.FewhaContext(spec, device=DEV)
    for t in range(4):
        b.fewha_solve_aug(dev(seq[t], np.float64))
    state = b.fewha_get_state()
    c = fw.FewhaContext(spec, device=DEV)
    c.fewha_set_state(state)
    for t in range(4, 8):
        out = host(c.fewha_solve_aug(dev(seq[t], np.float64)))
        assert np.array_equal(out, outs[t]), t
    d = fw.FewhaContext(spec, device=DEV)
    again = [host(d.fewha_solve_aug(dev(seq[t], np.float64))) for t in range(8)]
    assert all(np.array_equal(x, y) for x, y in zip(outs, again))


@pytest.mark.parametrize("name", ["small", "elt"])
def test_graph_replay_matches_direct_launches_bitwise(name):
    """Captured frame graphs (one per recycle-ring phase, replayed with changing slope and
    output buffers, torch work in between) give the same bits as direct launches."""
    spec, seq, sysm = system(name, "fp32" if name == "elt" else "fp64")
    dt = np.float64 if spec.precision == "fp64" else np.float32
    a = fw.FewhaContext(spec, device=DEV)
    b = fw.FewhaContext(spec, device=DEV)
    b.fewha_use_graphs(False)
    info_a, info_b = a.new_info(), b.new_info()
    for t in range(len(seq)):
        s_dev = dev(seq[t], dt)
        ca = a.fewha_solve_aug(s_dev.clone(), info=info_a)
        _ = torch.ones(1000, device=DEV).sum()          # unrelated stream work between replays
        cb = b.fewha_solve_aug(s_dev, info=info_b)
        assert torch.equal(ca, cb), t
        assert fw.decode_info(info_a) == fw.decode_info(info_b)


@pytest.mark.parametrize("name, precision", [("small", "fp64"), ("elt", "fp32")])
def test_kernel_timer_leaves_carried_state_and_rejects_bad_ids(name, precision):
    """The per-kernel timer runs operator kernels on scratch buffers only: the next frame is
    bitwise the one an untimed context computes."""
    spec, seq, _ = system(name, precision)
    dt = np.float64 if precision == "fp64" else np.float32
    a = fw.FewhaContext(spec, device=DEV)
    b = fw.FewhaContext(spec, device=DEV)
    for t in range(3):
        a.fewha_solve_aug(dev(seq[t], dt))
        b.fewha_solve_aug(dev(seq[t], dt))
    steps = a.fewha_wavelet_steps()
    for kid in range(5):
        for st in (range(len(steps)) if kid == 3 else [0]):
            assert a.fewha_time_kernel(kid, st, 3) > 0
    with pytest.raises(fw.FewhaError):
        a.fewha_time_kernel(5, 0, 3)
    with pytest.raises(fw.FewhaError):
        a.fewha_time_kernel(3, len(steps), 3)
    if name == "elt":   # one tiled analysis launch: 256 -> 32 (ground), 128 -> 32 (the 8 others)
        assert steps == [(256, 9)]
    ca = host(a.fewha_solve_aug(dev(seq[3], dt)))
    cb = host(b.fewha_solve_aug(dev(seq[3], dt)))
    assert np.array_equal(ca, cb)


def test_state_from_other_configuration_rejected():
    spec, seq, sysm = system("small")
    a = fw.FewhaContext(spec, device=DEV)
    b = fw.FewhaContext(system("tiny")[0], device=DEV)
    with pytest.raises(fw.FewhaError, match="FEWHA_E_STATE"):
        b.fewha_set_state(a.fewha_get_state())


STATE_MAGIC = 0x46455748415354


def load_oracle_state(ctx, ref, spec):
    """Round the oracle reconstructor's carried state (c, r, b_prev, recycled directions) to the
    context's element type, in place, and write it into the GPU context through
    fewha_set_state in the documented checkpoint layout (256-byte header of uint64: magic, N,
    slots, element size, ring head, stored count, previous iterations, first-frame flag,
    instances; then (p_j, q_j) per slot; c, r, b_prev; U and Q slot-major).  Both sides then
    continue from the same state; nothing flows from the GPU to the oracle."""
    esz = 8 if spec.precision == "fp64" else 4
    dt = np.float64 if esz == 8 else np.float32
    rnd = lambda v: np.asarray(v, dtype=dt).astype(np.float64)
    N = ref.sys.N
    slots = spec.recycle_k + spec.max_iter
    m = len(ref.store)
    ref.c, ref.r, ref.b_prev = rnd(ref.c), rnd(ref.r), rnd(ref.b_prev)
    ref.store = [(rnd(p), rnd(q), float(g)) for p, q, g in ref.store]
    hdr = np.zeros(32, dtype=np.uint64)
    hdr[:9] = [STATE_MAGIC, N, slots, esz, m % slots, m, spec.max_iter, int(ref.first), 1]
    gam = np.zeros(slots + 1)
    gam[slots] = m
    U = np.zeros((slots, N), dtype=dt)
    Q = np.zeros((slots, N), dtype=dt)
    for j, (p, q, g) in enumerate(ref.store):
        gam[j], U[j], Q[j] = g, p, q
    raw = b"".join([hdr.tobytes(), gam.tobytes(), ref.c.astype(dt).tobytes(), ref.r.astype(dt).tobytes(),
                    ref.b_prev.astype(dt).tobytes(), U.tobytes(), Q.tobytes()])
    buf = torch.from_numpy(np.frombuffer(raw, dtype=np.uint8).copy()).to(DEV)
    assert buf.numel() == ctx.fewha_state_size()
    ctx.fewha_set_state(buf)


@pytest.mark.parametrize("name, precision, frames, tol", [("elt", "fp32", 40, 5e-5), ("elt", "fp64", 12, 1e-10),
                                                          ("elt_full", "fp32", 24, 5e-5),
                                                          ("elt_full", "fp64", 8, 1e-10)])
def test_elt_frame_map_parity_from_identical_state(name, precision, frames, tol):
    """The frame update from an identical carried state at several points of a longer
    sequence (free-running sequences drift apart by the method's own sensitivity, see the
    free-running test): the oracle runs the sequence, its state is loaded into the GPU context,
    and one frame on each side is compared.  elt_full adds the three low-order natural guide
    stars (one 2x2, two 1x1)."""
    spec, _, sysm = system(name, precision)
    seq = synth.make_sequence(spec.copy(), frames + 1, seed=20201112)
    dt = np.float64 if precision == "fp64" else np.float32
    ref = AugmentedReconstructor(sysm)
    ctx = fw.FewhaContext(spec, device=DEV)
    info = ctx.new_info()
    checks = {1, frames // 2, frames}
    for t in range(frames + 1):
        s = seq[t].astype(dt).astype(np.float64)
        if t in checks:
            load_oracle_state(ctx, ref, spec)
            c = host(ctx.fewha_solve_aug(dev(s, dt), info=info))
            c_ref, i_ref = ref.solve(s)
            gi = fw.decode_info(info)
            assert rel(c, c_ref) <= tol, (t, rel(c, c_ref))
            assert gi["recycle_used"] == i_ref["recycle_used"] and gi["flags"] == 0
        else:
            ref.solve(s)


def test_free_running_elt_fp32_within_the_methods_own_sensitivity():
    """40 free-running cfg2 frames (FP32 operator, no state exchanged with the oracle).  Any
    rounding at FP32 level makes the frame sequence of Alg. 3 drift from the FP64 one: the
    oracle itself, with every operator output perturbed by a relative 2^-24 (seeded), drifts
    away from the unperturbed oracle by 1e-5 after 10 frames and by 1e-4 to 1e-3 after 30 (the
    recycled iteration amplifies it).  The bar per frame is therefore 10 times the largest such
    oracle-vs-oracle drift so far, and at least the 5e-5 split-precision bar; the final
    residuals of the two sequences agree within 5 %."""
    spec = synth.config_elt_mcao(precision="fp32")
    frames = 40
    seq = synth.make_sequence(spec, frames, seed=6).astype(np.float32).astype(np.float64)
    sysm = OracleSystem(spec)
    ref = AugmentedReconstructor(sysm)
    pert = AugmentedReconstructor(sysm, Jinv=ref.Jinv)
    rng = np.random.default_rng(5)
    pert.apply_M = lambda x: sysm.apply_M(x, ref.D) * (1 + 2.0 ** -24 * rng.standard_normal(sysm.N))
    ctx = fw.FewhaContext(spec, device=DEV)
    info = ctx.new_info()
    sens_max, rows = 0.0, []
    for t in range(frames):
        c_ref, i_ref = ref.solve(seq[t])
        c_pert, _ = pert.solve(seq[t])
        c = host(ctx.fewha_solve_aug(dev(seq[t], np.float32), info=info))
        gi = fw.decode_info(info)
        sens_max = max(sens_max, rel(c_pert, c_ref))
        err = rel(c, c_ref)
        rows.append((t, err, sens_max))
        assert err <= max(5e-5, 10 * sens_max), rows[-3:]
        assert abs(gi["rel_res"] - i_ref["rel_res"]) <= 0.05 * i_ref["rel_res"], (t, gi, i_ref)
    print("\nframe, GPU vs oracle, oracle drift under 2^-24 perturbations:",
          [(t, f"{e:.2e}", f"{s_:.2e}") for t, e, s_ in rows[::5]])


@pytest.mark.gpu
@pytest.mark.parametrize("name, precision", [("elt", "fp32"), ("small", "fp64")])
def test_autotuner_choices_change_no_bit(name, precision):
    """The autotuner times the four tile-shape candidates and keeps the fastest; frames solved
    with each candidate (set on a second context) are bit-identical to the default's."""
    spec, seq, _ = system(name, precision)
    dt = np.float64 if precision == "fp64" else np.float32
    a = fw.FewhaContext(spec, device=DEV)
    ref = [host(a.fewha_solve_aug(dev(seq[t], dt))) for t in range(3)]
    best, ms = a.fewha_autotune(reps=5)
    assert len(ms) == (4 if precision == "fp64" else 6) and all(v > 0 for v in ms.values())
    assert ms[f"syn{best['syn_tile']}_rows{best['gather_rows']}"] == min(ms.values())
    assert a.fewha_get_tuning() == best
    for syn_tile, rows in [(16, 1), (16, 4), (32, 1), (32, 4)] + ([(64, 1), (64, 4)] if precision == "fp32" else []):
        b = fw.FewhaContext(spec, device=DEV)
        b.fewha_set_tuning(syn_tile, rows)
        assert b.fewha_get_tuning() == {"syn_tile": syn_tile, "gather_rows": rows}
        for t in range(3):
            assert np.array_equal(host(b.fewha_solve_aug(dev(seq[t], dt))), ref[t]), (syn_tile, rows, t)
    with pytest.raises(fw.FewhaError):
        a.fewha_set_tuning(24, 1)
    if precision == "fp64":
        with pytest.raises(fw.FewhaError):
            a.fewha_set_tuning(64, 1)
