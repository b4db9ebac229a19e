"""Failure handling through the C ABI, forced from the host: frames with non-finite slopes,
a non-finite first frame, identical consecutive frames, and a broken instance inside a batch.
The oracle mirrors the library's breakdown rules (the paper is silent on them): a frame whose
right-hand side is not finite is not solved, the carried state keeps its values and the frame
stores null directions.  Every kernel exits normally on these inputs (they only carry NaN/Inf
values through arithmetic)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth
from oracle import AugmentedReconstructor, OracleSystem
import paper_2011_06842_amd as fw

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]
DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def dev(x, dtype=np.float64):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dtype)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def _small(frames=6, seed=5):
    spec = synth.config_small()
    seq = synth.make_sequence(spec, frames, seed=seed)
    return spec, seq


def _slope_index(spec, active):
    """Index of an x-slope of sensor 0 on an active (or inactive) subaperture."""
    m = spec.wfs[0].mask.ravel()
    return int(np.flatnonzero(m if active else ~m)[len(np.flatnonzero(m if active else ~m)) // 2])


@pytest.mark.parametrize("bad", [np.nan, np.inf])
@pytest.mark.parametrize("mode", ["galerkin", "paper"])
@pytest.mark.parametrize("graphs", [True, False])
def test_nonfinite_slopes_frame_is_skipped_fp64(bad, mode, graphs):
    """Frame 2 carries a non-finite slope: its output is the previous frame's coefficients,
    bit for bit, with flags 1 | 8 and a NaN relative residual; the next frame call reports
    FEWHA_E_BREAKDOWN once; every other frame matches the oracle (which skips the same frame)
    at 1e-10."""
    spec, seq = _small()
    spec = spec.copy(recycle_mode=mode)
    sysm = OracleSystem(spec)
    ctx = fw.FewhaContext(spec, device=DEV)
    ctx.fewha_use_graphs(graphs)
    ref = AugmentedReconstructor(sysm)
    info = ctx.new_info()
    frames = seq.copy()
    frames[2, _slope_index(spec, True)] = bad
    prev = None
    for t in range(frames.shape[0]):
        print(f"frame {t} bad={bad} mode={mode} graphs={graphs}", flush=True)
        c_ref, i_ref = ref.solve(frames[t])
        c = host(ctx.fewha_solve_aug(dev(frames[t]), info=info))
        gi = fw.decode_info(info)
        if t == 2:
            np.testing.assert_array_equal(c, prev)
            assert gi["flags"] == 9 and np.isnan(gi["rel_res"]) and i_ref["flags"] == 9
            assert ctx.breakdown_reports == []
        else:
            assert gi["flags"] == 0, (t, gi)
            assert rel(c, c_ref) <= 1e-10, (t, rel(c, c_ref))
            assert gi["recycle_used"] == i_ref["recycle_used"] and gi["dropped"] == i_ref["dropped"]
        if t == 3:
            assert len(ctx.breakdown_reports) == 1 and "frame 3 " in ctx.breakdown_reports[0]
        prev = c
    assert len(ctx.breakdown_reports) == 1


def test_nonfinite_slope_of_an_inactive_subaperture_is_ignored():
    """Inactive subapertures do not enter the operator: a NaN there changes nothing."""
    spec, seq = _small(3)
    sysm = OracleSystem(spec)
    ctx = fw.FewhaContext(spec, device=DEV)
    ref = AugmentedReconstructor(sysm)
    info = ctx.new_info()
    frames = seq.copy()
    frames[:, _slope_index(spec, False)] = np.nan
    for t in range(frames.shape[0]):
        c_ref, i_ref = ref.solve(frames[t])
        c = host(ctx.fewha_solve_aug(dev(frames[t]), info=info))
        gi = fw.decode_info(info)
        assert gi["flags"] == 0 and i_ref["flags"] == 0 and rel(c, c_ref) <= 1e-10, (t, gi)
    assert ctx.breakdown_reports == []


def test_nonfinite_first_frame_keeps_the_residual_consistent():
    """A non-finite first frame (after setup: c = 0) returns c = 0; the next frames are the
    oracle's."""
    spec, seq = _small(4)
    sysm = OracleSystem(spec)
    ctx = fw.FewhaContext(spec, device=DEV)
    ref = AugmentedReconstructor(sysm)
    info = ctx.new_info()
    frames = np.concatenate([np.full_like(seq[:1], np.nan), seq])
    for t in range(frames.shape[0]):
        c_ref, _ = ref.solve(frames[t])
        c = host(ctx.fewha_solve_aug(dev(frames[t]), info=info))
        gi = fw.decode_info(info)
        if t == 0:
            np.testing.assert_array_equal(c, 0.0)
            assert gi["flags"] == 9
        else:
            assert gi["flags"] == 0 and rel(c, c_ref) <= 1e-10, (t, gi, rel(c, c_ref))


def test_nonfinite_frame_fp32_continues_within_split_precision_bar():
    """FP32 operator: the skipped frame returns the previous coefficients bit for bit, and the
    frames after it stay within the split-precision bar of the oracle."""
    spec, seq = _small()
    spec = spec.copy(precision="fp32")
    sysm = OracleSystem(spec)
    ctx = fw.FewhaContext(spec, device=DEV)
    ref = AugmentedReconstructor(sysm)
    info = ctx.new_info()
    frames = seq.astype(np.float32).astype(np.float64)
    frames[3, _slope_index(spec, True)] = np.inf
    prev = None
    for t in range(frames.shape[0]):
        c_ref, _ = ref.solve(frames[t])
        c = host(ctx.fewha_solve_aug(dev(frames[t], np.float32), info=info))
        gi = fw.decode_info(info)
        if t == 3:
            np.testing.assert_array_equal(c, prev)
            assert gi["flags"] == 9
        else:
            assert gi["flags"] == 0 and rel(c, c_ref) <= 5e-5, (t, rel(c, c_ref))
        prev = c


@pytest.mark.parametrize("mode", ["galerkin", "paper"])
def test_identical_consecutive_frames_fp64(mode):
    """The same slopes frame after frame (the new residual is already orthogonal to the last
    directions, the Gram matrix becomes nearly singular, the solve continues past 50
    iterations): no breakdown, the same dropped columns as the oracle, and coefficients within
    10 times the oracle's own deviation when its slopes are perturbed by a relative 1e-14 (the
    size of the summation-order differences one FP64 application of M accumulates over its
    ~10^2 terms per coefficient; long CG runs amplify them), and at least 1e-10."""
    spec, seq = _small(1)
    spec = spec.copy(recycle_mode=mode)
    sysm = OracleSystem(spec)
    ctx = fw.FewhaContext(spec, device=DEV)
    ref, ref_p = AugmentedReconstructor(sysm), AugmentedReconstructor(sysm)
    s_p = seq[0] * (1 + 1e-14 * np.random.default_rng(0).standard_normal(seq[0].shape))
    info = ctx.new_info()
    for t in range(6):
        c_ref, i_ref = ref.solve(seq[0])
        c_pp, _ = ref_p.solve(s_p)
        c = host(ctx.fewha_solve_aug(dev(seq[0]), info=info))
        gi = fw.decode_info(info)
        assert gi["flags"] == 0 and gi["dropped"] == i_ref["dropped"], (t, gi, i_ref)
        assert rel(c, c_ref) <= max(1e-10, 10 * rel(c_pp, c_ref)), (t, rel(c, c_ref), rel(c_pp, c_ref))
    assert ctx.breakdown_reports == []


def test_broken_instance_leaves_the_rest_of_a_batch_alone():
    """In a batch of three, instance 1 gets a non-finite frame: it is skipped, and instances 0
    and 2 give the bits they give alone; the batch reports the breakdown once."""
    specs, seqs = [], []
    for i, seed in enumerate((5, 6, 7)):
        sp = synth.config_tiny(seed=3 + i)
        sp.max_iter, sp.recycle_k = 4, 6
        specs.append(sp)
        rng = np.random.default_rng(seed)
        base = rng.standard_normal(synth.n_slopes(sp))
        seqs.append(np.stack([base + 0.1 * t * rng.standard_normal(base.size) for t in range(4)]))
    seqs[1][1, :] = np.nan
    batch = fw.FewhaContext(specs, device=DEV)
    solos = [fw.FewhaContext(sp, device=DEV) for sp in specs]
    info = batch.new_info()
    so = batch.slope_offsets
    co = batch.coeff_offsets
    for t in range(4):
        s = np.concatenate([sq[t] for sq in seqs])
        c = host(batch.fewha_solve_aug(dev(s), info=info))
        infos = fw.decode_info(info)
        for i in range(3):
            ci = host(solos[i].fewha_solve_aug(dev(seqs[i][t])))
            np.testing.assert_array_equal(c[co[i]:co[i + 1]], ci)
            assert infos[i]["flags"] == (9 if (i == 1 and t == 1) else 0), (t, i, infos[i])
    assert len(batch.breakdown_reports) == 1 and len(solos[1].breakdown_reports) == 1
    assert so[-1] == sum(synth.n_slopes(sp) for sp in specs)
