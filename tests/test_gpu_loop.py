"""The closed-loop wrapper (Alg. 3) through the C ABI against the closed-loop oracle: the
DM-to-sensor map, both fitting forms, and whole loop sequences (pseudo-open-loop slopes, frame
solve, fitting, gain control) in closed and open loop."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth
from oracle import AugmentedReconstructor, OracleSystem
from oracle.closed_loop import ClosedLoopOracle, DmSpec
import paper_2011_06842_amd as fw

pytestmark = [pytest.mark.gpu]

DEV = "cuda:0"
ARC = synth.ARCSEC


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def dev(x, dtype=np.float64):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dtype)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


DMS = [(0.0, 9, 0.6), (6000.0, 11, 0.6, 0.3, -0.2)]
DIRS = [(0.0, 0.0), (15 * ARC, -10 * ARC), (-12 * ARC, 8 * ARC)]


def tiny_pair(fit_iter=4, closed=True, precision="fp64"):
    spec = synth.config_tiny()
    spec.precision = precision
    sysm = OracleSystem(spec)
    ctx = fw.FewhaContext(spec, device=DEV)
    loop = fw.LoopContext(ctx, DMS, gain=0.4, closed=closed, fit_iter=fit_iter, dirs=DIRS, n_pts=9,
                          pupil_d=spec.D, obstruction=spec.obstruction)
    ref = ClosedLoopOracle(AugmentedReconstructor(sysm), [DmSpec(*d) for d in DMS], gain=0.4, closed=closed,
                           fit_dirs=DIRS, n_pts=9, fit_iter=fit_iter)
    return spec, sysm, ctx, loop, ref


def test_dm_to_sensor_map_matches_oracle():
    spec, sysm, ctx, loop, ref = tiny_pair()
    a = np.random.default_rng(0).standard_normal(loop.n_act)
    assert rel(host(loop.piece(fw.LOOP_DM_SLOPES, dev(a))), ref.dm_slopes(a)) <= 1e-12


@pytest.mark.parametrize("fit_iter", [4, 12])
def test_cg_fitting_matches_oracle_from_a_given_start(fit_iter):
    spec, sysm, ctx, loop, ref = tiny_pair(fit_iter=fit_iter)
    rng = np.random.default_rng(1)
    c = rng.standard_normal(sysm.N)
    x0 = rng.standard_normal(loop.n_act)
    loop.set_commands(fit=dev(x0))
    ref.a_fit = x0.copy()
    assert rel(host(loop.piece(fw.LOOP_FIT, dev(c))), ref.fit(c)) <= 1e-10
    np.testing.assert_array_equal(host(loop.get_commands(2)), x0)       # the piece leaves the loop's state


def test_direct_fitting_matches_oracle():
    spec = synth.config_tiny()
    sysm = OracleSystem(spec)
    dms = [(l.height, 7, 0.5, l.origin_x + 0.1, l.origin_y - 0.05) for l in spec.layers]
    ctx = fw.FewhaContext(spec, device=DEV)
    loop = fw.LoopContext(ctx, dms, fit_iter=0)
    ref = ClosedLoopOracle(AugmentedReconstructor(sysm), [DmSpec(*d) for d in dms], fit_iter=0)
    c = np.random.default_rng(2).standard_normal(sysm.N)
    assert rel(host(loop.piece(fw.LOOP_FIT, dev(c))), ref.fit(c)) <= 1e-12


def test_direct_fitting_rejects_dms_off_the_layer_altitudes():
    spec = synth.config_tiny()
    ctx = fw.FewhaContext(spec, device=DEV)
    with pytest.raises(fw.FewhaError, match="altitude"):
        fw.LoopContext(ctx, [(0.0, 7, 0.5), (5000.0, 7, 0.5)], fit_iter=0)


@pytest.mark.parametrize("closed, fit_iter", [(True, 4), (False, 4), (True, 0)])
def test_loop_sequence_matches_oracle_fp64(closed, fit_iter):
    """Eight frames of Alg. 3 from rest on a slowly varying sequence: the commands (and the
    frame's coefficients) match the oracle at 1e-10 in FP64."""
    if fit_iter == 0:
        spec = synth.config_tiny()
        sysm = OracleSystem(spec)
        dms = [(l.height, l.n, l.spacing, l.origin_x, l.origin_y) for l in spec.layers]
        ctx = fw.FewhaContext(spec, device=DEV)
        loop = fw.LoopContext(ctx, dms, gain=0.4, closed=closed, fit_iter=0)
        ref = ClosedLoopOracle(AugmentedReconstructor(sysm), [DmSpec(*d) for d in dms], gain=0.4, closed=closed,
                               fit_iter=0)
    else:
        spec, sysm, ctx, loop, ref = tiny_pair(fit_iter=fit_iter, closed=closed)
    rng = np.random.default_rng(3)
    base = rng.standard_normal(sysm.S)
    info = ctx.new_info()
    for t in range(8):
        s = base + 0.1 * t * rng.standard_normal(sysm.S)
        if closed:   # what the sensors see behind the DMs (two-step delay): open-loop minus H a^(i-1)
            s = s - ref.dm_slopes(ref.a_prev)
        a = host(loop.step(dev(s), info=info))
        a_ref, i_ref = ref.step(s)
        assert rel(a, a_ref) <= 1e-10, (t, rel(a, a_ref))
        gi = fw.decode_info(info)
        assert gi["flags"] == 0 and gi["iters"] == i_ref["iters"]
    np.testing.assert_allclose(host(loop.get_commands(0)), ref.a_prev, rtol=0, atol=1e-10 * np.abs(ref.a_prev).max())


def test_elt_mcao_closed_loop_fp32():
    """The full ELT system (6 LGS + 3 low-order NGS), FP32 operator, three DMs of the MCAO system
    table (85 x 85 at 0 m with 0.5 m spacing, 47 x 47 at 4 km and 53 x 53 at 12.7 km with 1 m),
    least-squares fitting with 4 CG iterations over the 5 x 5 evaluation grid of the asterism
    figure (+-60 arcsec in steps of 30), gain 0.4, closed loop: four frames against the FP64
    oracle; the frame solves are within the split-precision bar (5e-5), the commands within
    1e-4 (a second FP32 stage, the fitting, follows)."""
    spec = synth.config_elt_full(precision="fp32")
    seq = synth.make_sequence(spec, 4, seed=9).astype(np.float32).astype(np.float64)
    sysm = OracleSystem(spec)
    dms, dirs = synth.elt_mcao_dms(), synth.mcao_fit_directions()
    ctx = fw.FewhaContext(spec, device=DEV)
    loop = fw.LoopContext(ctx, dms, gain=0.4, closed=True, fit_iter=4, dirs=dirs, n_pts=40, pupil_d=spec.D,
                          obstruction=spec.obstruction)
    ref = ClosedLoopOracle(AugmentedReconstructor(sysm), [DmSpec(*d) for d in dms], gain=0.4, closed=True,
                           fit_dirs=dirs, n_pts=40, fit_iter=4)
    for t in range(4):
        s = (seq[t] - ref.dm_slopes(ref.a_prev)).astype(np.float32).astype(np.float64)
        a = host(loop.step(dev(s, np.float32)))
        a_ref, _ = ref.step(s)
        assert rel(a, a_ref) <= 1e-4, (t, rel(a, a_ref))
