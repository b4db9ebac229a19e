"""The laser-guide-star noise model on the GPU (2x2 C_eta^-1 blocks from radial spot
elongation, tip/tilt filtering of the LGS data) against the oracle, which assembles the same
C_eta^-1 from the same per-subaperture entries with its own projection formula."""
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


def dev(x, dtype=np.float64):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dtype)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def _tiny(tt=True, elongation=2.5, frames=6):
    spec = synth.config_tiny()
    for w in spec.wfs:
        if w.lgs_height > 0:
            w.elongation, w.tt_filter, w.tt_jitter = elongation, tt, 3.0
    seq = synth.make_sequence(spec, frames, seed=11)
    return spec, seq


@pytest.mark.parametrize("tt, elongation", [(True, 2.5), (False, 2.5), (True, 0.0)])
def test_operator_rhs_and_jacobi_match_oracle_fp64(tt, elongation):
    spec, seq = _tiny(tt, elongation)
    sysm = OracleSystem(spec)
    ctx = fw.FewhaContext(spec, device=DEV)
    x = np.random.default_rng(1).standard_normal(sysm.N)
    assert rel(host(ctx.fewha_apply_A(dev(x))), sysm.apply_M(x)) <= 1e-12
    assert rel(host(ctx.fewha_rhs(dev(seq[1]))), sysm.rhs(seq[1])) <= 1e-12
    jinv = ctx.fewha_get_vector(1).double().cpu().numpy()
    assert rel(jinv, 1.0 / sysm.diag_M()) <= 1e-12


def test_frames_match_oracle_fp64():
    spec, seq = _tiny()
    ctx = fw.FewhaContext(spec, device=DEV)
    ref = AugmentedReconstructor(OracleSystem(spec))
    for t in range(len(seq)):
        c = host(ctx.fewha_solve_aug(dev(seq[t])))
        c_ref, _ = ref.solve(seq[t])
        assert rel(c, c_ref) <= 1e-10, (t, rel(c, c_ref))


def test_rhs_ignores_a_filtered_sensors_tip_tilt():
    spec, seq = _tiny()
    sysm = OracleSystem(spec)
    ctx = fw.FewhaContext(spec, device=DEV)
    g = next(i for i, w in enumerate(spec.wfs) if w.lgs_height > 0)
    n2 = spec.wfs[g].n_sub ** 2
    act = np.flatnonzero(spec.wfs[g].mask.ravel())
    s2 = seq[2].copy()
    s2[sysm.soff[g] + act] += 0.37
    s2[sysm.soff[g] + n2 + act] -= 0.81
    b1, b2 = host(ctx.fewha_rhs(dev(seq[2]))), host(ctx.fewha_rhs(dev(s2)))
    assert rel(b2, b1) <= 1e-12


def test_noalloc_entry_matches_with_the_filter():
    spec, _ = _tiny()
    ctx = fw.FewhaContext(spec, device=DEV)
    x = dev(np.random.default_rng(2).standard_normal(ctx.N))
    y = host(ctx.fewha_apply_A(x))
    y2 = torch.empty_like(x)
    ctx.fewha_apply_A_noalloc(x, y2)
    assert np.array_equal(host(y2), y)


def test_elt_lgs_noise_frames_fp32():
    """The full ELT system with elongated LGS spots, LGS tip/tilt jitter and its filter, FP32
    operator: four frames against the FP64 oracle within the split-precision bar."""
    spec = synth.config_elt_lgs_noise(precision="fp32")
    seq = synth.make_sequence(spec, 4, seed=9).astype(np.float32)
    ctx = fw.FewhaContext(spec, device=DEV)
    ref = AugmentedReconstructor(OracleSystem(spec))
    for t in range(4):
        c = host(ctx.fewha_solve_aug(dev(seq[t], np.float32)))
        c_ref, _ = ref.solve(seq[t].astype(np.float64))
        assert rel(c, c_ref) <= 5e-5, (t, rel(c, c_ref))
