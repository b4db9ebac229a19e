"""CPU pins of the oracle's inverse noise covariance with the laser-guide-star noise model
(the paper leaves its form unstated; the readings are a 2x2 block per subaperture from the
radial spot elongation, and for a tip/tilt-filtered sensor C^-1 = B - B T (T^T B T)^-1 T^T B,
T the sensor's global tip and tilt slope patterns).  The pins do not re-derive the oracle's
formulas: they check the block against a matrix inverse of the simulator's covariance, the
projection's defining properties, the right-hand side's invariance to a sensor's tip/tilt,
and the separable diagonal against a brute-force assembly."""
import numpy as np

import synth
from oracle import OracleSystem


def _tiny_lgs(tt=True, elongation=2.5):
    spec = synth.config_tiny()
    for w in spec.wfs:
        if w.lgs_height > 0:
            w.elongation, w.tt_filter, w.tt_jitter = elongation, tt, 3.0
    seq = synth.make_sequence(spec, 2, seed=11)
    return spec, seq


def _lgs_index(spec):
    return next(g for g, w in enumerate(spec.wfs) if w.lgs_height > 0)


def test_elongation_block_is_the_inverse_covariance():
    spec, _ = _tiny_lgs()
    w = spec.wfs[_lgs_index(spec)]
    ex, ey, k = synth.atmosphere.SlopeSimulator.elongation_geometry(w)
    n2 = w.n_sub ** 2
    for i in np.flatnonzero(w.mask.ravel()):
        e = np.array([ex[i], ey[i]])
        cov = w.sigma ** 2 * (np.eye(2) + (k[i] - 1.0) * np.outer(e, e))
        B = np.array([[w.weight[i], w.cross_weight[i]], [w.cross_weight[i], w.weight[n2 + i]]])
        np.testing.assert_allclose(B, np.linalg.inv(cov), rtol=1e-12, atol=1e-12 / w.sigma ** 2)
    assert np.abs(w.cross_weight).max() > 0


def test_filtered_sensor_is_blind_to_its_tip_tilt():
    spec, _ = _tiny_lgs()
    sysm = OracleSystem(spec)
    g = _lgs_index(spec)
    w = spec.wfs[g]
    n2 = w.n_sub ** 2
    act = w.mask.ravel()
    for comp in (0, 1):
        s = np.zeros(sysm.S)
        s[sysm.soff[g] + comp * n2 + np.flatnonzero(act)] = 1.0
        out = sysm.apply_Cinv(s)[sysm.soff[g]:sysm.soff[g + 1]]
        assert np.abs(out).max() < 1e-12 * np.abs(w.weight).max()


def test_inverse_covariance_is_symmetric_and_psd():
    spec, _ = _tiny_lgs()
    sysm = OracleSystem(spec)
    rng = np.random.default_rng(0)
    for _ in range(5):
        a, b = rng.standard_normal(sysm.S), rng.standard_normal(sysm.S)
        ab, ba = sysm.apply_Cinv(a) @ b, a @ sysm.apply_Cinv(b)
        assert abs(ab - ba) <= 1e-12 * (abs(ab) + abs(ba))
        assert sysm.apply_Cinv(a) @ a >= -1e-12 * np.abs(a).sum() * np.abs(sysm.weights).max()


def test_plain_sensors_keep_diagonal_weights():
    spec, seq = _tiny_lgs(tt=False, elongation=0.0)
    sysm = OracleSystem(spec)
    s = seq[1]
    np.testing.assert_allclose(sysm.apply_Cinv(s), sysm.weights * s, rtol=1e-15, atol=0)


def test_right_hand_side_invariant_to_lgs_tip_tilt():
    spec, seq = _tiny_lgs()
    sysm = OracleSystem(spec)
    g = _lgs_index(spec)
    n2 = spec.wfs[g].n_sub ** 2
    act = spec.wfs[g].mask.ravel()
    s2 = seq[1].copy()
    s2[sysm.soff[g] + np.flatnonzero(act)] += 0.37
    s2[sysm.soff[g] + n2 + np.flatnonzero(act)] -= 0.81
    b1, b2 = sysm.rhs(seq[1]), sysm.rhs(s2)
    assert np.linalg.norm(b1 - b2) <= 1e-12 * np.linalg.norm(b1)


def test_diagonal_with_cross_weights_matches_brute_force():
    """diag(M) from the separable formula (cross term included, the filter's rank-2 term left
    out of the preconditioner) against e_i^T M_B e_i of the assembled operator with the
    block-diagonal part of C^-1."""
    spec, _ = _tiny_lgs()
    sysm = OracleSystem(spec)
    d = sysm.diag_M()
    sysm.tt = [False] * len(sysm.tt)           # the block-diagonal part B
    D = sysm.prior()
    brute = np.array([sysm.apply_M(e, D)[i] for i, e in enumerate(np.eye(sysm.N))])
    np.testing.assert_allclose(d, brute, rtol=1e-10)
