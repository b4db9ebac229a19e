"""Pins of the closed-loop oracle (Alg. 3: pseudo-open-loop slopes, fitting, gain control)
against closed forms, adjoint identities, dense least squares, SciPy's CG and the closed-form
solution of the gain recurrences.  CPU only."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle import AugmentedReconstructor, OracleSystem
from oracle.closed_loop import ClosedLoopOracle, DmSpec, bilinear_zero, bilinear_zero_T, gain_update


def _act_coords(d):
    t = (np.arange(d.n) - (d.n - 1) / 2.0) * d.spacing
    return np.meshgrid(d.origin_x + t, d.origin_y + t, indexing="xy")


def tiny_loop(fit_iter=4, closed=True):
    spec = synth.config_tiny()
    rec = AugmentedReconstructor(OracleSystem(spec))
    # two DMs at the layer heights, larger than the footprints, coarser than the layer grids
    dms = [DmSpec(0.0, 9, 0.6), DmSpec(6000.0, 11, 0.6, origin_x=0.3, origin_y=-0.2)]
    dirs = [(0.0, 0.0), (15 * synth.ARCSEC, -10 * synth.ARCSEC), (-12 * synth.ARCSEC, 8 * synth.ARCSEC)]
    return ClosedLoopOracle(rec, dms, gain=0.4, closed=closed, fit_dirs=dirs, n_pts=9, fit_iter=fit_iter)


def test_bilinear_zero_is_exact_inside_and_fades_to_zero_outside():
    n = 6
    A, B = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    img = 0.3 * A - 0.7 * B + 2.0
    u, v = np.array([0.25, 3.5, 4.9]), np.array([1.5, 0.1, 4.5])
    np.testing.assert_allclose(bilinear_zero(img, u, v), 0.3 * u - 0.7 * v + 2.0, rtol=1e-14)
    # half a cell beyond the last column: half of the edge value (the next node is zero)
    np.testing.assert_allclose(bilinear_zero(img, np.array([n - 0.5]), np.array([2.0])), 0.5 * img[2, n - 1])
    assert bilinear_zero(img, np.array([-1.5]), np.array([2.0]))[0] == 0.0
    # adjoint in the node values
    rng = np.random.default_rng(0)
    uu, vv = rng.uniform(-1.2, n + 0.2, 50), rng.uniform(-1.2, n + 0.2, 50)
    x, y = rng.standard_normal((n, n)), rng.standard_normal(50)
    assert abs(bilinear_zero(x, uu, vv) @ y - (x * bilinear_zero_T(y, uu, vv, n)).sum()) < 1e-12


def test_dm_to_sensor_map_affine_closed_form_and_adjoint():
    """DM surfaces a_d = alpha_d x + beta_d y + c_d (inside their grids) seen by sensor g give
    s^x = sum_d alpha_d (1 - h_d/H_g) d_s and s^y likewise on active subapertures; and H has the
    separately written adjoint H^T to 1e-12."""
    loop = tiny_loop()
    coef = [(0.4, -0.3, 1.0), (-0.2, 0.5, -2.0)]
    a = np.concatenate([(al * X + be * Y + c0).ravel() for (al, be, c0), d in zip(coef, loop.dms)
                        for X, Y in [_act_coords(d)]])
    s = loop.dm_slopes(a)
    for g, (w, sg) in enumerate(zip(loop.sys.wfs, loop.sys.split_slopes(s))):
        ns, m = w.n_sub, w.mask.ravel()
        sc = [1.0 - d.height / w.lgs_height if w.lgs_height > 0 else 1.0 for d in loop.dms]
        np.testing.assert_allclose(sg[:ns * ns][m], sum(c[0] * f for c, f in zip(coef, sc)) * w.subap, rtol=1e-12)
        np.testing.assert_allclose(sg[ns * ns:][m], sum(c[1] * f for c, f in zip(coef, sc)) * w.subap, rtol=1e-12)
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal(loop.n_act), rng.standard_normal(loop.sys.S)
    assert abs(loop.dm_slopes(x) @ y - x @ loop.dm_slopes_T(y)) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(y) * 10


def test_pseudo_open_loop_slopes_recover_the_open_loop_measurement():
    """Closed-loop slopes are the open-loop ones minus H a^(i-1) (two-step delay); the frame
    reconstructs from s + H a^(i-1), i.e. from the open-loop slopes (compared with an open-loop
    reconstructor fed the open-loop slopes directly)."""
    loop = tiny_loop(closed=True)
    ref = AugmentedReconstructor(loop.sys)
    rng = np.random.default_rng(2)
    s_open = rng.standard_normal(loop.sys.S)
    loop.a_prev = rng.standard_normal(loop.n_act)
    loop.a_cur = rng.standard_normal(loop.n_act)
    s_closed = s_open - loop.dm_slopes(loop.a_prev)
    loop.step(s_closed)
    c_ref, _ = ref.solve(s_open)
    np.testing.assert_allclose(loop.rec.c, c_ref, rtol=0, atol=1e-12 * np.abs(c_ref).max())


def test_direct_fitting_samples_the_layers_at_the_actuators():
    """Layers at the DM altitudes: an affine layer function gives commands equal to that
    function at the actuator positions (bilinear interpolation is exact on it)."""
    spec = synth.config_tiny()
    sysm = OracleSystem(spec)
    dms = [DmSpec(l.height, 7, 0.5, l.origin_x + 0.1, l.origin_y - 0.05) for l in spec.layers]
    loop = ClosedLoopOracle(AugmentedReconstructor(sysm), dms, fit_iter=0)
    coef = [(0.3, -0.8, 1.0), (-1.1, 0.4, -2.0)]
    phis = []
    for lay, (al, be, c0) in zip(spec.layers, coef):
        t = (np.arange(lay.n) - (lay.n - 1) / 2.0) * lay.spacing
        X, Y = np.meshgrid(lay.origin_x + t, lay.origin_y + t, indexing="xy")
        phis.append(al * X + be * Y + c0)
    # coefficients whose nodal fields are these layers (W^-1 c = phi <=> c = d DWT phi)
    from oracle import warm_start_correction
    c = warm_start_correction(sysm, np.concatenate([p.ravel() for p in phis]))
    a = loop.fit(c)
    want = np.concatenate([(al * X + be * Y + c0).ravel() for (al, be, c0), d in zip(coef, dms)
                           for X, Y in [_act_coords(d)]])
    np.testing.assert_allclose(a, want, rtol=1e-10, atol=1e-10)


def test_cg_fitting_matches_scipy_and_converges_to_least_squares():
    """The fitting's normal-equation operator is symmetric; 4 unpreconditioned iterations from a
    start vector equal SciPy's CG; many iterations reach the dense least-squares commands."""
    loop = tiny_loop(fit_iter=4)
    n = loop.n_act
    A = np.stack([loop.fit_normal(e) for e in np.eye(n)], axis=1)
    assert np.abs(A - A.T).max() <= 1e-12 * np.abs(A).max()
    rng = np.random.default_rng(3)
    c = rng.standard_normal(loop.sys.N)
    b = loop.fit_rhs(loop.sys.W_inv(c))
    x0 = rng.standard_normal(n)
    loop.a_fit = x0.copy()
    xs = []
    spla.cg(A, b, x0=x0.copy(), maxiter=4, rtol=1e-300, atol=0.0, callback=lambda xk: xs.append(xk.copy()))
    np.testing.assert_allclose(loop.fit(c), xs[-1], rtol=0, atol=1e-9 * np.abs(xs[-1]).max())
    # dense least squares of the stacked projections (pupil points x directions)
    P = np.concatenate([np.stack([loop._dms_at(e, th) for e in np.eye(n)], axis=1) for th in loop.fit_dirs])
    y = np.concatenate([loop._layers_at(loop.sys.W_inv(c), th) for th in loop.fit_dirs])
    x_ls = np.linalg.lstsq(P, y, rcond=None)[0]
    loop.fit_iter, loop.a_fit = 400, np.zeros(n)
    np.testing.assert_allclose(P @ loop.fit(c), P @ x_ls, atol=1e-8 * np.abs(P @ x_ls).max())


@pytest.mark.parametrize("closed", [True, False])
def test_gain_control_matches_closed_form_recurrence(closed):
    """A constant fitted shape a~ from rest: open loop a_n = (1 - (1 - g)^n) a~; closed loop
    a_{n+1} = a_n + g (a~ - a_{n-1}), whose solution is a~ + A l1^n + B l2^n with l the roots of
    l^2 - l + g = 0 (complex for g = 0.4: a damped oscillation onto a~)."""
    g, target = 0.4, np.array([1.5, -0.5])
    a_prev, a_cur = np.zeros(2), np.zeros(2)
    l1, l2 = (1 + np.sqrt(complex(1 - 4 * g))) / 2, (1 - np.sqrt(complex(1 - 4 * g))) / 2
    # a_0 = a_{-1} = 0: A + B = -1 (in units of a~) and A l1^-1 + B l2^-1 = -1
    M = np.array([[1, 1], [1 / l1, 1 / l2]])
    A_, B_ = np.linalg.solve(M, np.array([-1, -1], dtype=complex))
    for n in range(1, 40):
        a_next = gain_update(a_prev, a_cur, target, g, closed)
        a_prev, a_cur = a_cur, a_next
        want = (1 - (1 - g) ** n) if not closed else (1 + A_ * l1 ** n + B_ * l2 ** n).real
        np.testing.assert_allclose(a_cur, want * target, rtol=1e-12, atol=1e-14)


def test_closed_loop_on_a_static_atmosphere_reaches_the_map_fitted_commands():
    """A static atmosphere under closed-loop control (pseudo-open-loop slopes, gain 0.4):
    repeated frames converge the reconstruction to the exact MAP solution c* of the open-loop
    slopes (dense solve), and the commands to its fitted shape F W^-1 c* -- the fixed point of
    the gain recurrence."""
    loop = tiny_loop(fit_iter=200)
    sysm = loop.sys
    rng = np.random.default_rng(4)
    s_open = rng.standard_normal(sysm.S)
    cstar = np.linalg.solve(sysm.dense_M(), sysm.rhs(s_open))
    for _ in range(60):
        loop.step(s_open - loop.dm_slopes(loop.a_prev))
    a_star = loop.fit(cstar)
    np.testing.assert_allclose(loop.a_cur, a_star, rtol=0, atol=1e-6 * np.abs(a_star).max())
