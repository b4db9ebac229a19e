"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics
(published filter values, closed forms, library routines, invariants, brute force on
tiny grids).  CPU only."""
import json
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synth
from oracle.fewha_oracle import (OracleSystem, AugmentedReconstructor, aug_pcg, db3_filters, dwt1,
                                 dwt2, exact_solution, idwt1, idwt2, pcg)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- wavelets (Sec. 3)

def test_db3_matches_published_table():
    ref = json.load(open(os.path.join(GOLDEN, "db3_scaling_filter.json")))["h"]
    h, _ = db3_filters()
    np.testing.assert_allclose(h, ref, rtol=0, atol=5e-16)


def test_db3_orthonormality_and_vanishing_moments():
    h, g = db3_filters()
    assert abs(h.sum() - np.sqrt(2)) < 1e-15
    assert abs((h ** 2).sum() - 1) < 1e-15
    for m in (1, 2):
        assert abs(h[: 6 - 2 * m] @ h[2 * m:]) < 1e-15
    k = np.arange(6.0)
    for p in range(3):
        assert abs(g @ k ** p) < 1e-13
    assert abs(g @ k ** 3) > 1e-3          # exactly three vanishing moments


def test_dwt1_equals_library_correlation():
    """One periodic analysis level = correlation with the filter on the periodic extension,
    downsampled by two (numpy.correlate)."""
    h, g = db3_filters()
    x = np.random.default_rng(0).standard_normal(32)
    ext = np.concatenate([x, x[:5]])
    a = np.correlate(ext, h, "valid")[::2][:16]
    d = np.correlate(ext, g, "valid")[::2][:16]
    np.testing.assert_allclose(dwt1(x), np.concatenate([a, d]), atol=1e-14)


@pytest.mark.parametrize("n", [8, 16])
def test_dwt2_dense_orthogonal_all_levels(n):
    for lv in range(1, int(np.log2(n)) + 1):
        Wd = np.stack([dwt2(e.reshape(n, n), lv).ravel() for e in np.eye(n * n)], axis=1)
        np.testing.assert_allclose(Wd.T @ Wd, np.eye(n * n), atol=1e-14)
        Wi = np.stack([idwt2(e.reshape(n, n), lv).ravel() for e in np.eye(n * n)], axis=1)
        np.testing.assert_allclose(Wi, Wd.T, atol=1e-15)


def test_dwt2_constant_and_quadratic_images():
    n, lv, v = 32, 3, 1.7
    c = dwt2(np.full((n, n), v), lv)
    m = n >> lv
    np.testing.assert_allclose(c[:m, :m], v * 2 ** lv, rtol=1e-14)
    c[:m, :m] = 0
    assert np.abs(c).max() < 1e-13
    # quadratic image: all first-level detail coefficients vanish away from the wrap seam
    y, x = np.mgrid[0:n, 0:n].astype(float)
    img = 0.3 * x ** 2 - 0.2 * x * y + 0.1 * y ** 2 + x - 2 * y + 3
    c1 = dwt2(img, 1)
    h2 = n // 2
    inner = slice(0, h2 - 3)             # filters starting at 2k with 2k + 5 < n
    assert np.abs(c1[inner, h2:][:, inner]).max() < 1e-9 * np.abs(img).max()
    assert np.abs(c1[h2:, inner][inner, :]).max() < 1e-9 * np.abs(img).max()


def test_idwt1_is_inverse_and_transpose():
    x = np.random.default_rng(1).standard_normal((3, 16))
    np.testing.assert_allclose(idwt1(dwt1(x)), x, atol=1e-14)
    y = np.random.default_rng(2).standard_normal((3, 16))
    assert abs((dwt1(x) * y).sum() - (x * idwt1(y)).sum()) < 1e-13


# ---------------------------------------------------------------- operators (Sec. 2)

@pytest.fixture(scope="module")
def tiny():
    return OracleSystem(synth.config_tiny())


def test_shack_hartmann_affine_closed_form(tiny):
    """Bilinear SH model on an affine wavefront a x + b y + c: s^x = a d_s, s^y = b d_s on
    active subapertures (this also pins the reading of the garbled y-slope formula)."""
    for g, w in enumerate(tiny.wfs):
        x = synth.wfs_node_coords(w)
        X, Y = np.meshgrid(x, x, indexing="xy")
        a, b, c = 0.7, -1.3, 5.0
        s = tiny.shack_hartmann(a * X + b * Y + c, g)
        ns = w.n_sub
        m = w.mask.ravel()
        np.testing.assert_allclose(s[:ns * ns][m], a * w.subap, rtol=1e-13)
        np.testing.assert_allclose(s[ns * ns:][m], b * w.subap, rtol=1e-13)
        assert np.all(s[:ns * ns][~m] == 0) and np.all(s[ns * ns:][~m] == 0)
        # pure x-tilt gives no y-slope and vice versa; constants give nothing
        assert np.abs(tiny.shack_hartmann(X, g)[ns * ns:]).max() < 1e-14
        assert np.abs(tiny.shack_hartmann(Y, g)[:ns * ns]).max() < 1e-14
        assert np.abs(tiny.shack_hartmann(np.full_like(X, 3.0), g)).max() == 0


def _layer_coords(lay):
    t = (np.arange(lay.n) - (lay.n - 1) / 2.0) * lay.spacing
    return lay.origin_x + t, lay.origin_y + t


def test_propagation_affine_closed_form(tiny):
    """Bilinear layers reproduce affine functions exactly: P_g sums them at the cone-scaled,
    shifted points (1 - h/H) x + theta h (NGS: H = infinity)."""
    coef = [(0.3, -0.8, 1.0), (-1.1, 0.4, -2.0)]
    phis = []
    for lay, (a, b, c) in zip(tiny.layers, coef):
        xs, ys = _layer_coords(lay)
        X, Y = np.meshgrid(xs, ys, indexing="xy")
        phis.append(a * X + b * Y + c)
    for g, w in enumerate(tiny.wfs):
        x = synth.wfs_node_coords(w)
        X, Y = np.meshgrid(x, x, indexing="xy")
        want = np.zeros_like(X)
        for lay, (a, b, c) in zip(tiny.layers, coef):
            sc = 1 - lay.height / w.lgs_height if w.lgs_height > 0 else 1.0
            want += a * (sc * X + w.theta_x * lay.height) + b * (sc * Y + w.theta_y * lay.height) + c
        np.testing.assert_allclose(tiny.propagate(phis, g), want, rtol=1e-12, atol=1e-12)


def test_propagation_bilinear_product_exact(tiny):
    """x*y is bilinear on every cell, so the interpolation is exact for it as well."""
    lay = tiny.layers[1]
    xs, ys = _layer_coords(lay)
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    phis = [np.zeros((tiny.layers[0].n,) * 2), X * Y]
    w = tiny.wfs[1]
    x = synth.wfs_node_coords(w)
    Xw, Yw = np.meshgrid(x, x, indexing="xy")
    sc = 1 - lay.height / w.lgs_height
    want = (sc * Xw + w.theta_x * lay.height) * (sc * Yw + w.theta_y * lay.height)
    np.testing.assert_allclose(tiny.propagate(phis, 1), want, rtol=1e-12, atol=1e-12)


def test_propagation_reduces_to_sampling_and_ngs_limit():
    spec = synth.config_tiny()
    lay = spec.layers[0]                  # ground layer: align the grid with WFS 0's nodes
    w = spec.wfs[0]
    lay.spacing = w.subap
    lay.origin_x = lay.origin_y = 0.5 * w.subap * ((lay.n - 1) % 2)
    sysm = OracleSystem(spec)
    rng = np.random.default_rng(5)
    phis = [rng.standard_normal((l.n, l.n)) for l in spec.layers]
    phis[1][:] = 0
    off = (lay.n - 1) / 2.0 - w.n_sub / 2.0 + ((lay.n - 1) % 2) * -0.5
    i0 = int(round(off))
    np.testing.assert_allclose(sysm.propagate(phis, 0),
                               phis[0][i0:i0 + w.n_sub + 1, i0:i0 + w.n_sub + 1], atol=1e-14)
    # an LGS at (numerically) infinite height is an NGS
    spec2 = synth.config_tiny()
    spec3 = synth.config_tiny()
    spec2.wfs[1].lgs_height = 0.0
    spec3.wfs[1].lgs_height = 1e30
    spec3.layers = spec2.layers
    s2, s3 = OracleSystem(spec2), OracleSystem(spec3)
    phis = [rng.standard_normal((l.n, l.n)) for l in spec2.layers]
    np.testing.assert_allclose(s2.propagate(phis, 1), s3.propagate(phis, 1), atol=1e-12)


def test_footprint_outside_grid_is_rejected():
    spec = synth.config_tiny()
    spec.layers[1].spacing *= 0.5
    with pytest.raises(ValueError):
        OracleSystem(spec)


def test_adjoints(tiny):
    rng = np.random.default_rng(7)
    for g, w in enumerate(tiny.wfs):
        phis = [rng.standard_normal((l.n, l.n)) for l in tiny.layers]
        psi = rng.standard_normal((w.n_sub + 1, w.n_sub + 1))
        lhs = (tiny.propagate(phis, g) * psi).sum()
        rhs = sum((p * q).sum() for p, q in zip(phis, tiny.propagate_T(psi, g)))
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
        s = rng.standard_normal(2 * w.n_sub ** 2)
        lhs = tiny.shack_hartmann(psi, g) @ s
        rhs = (psi * tiny.shack_hartmann_T(s, g)).sum()
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    x = rng.standard_normal(tiny.N)
    s = rng.standard_normal(tiny.S)
    lhs = tiny.A(tiny.W_inv(x)) @ s
    rhs = x @ tiny.W_invT(tiny.A_T(s))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_M_symmetric_positive_definite_and_composition(tiny):
    Md = tiny.dense_M()
    assert np.abs(Md - Md.T).max() <= 1e-13 * np.abs(Md).max()
    np.linalg.cholesky(Md)
    assert np.linalg.eigvalsh(Md).min() > 0
    A = tiny.dense_A()                     # columns A W^-1 e_i, from the pinned forward operators
    D = tiny.prior()
    want = A.T @ (tiny.weights[:, None] * A) + tiny.alpha * np.diag(D)
    np.testing.assert_allclose(Md, want, atol=1e-12 * np.abs(Md).max())
    s = np.random.default_rng(3).standard_normal(tiny.S)
    np.testing.assert_allclose(tiny.rhs(s), A.T @ (tiny.weights * s), atol=1e-12 * np.abs(A).max())


@pytest.mark.parametrize("cfg", [dict(), dict(n=32, levels=5, n_sub=12, seed=9)])
def test_exact_diagonal_matches_dense(cfg):
    sysm = OracleSystem(synth.config_tiny(**cfg))
    Md = sysm.dense_M()
    np.testing.assert_allclose(sysm.diag_M(), np.diag(Md), rtol=1e-12)


def test_prior_spectral_shape():
    """D is the inverse von Karman spectrum at the band frequency: finest level at the grid
    Nyquist frequency 1/(2 d); one level coarser halves f; D scales as r0^(5/3)/gamma."""
    spec = synth.config_tiny(n=32, levels=4)
    sysm = OracleSystem(spec)
    D = sysm.split_layers(sysm.prior())
    for lay, Dl in zip(spec.layers, D):
        L0, r0 = spec.L0, spec.r0
        vk = lambda f: 0.023 * (r0 / lay.weight ** 0.6) ** (-5 / 3) * (f ** 2 + L0 ** -2) ** (-11 / 6)
        f1 = 1.0 / (2 * lay.spacing)
        np.testing.assert_allclose(Dl[0, 31], 1 / vk(f1), rtol=1e-12)          # finest detail
        np.testing.assert_allclose(Dl[5, 3], 1 / vk(f1 / 4), rtol=1e-12)       # level 3 detail
        np.testing.assert_allclose(Dl[9, 3], 1 / vk(f1 / 2), rtol=1e-12)       # level 2 detail
        np.testing.assert_allclose(Dl[0, 0], 1 / vk(f1 / 8), rtol=1e-12)       # approximation
    spec2 = synth.config_tiny(n=32, levels=4)
    spec2.r0 *= 2
    np.testing.assert_allclose(OracleSystem(spec2).prior(), sysm.prior() * 2 ** (5 / 3), rtol=1e-13)


# ---------------------------------------------------------------- PCG (Sec. 4, Alg. 1)

@pytest.fixture(scope="module")
def tiny_dense(tiny):
    Md = tiny.dense_M()
    s = np.random.default_rng(11).standard_normal(tiny.S)
    b = tiny.rhs(s)
    return Md, b, 1.0 / np.diag(Md)


def test_pcg_matches_scipy_iterates(tiny, tiny_dense):
    Md, b, Jinv = tiny_dense
    iters = []
    pcg(lambda x: Md @ x, b, np.zeros_like(b), Jinv, 8, callback=lambda c, r: iters.append(c.copy()))
    ref = []
    spla.cg(Md, b, x0=np.zeros_like(b), maxiter=8, rtol=1e-300, atol=0.0,
            M=spla.LinearOperator(Md.shape, matvec=lambda v: Jinv * v), callback=lambda xk: ref.append(xk.copy()))
    assert len(ref) == 8
    for a, r in zip(iters, ref):
        np.testing.assert_allclose(a, r, rtol=0, atol=1e-10 * np.abs(r).max())


def test_pcg_krylov_optimality_and_convergence(tiny, tiny_dense):
    Md, b, Jinv = tiny_dense
    cstar = np.linalg.solve(Md, b)
    np.testing.assert_allclose(exact_solution(tiny, b), cstar, rtol=1e-10, atol=1e-12 * np.abs(cstar).max())
    k = 6
    c, r, dirs = pcg(lambda x: Md @ x, b, np.zeros_like(b), Jinv, k)
    # c_k minimises the M-norm error over K_k(J^-1 M, J^-1 b)
    K = [Jinv * b]
    for _ in range(k - 1):
        K.append(Jinv * (Md @ K[-1]))
    V, _ = np.linalg.qr(np.stack(K, 1))
    y = np.linalg.solve(V.T @ Md @ V, V.T @ b)
    np.testing.assert_allclose(c, V @ y, atol=1e-9 * np.abs(c).max())
    # M-conjugate directions (P^T M P diagonal), J^-1-orthogonal residuals
    P = np.stack([p for p, _, _ in dirs], 1)
    G = P.T @ Md @ P
    assert np.abs(G - np.diag(np.diag(G))).max() <= 1e-8 * np.abs(np.diag(G)).max()
    # run to convergence (kappa(J^-1 M) ~ 90 here): the exact solution
    cN, _, _ = pcg(lambda x: Md @ x, b, np.zeros_like(b), Jinv, 150)
    np.testing.assert_allclose(cN, cstar, atol=1e-10 * np.abs(cstar).max())


def test_pcg_energy_decreases(tiny, tiny_dense):
    Md, b, Jinv = tiny_dense
    f = []
    pcg(lambda x: Md @ x, b, np.zeros_like(b), Jinv, 10, callback=lambda c, r: f.append(0.5 * c @ Md @ c - b @ c))
    assert all(f[i + 1] < f[i] for i in range(len(f) - 1))


# ---------------------------------------------------------------- augmented PCG (Alg. 2)

def _two_rhs(tiny, tiny_dense, m):
    Md, b, Jinv = tiny_dense
    s2 = np.random.default_rng(12).standard_normal(tiny.S)
    b2 = b + 0.3 * tiny.rhs(s2)
    _, _, dirs = pcg(lambda x: Md @ x, b, np.zeros_like(b), Jinv, m)
    U = [p for p, _, _ in dirs]
    Q = [q for _, q, _ in dirs]
    gam = [g for _, _, g in dirs]
    return Md, b2, Jinv, U, Q, gam


@pytest.mark.parametrize("mode", ["paper", "galerkin"])
def test_aug_initial_residual_and_direction_conditions(tiny, tiny_dense, mode):
    Md, b2, Jinv, U, Q, gam = _two_rhs(tiny, tiny_dense, 6)
    c0 = np.zeros_like(b2)
    # zero iterations expose the Galerkin step; one iteration exposes p_0 and the next p
    c, r, _, _ = aug_pcg(lambda x: Md @ x, c0, b2.copy(), Jinv, U, Q, gam, 0, mode)
    Um = np.stack(U, 1)
    assert np.abs(Um.T @ r).max() <= 1e-10 * np.linalg.norm(r) * np.abs(Um).max()
    # the Galerkin step is the M-norm minimiser over c0 + span(U)
    cstar = np.linalg.solve(Md, b2)
    y = np.linalg.solve(Um.T @ Md @ Um, Um.T @ Md @ cstar)
    np.testing.assert_allclose(c, Um @ y, atol=1e-9 * np.abs(c).max())
    _, _, new, _ = aug_pcg(lambda x: Md @ x, c0, b2.copy(), Jinv, U, Q, gam, 2, mode)
    p0, p1 = new[0][0], new[1][0]
    assert np.abs(Um.T @ Md @ p0).max() <= 1e-9 * np.abs(p0 @ Md @ p0)
    assert abs(p1 @ Md @ U[-1]) <= 1e-9 * np.sqrt(abs(p1 @ Md @ p1) * abs(U[-1] @ Md @ U[-1]))


@pytest.mark.parametrize("mode", ["paper", "galerkin"])
def test_augcg_optimality_brute_force(tiny, tiny_dense, mode):
    """With U the complete direction set of a PCG solve (same M, other right-hand side),
    augmented PCG iterate k minimises the M-norm error over c0 + span(U) + span(z_0..z_k-1)
    (Petrov-Galerkin condition 3).  The printed (p_m, p_m) denominator fails this."""
    Md, b2, Jinv, U, Q, gam = _two_rhs(tiny, tiny_dense, 5)
    cstar = np.linalg.solve(Md, b2)
    c0 = np.zeros_like(b2)
    for k in (1, 2, 4, 6):
        c, r, new, _ = aug_pcg(lambda x: Md @ x, c0, b2.copy(), Jinv, U, Q, gam, k, mode)
        Z = []
        cc, rr, _, _ = aug_pcg(lambda x: Md @ x, c0, b2.copy(), Jinv, U, Q, gam, 0, mode)
        Z.append(Jinv * rr)
        for j in range(1, k):
            _, rj, _, _ = aug_pcg(lambda x: Md @ x, c0, b2.copy(), Jinv, U, Q, gam, j, mode)
            Z.append(Jinv * rj)
        V, _ = np.linalg.qr(np.stack(U + Z, 1))
        y = np.linalg.solve(V.T @ Md @ V, V.T @ Md @ (cstar - c0))
        best = c0 + V @ y
        errM = lambda v: np.sqrt((v - cstar) @ Md @ (v - cstar))
        assert errM(c) <= errM(best) * (1 + 1e-6) + 1e-12 * np.sqrt(cstar @ Md @ cstar)


def test_typo_denominator_breaks_conjugacy(tiny, tiny_dense):
    """Negative control for the (p_m, q_m) reading: with (p_m, p_m) the new direction is not
    M-conjugate to p_m."""
    Md, b2, Jinv, U, Q, gam = _two_rhs(tiny, tiny_dense, 5)
    wrong = [float(u @ u) for u in U]        # plant (p_j, p_j) in place of (p_j, q_j) in the loop
    r0 = b2.copy()
    c, r, new, _ = aug_pcg(lambda x: Md @ x, np.zeros_like(b2), r0, Jinv, U, Q, gam[:-1] + [wrong[-1]], 2, "galerkin")
    p1 = new[1][0]
    assert abs(p1 @ Md @ U[-1]) > 1e-6 * np.sqrt(abs(p1 @ Md @ p1) * abs(U[-1] @ Md @ U[-1]))


def test_aug_error_bound(tiny, tiny_dense):
    """||c_k - c||_M <= 2 ||c_0 - c||_M ((sqrt(kappa)-1)/(sqrt(kappa)+1))^k with kappa the
    condition number of the projected, preconditioned operator on range(H) (Sec. 6.2)."""
    Md, b2, Jinv, U, Q, gam = _two_rhs(tiny, tiny_dense, 4)
    cstar = np.linalg.solve(Md, b2)
    Um = np.stack(U, 1)
    H = np.eye(tiny.N) - Um @ np.linalg.solve(Um.T @ Md @ Um, (Md @ Um).T)
    Jh = np.diag(np.sqrt(Jinv))
    Kmat = Jh @ H.T @ Md @ H @ Jh
    ev = np.linalg.eigvalsh(0.5 * (Kmat + Kmat.T))
    ev = ev[ev > 1e-9 * ev.max()]
    kappa = ev.max() / ev.min()
    rho = (np.sqrt(kappa) - 1) / (np.sqrt(kappa) + 1)
    errM = lambda v: np.sqrt((v - cstar) @ Md @ (v - cstar))
    cg0, _, _, _ = aug_pcg(lambda x: Md @ x, np.zeros_like(b2), b2.copy(), Jinv, U, Q, gam, 0, "galerkin")
    for k in (1, 3, 6, 10):
        c, _, _, _ = aug_pcg(lambda x: Md @ x, np.zeros_like(b2), b2.copy(), Jinv, U, Q, gam, k, "galerkin")
        assert errM(c) <= 2 * errM(cg0) * rho ** k * (1 + 1e-9)


# ---------------------------------------------------------------- Alg. 3 frame sequence

def test_frame_sequence_residual_identity_and_store():
    spec = synth.config_tiny()
    spec.max_iter, spec.recycle_k = 3, 5
    sysm = OracleSystem(spec)
    rec = AugmentedReconstructor(sysm)
    rng = np.random.default_rng(21)
    base = rng.standard_normal(sysm.S)
    for t in range(6):
        s = base + 0.05 * t * rng.standard_normal(sysm.S)
        c_prev, r_prev, bp = rec.c.copy(), rec.r.copy(), rec.b_prev.copy()
        c, info = rec.solve(s)
        b = sysm.rhs(s)
        if t > 0:
            # (b_new - b_old) + r_old equals b_new - M c_old up to drift
            lhs = (b - bp) + r_prev
            np.testing.assert_allclose(lhs, b - sysm.apply_M(c_prev), atol=1e-10 * np.abs(b).max())
            assert info["recycle_used"] == min(5, 3 * t)
        # the carried residual is the true residual of the returned iterate
        np.testing.assert_allclose(rec.r, b - sysm.apply_M(c), atol=1e-9 * np.abs(b).max())
        assert len(rec.store) == min(5, 3 * (t + 1))


def test_recycling_reduces_error_on_slowly_varying_sequence():
    """Recycling lowers the error at equal iterations on a frozen-flow sequence (the
    qualitative claim of Sec. 6 / Sec. 7.1)."""
    spec = synth.config_small()
    seq = synth.make_sequence(spec, 5, seed=4)
    sysm = OracleSystem(spec)
    D = sysm.prior()
    Jinv = 1.0 / sysm.diag_M(D)
    aug = AugmentedReconstructor(sysm, Jinv=Jinv, max_iter=5, k=5)
    plain = AugmentedReconstructor(sysm, Jinv=Jinv, max_iter=5, k=0)
    for t in range(5):
        ca, ia = aug.solve(seq[t])
        cp, ip = plain.solve(seq[t])
    assert ia["rel_res"] < ip["rel_res"]


@pytest.mark.parametrize("mode", ["galerkin", "paper"])
def test_zero_frame_then_frames_match_plain_pcg(mode):
    """An all-zero slope frame has b = 0: its solution is exactly c = 0 with residual 0, and
    the directions it stores are zero vectors ((p, M p) = 0).  A zero direction contributes
    nothing, so the next frame (r = b - 0 + 0 = b) equals Alg. 1 from c = 0: the iterates of
    SciPy's preconditioned CG."""
    spec = synth.config_tiny()
    spec.max_iter, spec.recycle_k = 4, 3
    sysm = OracleSystem(spec)
    Md = sysm.dense_M()
    rec = AugmentedReconstructor(sysm, Jinv=1.0 / np.diag(Md), mode=mode)
    c0, i0 = rec.solve(np.zeros(sysm.S))
    np.testing.assert_array_equal(c0, 0.0)
    assert i0["rel_res"] == 0.0 and all(g == 0.0 for _, _, g in rec.store)
    s = np.random.default_rng(31).standard_normal(sysm.S)
    c1, i1 = rec.solve(s)
    b = sysm.rhs(s)
    ref = []
    spla.cg(Md, b, x0=np.zeros_like(b), maxiter=4, rtol=1e-300, atol=0.0,
            M=spla.LinearOperator(Md.shape, matvec=lambda v: v / np.diag(Md)),
            callback=lambda xk: ref.append(xk.copy()))
    assert np.all(np.isfinite(c1)) and i1["recycle_used"] == 3
    np.testing.assert_allclose(c1, ref[-1], rtol=0, atol=1e-10 * np.abs(ref[-1]).max())


# ---------------------------------------------------------------- wavelet scaling delta_l (Sec. 3)

def test_wavelet_scaling_makes_coefficients_l2_normalised():
    """delta_l = d_l: the coefficients are the L2-normalised representation of the layer, i.e.
    the nodal quadrature of the squared layer function, sum_i phi_i^2 d_l^2, equals ||c_l||^2
    on every layer (layers of different spacing and level count), and W^-T is the adjoint of
    W^-1 under the plain Euclidean inner products (so W^-T x = DWT x / d_l as well)."""
    sysm = OracleSystem(synth.config_mixed())
    assert len({round(l.spacing, 12) for l in sysm.layers}) > 1
    rng = np.random.default_rng(41)
    c = rng.standard_normal(sysm.N)
    for cl, phi, lay in zip(sysm.split_layers(c), sysm.W_inv(c), sysm.layers):
        np.testing.assert_allclose((phi ** 2).sum() * lay.spacing ** 2, (cl ** 2).sum(), rtol=1e-12)
    x = rng.standard_normal(sysm.N)
    lhs = sum((p * xl).sum() for p, xl in zip(sysm.W_inv(c), sysm.split_layers(x)))
    np.testing.assert_allclose(lhs, c @ sysm.W_invT(sysm.split_layers(x)), rtol=1e-12)


# ---------------------------------------------------------------- project_all (Alg. 2, all of U)

def _non_conjugate_U(tiny, tiny_dense):
    """Recycled directions that are not mutually M-conjugate: three PCG directions of each of
    two different right-hand sides (as a ring spanning two frames holds)."""
    Md, b, Jinv = tiny_dense
    rng = np.random.default_rng(13)
    U, Q, gam = [], [], []
    for bb in (b, tiny.rhs(rng.standard_normal(tiny.S))):
        _, _, dirs = pcg(lambda x: Md @ x, bb, np.zeros_like(bb), Jinv, 3)
        U += [p for p, _, _ in dirs]
        Q += [q for _, q, _ in dirs]
        gam += [g for _, _, g in dirs]
    Um = np.stack(U, 1)
    G = Um.T @ Md @ Um
    assert np.abs(G - np.diag(np.diag(G))).max() > 1e-3 * np.abs(np.diag(G)).max()   # really not conjugate
    b2 = tiny.rhs(rng.standard_normal(tiny.S))
    return Md, b2, Jinv, U, Q, gam


def test_project_all_keeps_every_direction_conjugate_to_all_of_U(tiny, tiny_dense):
    """With project_all every new direction is M-conjugate to every recycled direction (the
    deflated-CG form of condition 1 of Alg. 2), also when U is not a conjugate set; projecting
    against the most recent direction only does not give this (negative control)."""
    Md, b2, Jinv, U, Q, gam = _non_conjugate_U(tiny, tiny_dense)
    Um = np.stack(U, 1)
    _, _, new, _ = aug_pcg(lambda x: Md @ x, np.zeros_like(b2), b2.copy(), Jinv, U, Q, gam, 5, "galerkin",
                           project_all=True)
    for p, _, _ in new:
        scale = np.linalg.norm(Md @ p) * np.abs(Um).max() * np.sqrt(tiny.N)
        assert np.abs(Um.T @ Md @ p).max() <= 1e-9 * scale
    _, _, new_last, _ = aug_pcg(lambda x: Md @ x, np.zeros_like(b2), b2.copy(), Jinv, U, Q, gam, 5, "galerkin",
                                project_all=False)
    p = new_last[2][0]
    scale = np.linalg.norm(Md @ p) * np.abs(Um).max() * np.sqrt(tiny.N)
    assert np.abs(Um[:, :-1].T @ Md @ p).max() > 1e-6 * scale


def test_project_all_iterate_is_energy_optimal_over_U_plus_krylov(tiny, tiny_dense):
    """Deflated CG: with every direction projected against all of U, iterate k minimises the
    M-norm error over c0 + span(U) + span(z_0, ..., z_{k-1}) for any recycled set U (here not
    M-conjugate), by dense projection (brute force)."""
    Md, b2, Jinv, U, Q, gam = _non_conjugate_U(tiny, tiny_dense)
    cstar = np.linalg.solve(Md, b2)
    c0 = np.zeros_like(b2)
    errM = lambda v: np.sqrt((v - cstar) @ Md @ (v - cstar))
    for k in (1, 2, 4):
        c, _, _, _ = aug_pcg(lambda x: Md @ x, c0, b2.copy(), Jinv, U, Q, gam, k, "galerkin", project_all=True)
        Z = []
        for j in range(k):
            _, rj, _, _ = aug_pcg(lambda x: Md @ x, c0, b2.copy(), Jinv, U, Q, gam, j, "galerkin", project_all=True)
            Z.append(Jinv * rj)
        V, _ = np.linalg.qr(np.stack(U + Z, 1))
        best = c0 + V @ np.linalg.solve(V.T @ Md @ V, V.T @ Md @ (cstar - c0))
        assert errM(c) <= errM(best) * (1 + 1e-7) + 1e-12 * np.sqrt(cstar @ Md @ cstar), k


# ---------------------------------------------------------------- tolerance stop

def test_rel_tol_stop_is_first_crossing_of_scipy_cg(tiny, tiny_dense):
    """Without recycled directions the tolerance-stopped solve stops at the first iteration k
    with ||b - M c_k|| <= tol ||b|| of SciPy's preconditioned CG, and returns that iterate; a
    tolerance never met runs the full count."""
    Md, b, Jinv = tiny_dense
    xs = []
    spla.cg(Md, b, x0=np.zeros_like(b), maxiter=40, rtol=1e-300, atol=0.0,
            M=spla.LinearOperator(Md.shape, matvec=lambda v: Jinv * v), callback=lambda xk: xs.append(xk.copy()))
    res = np.array([np.linalg.norm(b - Md @ x) for x in xs]) / np.linalg.norm(b)
    checked = 0
    for k_first in (3, 7, 12):
        tol = np.sqrt(res[k_first - 1] * res[k_first - 2]) if res[k_first - 1] < res[k_first - 2] else None
        if tol is None or np.any(res[:k_first - 1] <= tol):
            continue
        c, r, _, info = aug_pcg(lambda x: Md @ x, np.zeros_like(b), b.copy(), Jinv, [], [], [], 40,
                                rel_tol=tol, b_norm=np.linalg.norm(b))
        assert info["iters"] == k_first
        np.testing.assert_allclose(c, xs[k_first - 1], atol=1e-10 * np.abs(xs[k_first - 1]).max())
        checked += 1
    assert checked >= 2
    _, _, _, info = aug_pcg(lambda x: Md @ x, np.zeros_like(b), b.copy(), Jinv, [], [], [], 5,
                            rel_tol=1e-12, b_norm=np.linalg.norm(b))
    assert info["iters"] == 5


@pytest.mark.parametrize("mode", ["paper", "galerkin"])
def test_rel_tol_stop_with_recycling_is_first_crossing(tiny, tiny_dense, mode):
    """With recycled directions: the stop is the smallest fixed count whose final residual meets
    the tolerance, and the iterate equals that fixed-count run's."""
    Md, b2, Jinv, U, Q, gam = _two_rhs(tiny, tiny_dense, 4)
    bn = np.linalg.norm(b2)
    runs = [aug_pcg(lambda x: Md @ x, np.zeros_like(b2), b2.copy(), Jinv, U, Q, gam, k, mode)
            for k in range(1, 16)]
    res = np.array([np.linalg.norm(r) / bn for _, r, _, _ in runs])
    k_first = 6
    tol = np.sqrt(res[k_first - 1] * res[k_first - 2])
    assert res[k_first - 1] <= tol < res[k_first - 2]
    first = 1 + int(np.argmax(res <= tol))
    c, _, _, info = aug_pcg(lambda x: Md @ x, np.zeros_like(b2), b2.copy(), Jinv, U, Q, gam, 40, mode,
                            rel_tol=tol, b_norm=bn)
    assert info["iters"] == first
    np.testing.assert_allclose(c, runs[first - 1][0], rtol=0, atol=1e-12 * np.abs(c).max())


# ---------------------------------------------------------------- learned warm start step

def test_warm_start_step_is_exact_line_search(tiny, tiny_dense):
    """tau minimises the energy 1/2 c^T M c - b^T c along e (a dense 1-D minimisation), and a
    correction pointing uphill is not taken."""
    from scipy.optimize import minimize_scalar
    from oracle import warm_start_step
    Md, b, _ = tiny_dense
    rng = np.random.default_rng(51)
    c = np.linalg.solve(Md, b) + 0.1 * rng.standard_normal(tiny.N)
    r = b - Md @ c
    e = np.linalg.solve(Md, r) + 0.3 * rng.standard_normal(tiny.N)
    f = lambda t: 0.5 * (c + t * e) @ Md @ (c + t * e) - b @ (c + t * e)
    c1, r1, tau = warm_start_step(lambda x: Md @ x, c, r, e)
    t_ref = minimize_scalar(f, bracket=(0.0, 1.0), tol=1e-12).x
    assert tau > 0
    np.testing.assert_allclose(tau, t_ref, rtol=1e-6)
    np.testing.assert_allclose(r1, b - Md @ c1, atol=1e-10 * np.abs(b).max())
    c2, r2, tau2 = warm_start_step(lambda x: Md @ x, c, r, -e)
    assert tau2 == 0.0 and np.array_equal(c2, c) and np.array_equal(r2, r)
    assert minimize_scalar(f, bounds=(-10.0, 0.0), method="bounded").x < 0   # the minimum lies behind


def test_warm_start_correction_is_the_inverse_of_W_inv():
    """e = W d is the coefficient vector whose nodal field is d: W^-1 e = d on every layer."""
    from oracle import warm_start_correction
    sysm = OracleSystem(synth.config_mixed())
    d = np.random.default_rng(52).standard_normal(sysm.N)
    e = warm_start_correction(sysm, d)
    np.testing.assert_allclose(np.concatenate([p.ravel() for p in sysm.W_inv(e)]), d, atol=1e-12 * np.abs(d).max())


def test_warm_start_inputs_columns():
    """Columns: the nodal fields of c and of J^-1 r over their scales, then h / 20 km and gamma
    of each node's layer."""
    from oracle import warm_start_correction, warm_start_inputs
    sysm = OracleSystem(synth.config_mixed())
    rng = np.random.default_rng(53)
    phi, psi = rng.standard_normal(sysm.N), rng.standard_normal(sysm.N)
    Jinv = rng.uniform(0.5, 2.0, sysm.N)
    c = warm_start_correction(sysm, phi)
    r = warm_start_correction(sysm, psi) / Jinv
    x = warm_start_inputs(sysm, c, r, Jinv, 2.0, 4.0)
    np.testing.assert_allclose(x[:, 0], phi / 2.0, atol=1e-12)
    np.testing.assert_allclose(x[:, 1], psi / 4.0, atol=1e-12)
    for l, lay in enumerate(sysm.layers):
        sl = slice(sysm.coff[l], sysm.coff[l + 1])
        assert np.all(x[sl, 2] == lay.height / 20000.0) and np.all(x[sl, 3] == lay.weight)


def test_warm_start_frames_zero_and_exact_correction():
    """A zero correction leaves the frames those of plain augmented PCG; the exact correction
    (the nodal field of c* - c) makes the frame start at the solution (tau = 1)."""
    spec = synth.config_tiny()
    spec.max_iter, spec.recycle_k = 3, 4
    sysm = OracleSystem(spec)
    rng = np.random.default_rng(54)
    base = rng.standard_normal(sysm.S)
    plain, warm = AugmentedReconstructor(sysm), AugmentedReconstructor(sysm)
    for t in range(3):
        s = base + 0.1 * t * rng.standard_normal(sysm.S)
        cp, _ = plain.solve(s)
        cw, iw = warm.solve(s, correction=lambda x: np.zeros(sysm.N))
        np.testing.assert_array_equal(cw, cp)
        assert iw["tau"] == 0.0
    Md = sysm.dense_M()
    exact = AugmentedReconstructor(sysm)
    exact.solve(base)
    s = base + 0.2 * rng.standard_normal(sysm.S)
    cstar = np.linalg.solve(Md, sysm.rhs(s))
    field = np.concatenate([p.ravel() for p in sysm.W_inv(cstar - exact.c)])
    snap = AugmentedReconstructor(sysm)
    snap.c = exact.c.copy()
    snap.b_prev, snap.r, snap.first = exact.b_prev.copy(), exact.r.copy(), False
    snap.max_iter = 0
    c0, info = snap.solve(s, correction=lambda x: field / 3.0, scales=(1.0, 1.0, 3.0))
    np.testing.assert_allclose(info["tau"], 1.0, rtol=1e-8)
    np.testing.assert_allclose(c0, cstar, atol=1e-8 * np.abs(cstar).max())


# ---------------------------------------------------------------- breakdown (paper silent)

@pytest.mark.filterwarnings("ignore::RuntimeWarning")
@pytest.mark.parametrize("bad", [np.nan, np.inf])
def test_nonfinite_slopes_frame_is_skipped_and_next_frame_is_plain_pcg(bad):
    """A frame with non-finite slopes returns the previous coefficients unchanged (flags bits 0
    and 3) and stores null directions; the carried residual stays b - M c, so the next frame is
    Alg. 1 from the previous coefficients: SciPy's preconditioned CG from x0 = c."""
    spec = synth.config_tiny()
    spec.max_iter, spec.recycle_k = 4, 3
    sysm = OracleSystem(spec)
    Md = sysm.dense_M()
    Jinv = 1.0 / np.diag(Md)
    rng = np.random.default_rng(61)
    rec = AugmentedReconstructor(sysm, Jinv=Jinv)
    for t in range(2):
        c_prev, _ = rec.solve(rng.standard_normal(sysm.S))
    s_bad = rng.standard_normal(sysm.S)
    s_bad[5] = bad
    c_bad, info = rec.solve(s_bad)
    np.testing.assert_array_equal(c_bad, c_prev)
    assert info["flags"] == 9 and np.isnan(info["rel_res"])
    s = rng.standard_normal(sysm.S)
    c1, i1 = rec.solve(s)
    b = sysm.rhs(s)
    np.testing.assert_allclose(rec.r, b - Md @ c1, atol=1e-10 * np.abs(b).max())
    ref = []
    spla.cg(Md, b, x0=c_prev.copy(), maxiter=4, rtol=1e-300, atol=0.0,
            M=spla.LinearOperator(Md.shape, matvec=lambda v: Jinv * v), callback=lambda xk: ref.append(xk.copy()))
    assert i1["flags"] == 0
    np.testing.assert_allclose(c1, ref[-1], rtol=0, atol=1e-10 * np.abs(ref[-1]).max())


@pytest.mark.filterwarnings("ignore::RuntimeWarning")
def test_nonfinite_first_frame_keeps_residual_consistent():
    """A non-finite first frame leaves r = b_prev - M c, so the next residual update gives the
    true residual b - M c of the carried coefficients."""
    spec = synth.config_tiny()
    spec.max_iter, spec.recycle_k = 3, 3
    sysm = OracleSystem(spec)
    rec = AugmentedReconstructor(sysm)
    rng = np.random.default_rng(62)
    rec.c = rng.standard_normal(sysm.N)
    s_bad = np.full(sysm.S, np.nan)
    c0, info = rec.solve(s_bad)
    assert info["flags"] == 9 and not rec.first
    s = rng.standard_normal(sysm.S)
    b = sysm.rhs(s)
    np.testing.assert_allclose((b - rec.b_prev) + rec.r, b - sysm.apply_M(c0), atol=1e-12 * np.abs(b).max())


def test_breakdown_mid_frame_keeps_last_finite_iterate(tiny, tiny_dense):
    """A planted non-positive curvature at the third operator application (an indefinite
    operator; the oracle is where such a fault is planted): the frame keeps the iterate of the
    second iteration (SciPy's CG after two steps), flags the breakdown, and stores null
    directions from there on."""
    Md, b, Jinv = tiny_dense
    calls = [0]

    def bad_apply(x):
        calls[0] += 1
        return Md @ x if calls[0] < 3 else -(Md @ x)

    c, r, new, info = aug_pcg(bad_apply, np.zeros_like(b), b.copy(), Jinv, [], [], [], 6)
    ref = []
    spla.cg(Md, b, x0=np.zeros_like(b), maxiter=2, rtol=1e-300, atol=0.0,
            M=spla.LinearOperator(Md.shape, matvec=lambda v: Jinv * v), callback=lambda xk: ref.append(xk.copy()))
    assert info["flags"] == 1 and len(new) == 6
    np.testing.assert_allclose(c, ref[-1], rtol=0, atol=1e-10 * np.abs(ref[-1]).max())
    np.testing.assert_allclose(r, b - Md @ c, atol=1e-10 * np.abs(b).max())
    assert all(g == 0.0 and not p.any() for p, _, g in new[2:]) and new[1][2] > 0


def test_identical_consecutive_frames_converge_monotonically(tiny, tiny_dense):
    """Repeating one frame (singular-looking Gram: the new residual is already orthogonal to
    the last directions) continues the same solve: the M-norm error never grows from frame to
    frame and reaches the exact solution."""
    Md, _, Jinv = tiny_dense
    rec = AugmentedReconstructor(tiny, Jinv=Jinv, max_iter=3, k=6)
    s = np.random.default_rng(63).standard_normal(tiny.S)
    cstar = np.linalg.solve(Md, tiny.rhs(s))
    errM = lambda v: np.sqrt((v - cstar) @ Md @ (v - cstar))
    errs = []
    for t in range(40):
        c, info = rec.solve(s)
        assert info["flags"] == 0 and np.all(np.isfinite(c))
        errs.append(errM(c))
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-9) + 1e-14 for i in range(len(errs) - 1))
    assert errs[-1] <= 1e-8 * np.sqrt(cstar @ Md @ cstar)


def test_modified_jacobi_level_map_from_basis_support():
    """The frequency-weighted Jacobi weights land on the coefficients of the right wavelet
    level, identified independently of the level bookkeeping: the synthesised basis function
    of a level-l coefficient of periodic db3 spans 5 (2^l - 1) + 1 samples per direction, and
    the scaling (approximation) functions are the only ones of the coarsest level with a
    nonzero sum.  With distinct weights 2^j the returned J^-1 times diag(M) is 2^-j."""
    spec = synth.config_tiny(n=64, levels=3, n_sub=8)
    spec.layers = spec.layers[:1]
    sysm = OracleSystem(spec)
    weights = [2.0 ** j for j in range(11)]
    ratio = sysm.modified_jacobi(weights) * sysm.diag_M()
    n, L = 64, 3
    for i in range(0, n * n, 7):
        e = np.zeros(sysm.N)
        e[i] = 1.0
        f = sysm.W_inv(e)[0]
        sy, sx = int(np.any(f != 0, axis=1).sum()), int(np.any(f != 0, axis=0).sum())
        lev = {6: 1, 16: 2, 36: 3}[max(sy, sx)]
        j = L if (lev == L and abs(f.sum()) > 1e-9) else lev - 1
        assert abs(ratio[i] - 2.0 ** -j) < 1e-12, (i, lev, ratio[i])


def test_modified_jacobi_unit_weights_is_jacobi():
    sysm = OracleSystem(synth.config_tiny())
    np.testing.assert_allclose(sysm.modified_jacobi([1.0] * 11), 1.0 / sysm.diag_M(), rtol=1e-15)
