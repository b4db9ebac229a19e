"""Plain FP64 CPU oracle of augmented FEWHA (Ramlau & Stadler, "An augmented wavelet
reconstructor for atmospheric tomography").

TEST INFRASTRUCTURE ONLY: imported by tests, the smoke check and the CPU-baseline leg of
the benchmark; never by the GPU library.  Everything is float64 NumPy written for a
reader to check against the paper: no blocking, no fusion, no reordering beyond what
the cited definition states.

Readings taken where the paper is silent, garbled or inconsistent (all listed in the
design notes as well):

* Shack-Hartmann y-slope (Sec. 2): the printed second term subtracts the wrong node;
  it is read as the mirror image of the x-slope,
  ``s^y_ij = ((phi_{i+1,j} - phi_{i,j}) + (phi_{i+1,j+1} - phi_{i,j+1})) / 2``.
* Wavelets (Sec. 3): periodic orthonormal Daubechies-3 (6 taps), 2-D Mallat pyramid
  (rows, then columns, on the top-left block), scaling constant ``delta_l = d_l``
  (layer grid spacing), so ``W^-1 c = DWT^T c / d_l`` and ``W^-T x = DWT x / d_l``.
* Prior (Sec. 3, ``D`` diagonal in the frequency domain): inverse von Karman spectrum
  at each coefficient's band frequency ``f = 2^j / (n d_l)`` (``j = J - level``;
  finest level -> ``f = 1/(2 d_l)``; approximation block uses the coarsest level):
  ``D = (f^2 + L0^-2)^(11/6) r0^(5/3) / (0.023 gamma_l)``.
* Noise covariance (Sec. 3): diagonal inverse variances per slope, zero where masked.
* Preconditioner (Sec. 4): the plain Jacobi reading ``J = diag(M)``, computed exactly.
* Alg. 1 starts with ``p_0 = r_0``; read as ``p_0 = z_0 = J^-1 r_0`` (textbook PCG for
  the split-preconditioned system, and what Alg. 2 does).
* Loops "for k = 0, ..., maxIter" (Alg. 1, Alg. 2) perform exactly ``maxIter``
  applications of M (the per-iteration cost times n_iter of the FLOP table).
* Alg. 2, Galerkin loop: ``r`` in sigma_j is the running residual (updated inside the
  loop).  Initial-direction loop: the update is missing its vector and is read as
  ``z_0 -= (z_0, q_j) / (p_j, q_j) * p_j``.  In-loop projection: the denominator
  ``(p_m, p_m)`` is read as ``(p_m, q_m)`` (the only value making the new direction
  M-conjugate to p_m, and the stored inner product of Sec. 7.2).
* Recycle store: the ``k`` most recent stored directions ``(p_j, q_j = M p_j,
  (p_j, q_j))``.  Mode "paper": the Galerkin step and the initial-direction step are the
  sequential single-vector projections of Alg. 2.  Mode "galerkin": both use the full
  k x k Gram matrix ``G = U^T Q`` (upper triangle ``(u_i, q_j)``, i <= j) through a
  Cholesky factorisation that drops columns whose pivot is <= 1e-14 max(diag G).
  In-loop projection is against the most recent stored direction (both modes), or
  against all of U with the Gram solve when ``project_all`` is set (mode "galerkin").
"""
from __future__ import annotations

import numpy as np

# ----------------------------------------------------------------------------------------
# Sec. 3: periodic Daubechies-3 wavelet transform (the map W between the finite element
# and the wavelet domain).
# ----------------------------------------------------------------------------------------


def db3_filters():
    """Orthonormal 6-tap Daubechies scaling filter h (closed form, sum sqrt(2)) and the
    wavelet filter g_m = (-1)^m h_{5-m}."""
    s10 = np.sqrt(10.0)
    r = np.sqrt(5.0 + 2.0 * s10)
    h = np.sqrt(2.0) / 32.0 * np.array([1 + s10 + r, 5 + s10 + 3 * r, 10 - 2 * s10 + 2 * r,
                                         10 - 2 * s10 - 2 * r, 5 + s10 - 3 * r, 1 + s10 - r])
    g = np.array([(-1) ** m * h[5 - m] for m in range(6)])
    return h, g


_H, _G = db3_filters()


def dwt1(x: np.ndarray) -> np.ndarray:
    """One level of periodic analysis along the last axis: output [a | d] with
    a_k = sum_m h_m x_{(2k+m) mod n},  d_k = sum_m g_m x_{(2k+m) mod n}."""
    n = x.shape[-1]
    k = np.arange(n // 2)
    a = np.zeros(x.shape[:-1] + (n // 2,))
    d = np.zeros_like(a)
    for m in range(6):
        xm = x[..., (2 * k + m) % n]
        a += _H[m] * xm
        d += _G[m] * xm
    return np.concatenate([a, d], axis=-1)


def idwt1(y: np.ndarray) -> np.ndarray:
    """Exact transpose (= inverse) of :func:`dwt1` along the last axis."""
    n = y.shape[-1]
    k = np.arange(n // 2)
    a, d = y[..., : n // 2], y[..., n // 2:]
    x = np.zeros(y.shape)
    for m in range(6):
        x[..., (2 * k + m) % n] += _H[m] * a + _G[m] * d   # indices distinct for fixed m
    return x


def dwt2(img: np.ndarray, levels: int) -> np.ndarray:
    """Multi-level 2-D periodic DWT, Mallat layout: each level transforms the rows and
    then the columns of the current top-left approximation block."""
    c = np.array(img, dtype=np.float64, copy=True)
    n = c.shape[0]
    for lev in range(levels):
        m = n >> lev
        blk = dwt1(c[:m, :m])          # rows (x direction)
        blk = dwt1(blk.T).T            # columns (y direction)
        c[:m, :m] = blk
    return c


def idwt2(coef: np.ndarray, levels: int) -> np.ndarray:
    """Transpose (= inverse) of :func:`dwt2`."""
    x = np.array(coef, dtype=np.float64, copy=True)
    n = x.shape[0]
    for lev in reversed(range(levels)):
        m = n >> lev
        blk = idwt1(x[:m, :m].T).T     # columns
        blk = idwt1(blk)               # rows
        x[:m, :m] = blk
    return x


def idwt1_levels(y: np.ndarray, levels: int) -> np.ndarray:
    """Multi-level 1-D synthesis along the last axis (used for separable basis functions)."""
    x = np.array(y, dtype=np.float64, copy=True)
    n = x.shape[-1]
    for lev in reversed(range(levels)):
        m = n >> lev
        x[..., :m] = idwt1(x[..., :m])
    return x


# ----------------------------------------------------------------------------------------
# Sec. 2 / Sec. 3: tomography operator A = (Gamma_g P_g)_g in the finite element domain,
# the prior D, the system operator M (Eq. for M) and the right-hand side b.
# ----------------------------------------------------------------------------------------


class OracleSystem:
    """Discretised MAP system of one AO configuration (a ``synth.SystemSpec``)."""

    def __init__(self, spec):
        self.spec = spec
        self.layers = spec.layers
        self.wfs = spec.wfs
        self.L = len(spec.layers)
        self.G = len(spec.wfs)
        self.coff = np.cumsum([0] + [l.n * l.n for l in spec.layers])
        self.soff = np.cumsum([0] + [2 * w.n_sub * w.n_sub for w in spec.wfs])
        self.N = int(self.coff[-1])
        self.S = int(self.soff[-1])
        self.alpha = float(spec.alpha)
        for w in spec.wfs:
            if w.weight is None:
                raise ValueError("slope weights (inverse noise variances) are not set")
        self.weights = np.concatenate([np.asarray(w.weight, dtype=np.float64) for w in spec.wfs])
        # inverse noise covariance C_eta^-1 per sensor (readings of the LGS noise model, which the
        # paper leaves unstated): a symmetric 2x2 block per subaperture [[wx, wc], [wc, wy]]
        # (diagonal weights and an optional cross term), and for a tip/tilt-filtered sensor
        # B - B T (T^T B T)^-1 T^T B with T the sensor's global tip and tilt slope patterns
        self.cross = [None if getattr(w, "cross_weight", None) is None else np.asarray(w.cross_weight, np.float64)
                      for w in spec.wfs]
        self.tt = [bool(getattr(w, "tt_filter", False)) for w in spec.wfs]
        # 1-D bilinear interpolation data of every (guide star, layer) pair, Sec. 2
        self.interp = {}
        for g, w in enumerate(spec.wfs):
            x = (np.arange(w.n_sub + 1) - w.n_sub / 2.0) * w.subap
            for l, lay in enumerate(spec.layers):
                scale = 1.0 - lay.height / w.lgs_height if w.lgs_height > 0 else 1.0
                ux = (scale * x + w.theta_x * lay.height - lay.origin_x) / lay.spacing + (lay.n - 1) / 2.0
                vy = (scale * x + w.theta_y * lay.height - lay.origin_y) / lay.spacing + (lay.n - 1) / 2.0
                self.interp[g, l] = (self._cell(vy, lay.n), self._cell(ux, lay.n))

    @staticmethod
    def _cell(u: np.ndarray, n: int):
        if np.any(u < 0.0) or np.any(u > n - 1):
            raise ValueError("guide-star footprint leaves the layer grid")
        i0 = np.minimum(np.floor(u), n - 2).astype(np.int64)
        return i0, u - i0

    # --- vector layout helpers ---
    def split_layers(self, x):
        return [x[self.coff[l]:self.coff[l + 1]].reshape(lay.n, lay.n)
                for l, lay in enumerate(self.layers)]

    def split_slopes(self, s):
        return [s[self.soff[g]:self.soff[g + 1]] for g in range(self.G)]

    # --- W^-1 and W^-T (Sec. 3) ---
    def W_inv(self, c):
        return [idwt2(cl, lay.levels) / lay.spacing for cl, lay in zip(self.split_layers(c), self.layers)]

    def W_invT(self, phis):
        return np.concatenate([(dwt2(p, lay.levels) / lay.spacing).ravel()
                               for p, lay in zip(phis, self.layers)])

    # --- P_g (Sec. 2: NGS shift, LGS cone-scaled shift; bilinear layer functions) ---
    def propagate(self, phis, g):
        w = self.wfs[g]
        out = np.zeros((w.n_sub + 1, w.n_sub + 1))
        for l, ph in enumerate(phis):
            (a0, fy), (b0, fx) = self.interp[g, l]
            A, B = a0[:, None], b0[None, :]
            FY, FX = fy[:, None], fx[None, :]
            out += ((1 - FY) * ((1 - FX) * ph[A, B] + FX * ph[A, B + 1])
                    + FY * ((1 - FX) * ph[A + 1, B] + FX * ph[A + 1, B + 1]))
        return out

    def propagate_T(self, psi, g):
        outs = []
        for l, lay in enumerate(self.layers):
            (a0, fy), (b0, fx) = self.interp[g, l]
            A = np.broadcast_to(a0[:, None], psi.shape)
            B = np.broadcast_to(b0[None, :], psi.shape)
            FY, FX = fy[:, None], fx[None, :]
            o = np.zeros((lay.n, lay.n))
            np.add.at(o, (A, B), (1 - FY) * (1 - FX) * psi)
            np.add.at(o, (A, B + 1), (1 - FY) * FX * psi)
            np.add.at(o, (A + 1, B), FY * (1 - FX) * psi)
            np.add.at(o, (A + 1, B + 1), FY * FX * psi)
            outs.append(o)
        return outs

    # --- Gamma_g (Sec. 2, Shack-Hartmann operator on bilinear wavefronts) ---
    def shack_hartmann(self, wf, g):
        m = self.wfs[g].mask
        sx = 0.5 * ((wf[:-1, 1:] - wf[:-1, :-1]) + (wf[1:, 1:] - wf[1:, :-1]))
        sy = 0.5 * ((wf[1:, :-1] - wf[:-1, :-1]) + (wf[1:, 1:] - wf[:-1, 1:]))
        return np.concatenate([np.where(m, sx, 0.0).ravel(), np.where(m, sy, 0.0).ravel()])

    def shack_hartmann_T(self, s, g):
        w = self.wfs[g]
        ns = w.n_sub
        tx = np.where(w.mask, s[: ns * ns].reshape(ns, ns), 0.0)
        ty = np.where(w.mask, s[ns * ns:].reshape(ns, ns), 0.0)
        wf = np.zeros((ns + 1, ns + 1))
        wf[:-1, 1:] += 0.5 * tx
        wf[:-1, :-1] -= 0.5 * tx
        wf[1:, 1:] += 0.5 * tx
        wf[1:, :-1] -= 0.5 * tx
        wf[1:, :-1] += 0.5 * ty
        wf[:-1, :-1] -= 0.5 * ty
        wf[1:, 1:] += 0.5 * ty
        wf[:-1, 1:] -= 0.5 * ty
        return wf

    # --- the tomography operator A and its adjoint ---
    def A(self, phis):
        return np.concatenate([self.shack_hartmann(self.propagate(phis, g), g) for g in range(self.G)])

    def A_T(self, s):
        acc = [np.zeros((lay.n, lay.n)) for lay in self.layers]
        for g, sg in enumerate(self.split_slopes(s)):
            for l, o in enumerate(self.propagate_T(self.shack_hartmann_T(sg, g), g)):
                acc[l] += o
        return acc

    # --- prior D (Sec. 3) ---
    def coefficient_levels(self, lay):
        """Wavelet level (1 = finest) of every coefficient of an n x n Mallat pyramid; the
        approximation block gets the coarsest level."""
        n = lay.n
        idx = np.arange(n)
        mx = np.maximum(idx[:, None], idx[None, :])
        lev = np.full((n, n), lay.levels, dtype=np.int64)
        for l in range(1, lay.levels + 1):
            m = n >> l
            lev[(mx >= m) & (mx < 2 * m)] = l
        return lev

    def prior(self):
        spec = self.spec
        out = []
        for lay in self.layers:
            J = int(round(np.log2(lay.n)))
            j = J - self.coefficient_levels(lay)
            f = 2.0 ** j / (lay.n * lay.spacing)
            d = (f ** 2 + spec.L0 ** -2) ** (11.0 / 6.0) * spec.r0 ** (5.0 / 3.0) / (0.023 * lay.weight)
            out.append(d.ravel())
        return np.concatenate(out)

    # --- M (Eq. for M) and b (definition of the right-hand side) ---
    def apply_Cinv(self, s):
        """C_eta^-1 s.  Inactive subapertures (zero weights) contribute nothing, whatever their
        slope values."""
        out = []
        for g, (w, sg) in enumerate(zip(self.wfs, self.split_slopes(s))):
            n2 = w.n_sub * w.n_sub
            wt = np.asarray(w.weight, np.float64)
            wx, wy = wt[:n2], wt[n2:]
            wc = self.cross[g] if self.cross[g] is not None else np.zeros(n2)
            act = (wx != 0) | (wy != 0)
            sx = np.where(act, sg[:n2], 0.0)
            sy = np.where(act, sg[n2:], 0.0)
            bx = wx * sx + wc * sy
            by = wc * sx + wy * sy
            if self.tt[g]:
                G = np.array([[wx.sum(), wc.sum()], [wc.sum(), wy.sum()]])     # T^T B T
                m = np.linalg.solve(G, np.array([bx.sum(), by.sum()]))        # (T^T B T)^-1 T^T B s
                bx = bx - (wx * m[0] + wc * m[1])                              # - B T m
                by = by - (wc * m[0] + wy * m[1])
            out.append(np.concatenate([bx, by]))
        return np.concatenate(out)

    def apply_M(self, x, D=None):
        D = self.prior() if D is None else D
        s = self.A(self.W_inv(x))
        return self.W_invT(self.A_T(self.apply_Cinv(s))) + self.alpha * D * x

    def rhs(self, s):
        return self.W_invT(self.A_T(self.apply_Cinv(s)))

    # --- exact diag(M) (Jacobi preconditioner, Sec. 4) ---
    def diag_M(self, D=None):
        """diag(M)_i = alpha D_i + || B^1/2 A W^-1 e_i ||^2 with B the block-diagonal part of
        C_eta^-1 (a tip/tilt filter's rank-2 correction is left out of the preconditioner).
        Each 2-D basis function of the Mallat pyramid is an outer product of two 1-D level-l
        functions, bilinear interpolation of a separable function is separable, and so are
        both slope components and their product; the squared norm is then a small matrix
        product per (layer, level, guide star)."""
        D = self.prior() if D is None else D
        out = []
        for l, lay in enumerate(self.layers):
            n = lay.n
            diag = np.zeros((n, n))
            levs = self.coefficient_levels(lay)
            for lev in range(1, lay.levels + 1):
                m2 = n >> (lev - 1)
                B = idwt1_levels(np.eye(n)[:m2], lev).T            # (n, m2) 1-D basis functions
                blk = np.zeros((m2, m2))
                for g, w in enumerate(self.wfs):
                    ns = w.n_sub
                    (a0, fy), (b0, fx) = self.interp[g, l]
                    Iy = np.zeros((ns + 1, n))
                    Iy[np.arange(ns + 1), a0] += 1 - fy
                    Iy[np.arange(ns + 1), a0 + 1] += fy
                    Ix = np.zeros((ns + 1, n))
                    Ix[np.arange(ns + 1), b0] += 1 - fx
                    Ix[np.arange(ns + 1), b0 + 1] += fx
                    Yh, Xh = Iy @ B, Ix @ B
                    Sy, Dy = 0.5 * (Yh[:-1] + Yh[1:]), Yh[1:] - Yh[:-1]
                    Sx, Dx = 0.5 * (Xh[:-1] + Xh[1:]), Xh[1:] - Xh[:-1]
                    wx = w.weight[: ns * ns].reshape(ns, ns)
                    wy = w.weight[ns * ns:].reshape(ns, ns)
                    # s^x_ij = (Yh_i + Yh_i+1)/2 (Xh_j+1 - Xh_j); s^y_ij = (Yh_i+1 - Yh_i)(Xh_j + Xh_j+1)/2
                    blk += (Sy ** 2).T @ wx @ (Dx ** 2) + (Dy ** 2).T @ wy @ (Sx ** 2)
                    if self.cross[g] is not None:   # + 2 wc s^x s^y
                        wc = self.cross[g].reshape(ns, ns)
                        blk += 2.0 * (Sy * Dy).T @ wc @ (Dx * Sx)
                sel = levs[:m2, :m2] == lev
                diag[:m2, :m2][sel] = blk[sel]
            out.append(diag.ravel() / lay.spacing ** 2)
        return np.concatenate(out) + self.alpha * D

    # --- frequency-weighted ("modified") Jacobi preconditioner (Sec. 4) ---
    def modified_jacobi(self, level_weight, D=None):
        """J^-1 of J = diag(w) diag(M): the paper weights the low- and high-frequency parts of
        the Jacobi diagonal differently and gives no weights; here w is level_weight[l - 1] on
        the details of level l (1 = finest) and level_weight[levels] on the scaling
        (approximation) coefficients.  Parity unpinned: only the level bookkeeping and the
        product are checked."""
        d = self.diag_M(D)
        w = []
        for lay in self.layers:
            lev = self.coefficient_levels(lay) - 1
            nc = lay.n >> lay.levels
            lev[:nc, :nc] = lay.levels
            w.append(np.asarray(level_weight, dtype=np.float64)[lev].ravel())
        return 1.0 / (np.concatenate(w) * d)

    # --- dense assembly (tiny configurations only) ---
    def dense_M(self):
        D = self.prior()
        return np.stack([self.apply_M(e, D) for e in np.eye(self.N)], axis=1)

    def dense_A(self):
        """Matrix of c -> A W^-1 c (S x N)."""
        return np.stack([self.A(self.W_inv(e)) for e in np.eye(self.N)], axis=1)


# ----------------------------------------------------------------------------------------
# Sec. 4: PCG (Alg. 1) and augmented PCG (Alg. 2); Sec. 5: Alg. 3 (RHS, residual update,
# augmented PCG) for consecutive frames.
# ----------------------------------------------------------------------------------------


def _ratio(num, den):
    """num / den for the step lengths and projection coefficients of Alg. 1 and 2.  With M
    symmetric positive definite a denominator (p, M p) or (r, J^-1 r) vanishes only for a zero
    vector, after the residual has become exactly zero (an all-zero right-hand side): the
    step along, or the coefficient of, a zero direction is then taken as zero."""
    return num / den if den > 0 else 0.0


def _step_ok(rz, pq):
    """Whether the step length rz / pq of Alg. 1 / Alg. 2 can be taken.  A breakdown is a
    non-finite value, or a non-positive curvature (p, M p) <= 0 while the preconditioned
    residual (r, J^-1 r) is not zero; (p, M p) = 0 with a zero residual is exact convergence."""
    if not (np.isfinite(rz) and np.isfinite(pq)):
        return False
    if pq > 0:
        return bool(np.isfinite(rz / pq))
    return pq == 0 and rz == 0


def pcg(apply_M, b, c0, Jinv, max_iter, r0=None, callback=None):
    """Alg. 1 (PCG, split Jacobi preconditioner J^-1), exactly ``max_iter`` applies of M.
    Returns c, r and the list of (p_k, q_k, (p_k, q_k))."""
    c = np.array(c0, dtype=np.float64, copy=True)
    r = b - apply_M(c) if r0 is None else np.array(r0, dtype=np.float64, copy=True)
    z = Jinv * r
    p = z.copy()
    rz = r @ z
    dirs = []
    for k in range(max_iter):
        q = apply_M(p)
        pq = p @ q
        alpha = _ratio(rz, pq)
        c = c + alpha * p
        r = r - alpha * q
        dirs.append((p, q, pq))
        if callback is not None:
            callback(c, r)
        z = Jinv * r
        rz_new = r @ z
        beta = _ratio(rz_new, rz)
        p = z + beta * p
        rz = rz_new
    return c, r, dirs


def _chol_drop(G, tol=1e-14):
    """Upper Cholesky factor R (G = R^T R) of a symmetric Gram matrix, processing columns in
    order and dropping column j when its pivot is <= tol * max(diag G)."""
    k = G.shape[0]
    R = np.zeros((k, k))
    keep = np.zeros(k, dtype=bool)
    thr = tol * max(np.max(np.diag(G)), 0.0)
    for j in range(k):
        d = G[j, j] - R[:j, j] @ R[:j, j]
        if not d > thr:
            continue
        keep[j] = True
        R[j, j] = np.sqrt(d)
        R[j, j + 1:] = (G[j, j + 1:] - R[:j, j] @ R[:j, j + 1:]) / R[j, j]
    return R, keep


def _chol_solve(R, keep, v):
    k = len(v)
    t = np.zeros(k)
    for j in range(k):                 # R^T t = v
        if keep[j]:
            t[j] = (v[j] - R[:j, j] @ t[:j]) / R[j, j]
    y = np.zeros(k)
    for j in reversed(range(k)):       # R y = t
        if keep[j]:
            y[j] = (t[j] - R[j, j + 1:] @ y[j + 1:]) / R[j, j]
    return y


def aug_pcg(apply_M, c, r, Jinv, U, Q, gam, max_iter, mode="galerkin", project_all=False,
            rel_tol=0.0, b_norm=None):
    """Alg. 2 (augmented PCG).  ``U``, ``Q``, ``gam``: the recycled directions p_j, q_j = M p_j
    and (p_j, q_j), oldest first.  Returns c, r, the new directions and an info dict.

    Breakdown (the paper runs a fixed iteration count and says nothing of it): when a
    projection coefficient, a step length or beta is not finite, or the curvature is not
    positive (see :func:`_step_ok`), c and r keep their last finite values (they stay each
    other's residual pair), the frame sets info flag bit 0, and every direction it stores from
    then on is the zero direction (p, q, (p, q)) = (0, 0, 0), which later projections give no
    weight."""
    c = np.array(c, dtype=np.float64, copy=True)
    r = np.array(r, dtype=np.float64, copy=True)
    m = len(U)
    dropped = 0
    broken = False
    R = keep = None
    # Galerkin initial guess: c_0 += P_m D_m^-1 P_m^T r_0 so that U^T r_0 = 0 (Sec. 4.1)
    if m:
        if mode == "paper":
            cg, rg = c, r
            for j in range(m):
                sigma = _ratio(rg @ U[j], gam[j])
                cg = cg + sigma * U[j]
                rg = rg - sigma * Q[j]
                broken |= not np.isfinite(sigma)
        else:
            G = np.zeros((m, m))
            for i in range(m):
                for j in range(i, m):
                    G[i, j] = G[j, i] = U[i] @ Q[j]
            R, keep = _chol_drop(G)
            dropped = int(m - keep.sum())
            y = _chol_solve(R, keep, np.array([u @ r for u in U]))
            broken |= not np.all(np.isfinite(y))
            cg, rg = c, r
            for j in range(m):
                cg = cg + y[j] * U[j]
                rg = rg - y[j] * Q[j]
        if not broken:
            c, r = cg, rg
    # initial direction, M-conjugate to the recycled directions (condition 1)
    z = Jinv * r
    if m and not broken:
        if mode == "paper":
            for j in range(m):
                tau = _ratio(z @ Q[j], gam[j])
                broken |= not np.isfinite(tau)
                z = z - tau * U[j]
        else:
            y = _chol_solve(R, keep, np.array([qq @ z for qq in Q]))
            broken |= not np.all(np.isfinite(y))
            for j in range(m):
                z = z - y[j] * U[j]
    p = z
    rz = r @ z
    new = []
    it = 0
    met = False
    zero = np.zeros_like(r)
    for k in range(max_iter):
        if broken:
            new.append((zero, zero, 0.0))
            it = k + 1
            continue
        q = apply_M(p)
        pq = p @ q
        if not _step_ok(rz, pq):
            broken = True
            new.append((zero, zero, 0.0))
            it = k + 1
            continue
        alpha = _ratio(rz, pq)
        c = c + alpha * p
        r = r - alpha * q
        new.append((p, q, pq))
        it = k + 1
        if rel_tol > 0 and np.sqrt(r @ r) <= rel_tol * b_norm:
            met = True
            break
        if k == max_iter - 1:
            break
        z = Jinv * r
        if m:
            if project_all and mode != "paper":
                y = _chol_solve(R, keep, np.array([qq @ z for qq in Q]))
                for j in range(m):
                    z = z - y[j] * U[j]
                rz_new = r @ z
            else:
                mu = _ratio(z @ Q[-1], gam[-1])
                z = z - mu * U[-1]
                rz_new = r @ z
        else:
            rz_new = r @ z
        beta = _ratio(rz_new, rz)
        if not np.isfinite(beta):
            broken = True
            continue
        p = z + beta * p
        rz = rz_new
    flags = (1 if broken else 0) | (2 if rel_tol > 0 and not met else 0)
    info = {"iters": it, "recycle_used": m, "dropped": dropped, "flags": flags,
            "rel_res": float("nan") if b_norm is None else float(np.sqrt(r @ r) / b_norm) if b_norm > 0 else 0.0}
    return c, r, new, info


# ----------------------------------------------------------------------------------------
# Learned warm start (an extension: the paper has no learned part).  Between the residual
# update of Alg. 3 and the Galerkin step of Alg. 2 a network proposes a nodal correction d of
# every layer; the frame moves along its coefficient form e = W d by the step that minimises
# the energy 1/2 c^T M c - b^T c along e (what the PCG iterations minimise), and never uphill.
# ----------------------------------------------------------------------------------------


def warm_start_inputs(system, c, r, Jinv, scale_c, scale_r):
    """Network inputs of every layer node, (N, 4): the previous coefficients and the
    preconditioned new residual as nodal fields, W^-1 c / scale_c and W^-1 (J^-1 r) / scale_r,
    then the layer's height / 20 km and its turbulence weight gamma_l."""
    out = np.empty((system.N, 4))
    out[:, 0] = np.concatenate([p.ravel() for p in system.W_inv(c)]) / scale_c
    out[:, 1] = np.concatenate([p.ravel() for p in system.W_inv(Jinv * r)]) / scale_r
    for l, lay in enumerate(system.layers):
        sl = slice(system.coff[l], system.coff[l + 1])
        out[sl, 2] = lay.height / 20000.0
        out[sl, 3] = lay.weight
    return out


def warm_start_correction(system, d):
    """Coefficient vector e = W d of a nodal correction d (N, layers concatenated).  W is the
    inverse of W^-1 = DWT^T / delta_l; DWT being orthonormal, W = delta_l DWT = delta_l^2 W^-T."""
    return np.concatenate([(dwt2(dl, lay.levels) * lay.spacing).ravel()
                           for dl, lay in zip(system.split_layers(np.asarray(d, dtype=np.float64)),
                                              system.layers)])


def warm_start_step(apply_M, c, r, e):
    """Exact line search of the energy along e from c, never uphill:
    tau = (e, r) / (e, M e) when both are positive, else 0; returns c + tau e, r - tau M e, tau."""
    Me = apply_M(e)
    er, eMe = float(e @ r), float(e @ Me)
    tau = er / eMe if (eMe > 0 and er > 0) else 0.0
    if tau > 0:
        return c + tau * e, r - tau * Me, tau
    return np.array(c, copy=True), np.array(r, copy=True), 0.0


class AugmentedReconstructor:
    """Alg. 3 steps RHS -> residual update -> augmented PCG for consecutive frames.  The
    first frame (and the first after :meth:`reset`) runs Alg. 1 from ``r = b - M c``.

    A frame whose right-hand side has a non-finite squared norm (non-finite or overflowing
    slopes; the paper is silent) is not solved: c, r and the previous right-hand side keep
    their values (after a first frame r becomes b_prev - M c, so that the next frame's residual
    update gives b - M c), the frame stores ``max_iter`` zero directions, and info reports
    flags bits 0 and 3, ``max_iter`` iterations and a NaN relative residual."""

    def __init__(self, system: OracleSystem, Jinv=None, max_iter=None, k=None, mode=None,
                 project_all=None, rel_tol=None):
        spec = system.spec
        self.sys = system
        self.D = system.prior()
        lw = getattr(spec, "level_weight", None)
        if Jinv is not None:
            self.Jinv = np.asarray(Jinv, np.float64)
        elif lw is not None:
            self.Jinv = system.modified_jacobi(list(lw) + [1.0] * (16 - len(lw)), self.D)
        else:
            self.Jinv = 1.0 / system.diag_M(self.D)
        self.max_iter = spec.max_iter if max_iter is None else max_iter
        self.k = spec.recycle_k if k is None else k
        self.mode = spec.recycle_mode if mode is None else mode
        self.project_all = spec.project_all if project_all is None else project_all
        self.rel_tol = spec.rel_tol if rel_tol is None else rel_tol
        self.c = np.zeros(system.N)
        self.r = np.zeros(system.N)
        self.b_prev = np.zeros(system.N)
        self.store = []          # recycled (p, q, (p, q)), oldest first
        self.first = True

    def apply_M(self, x):
        return self.sys.apply_M(x, self.D)

    def reset(self):
        self.store = []
        self.first = True

    def _keep(self, new):
        if self.mode == "paper":
            self.store = new[-self.k:] if self.k > 0 else []
        else:
            self.store = (self.store + new)[-self.k:] if self.k > 0 else []

    def solve(self, s, correction=None, scales=(1.0, 1.0, 1.0)):
        """One frame for slopes s.  ``correction`` (warm start, optional): a callable mapping
        the network inputs (see :func:`warm_start_inputs`, with ``scales`` = (scale_c, scale_r,
        scale_out)) to a normalised nodal correction; the frame takes the line-search step
        along W (scale_out d) after the residual update (info key "tau")."""
        b = self.sys.rhs(s)
        bb = float(b @ b)
        if not np.isfinite(bb):
            zero = np.zeros(self.sys.N)
            if self.first:
                self.r = self.b_prev - self.apply_M(self.c)
            used = 0 if self.first else min(self.k, len(self.store))
            self._keep([(zero, zero, 0.0)] * self.max_iter)
            self.first = False
            return self.c.copy(), {"iters": self.max_iter, "recycle_used": used, "dropped": 0,
                                   "flags": 9 | (2 if self.rel_tol > 0 else 0), "rel_res": float("nan")}
        b_norm = float(np.sqrt(bb))
        if self.first:
            r = b - self.apply_M(self.c)
            used = []
        else:
            r = (b - self.b_prev) + self.r          # Alg. 3 residual update
            used = self.store[-self.k:] if self.k > 0 else []
        c0 = self.c
        tau = None
        if correction is not None:
            sc, sr, so = scales
            d = so * np.asarray(correction(warm_start_inputs(self.sys, c0, r, self.Jinv, sc, sr)), dtype=np.float64)
            c0, r, tau = warm_start_step(self.apply_M, c0, r, warm_start_correction(self.sys, d))
        U = [u for u, _, _ in used]
        Q = [q for _, q, _ in used]
        gam = [g for _, _, g in used]
        c, r, new, info = aug_pcg(self.apply_M, c0, r, self.Jinv, U, Q, gam, self.max_iter,
                                  self.mode, self.project_all, self.rel_tol, b_norm)
        self._keep(new)
        self.c, self.r, self.b_prev = c, r, b
        self.first = False
        if tau is not None:
            info["tau"] = tau
        return c, info


def exact_solution(system: OracleSystem, b, tol=1e-14, max_iter=20000, dense_limit=3000):
    """c* = M^-1 b: dense Cholesky for small N, otherwise Jacobi-PCG to ||r|| <= tol ||b||."""
    if system.N <= dense_limit:
        Md = system.dense_M()
        Lc = np.linalg.cholesky(Md)
        return np.linalg.solve(Lc.T, np.linalg.solve(Lc, b))
    D = system.prior()
    Jinv = 1.0 / system.diag_M(D)
    c = np.zeros_like(b)
    r = b.copy()
    z = Jinv * r
    p = z.copy()
    rz = r @ z
    bn = np.sqrt(b @ b)
    for _ in range(max_iter):
        q = system.apply_M(p, D)
        a = rz / (p @ q)
        c += a * p
        r -= a * q
        if np.sqrt(r @ r) <= tol * bn:
            break
        z = Jinv * r
        rzn = r @ z
        p = z + (rzn / rz) * p
        rz = rzn
    return c
