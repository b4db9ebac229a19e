"""Plain FP64 CPU oracle of the closed-loop wrapper of the augmented wavelet reconstructor
(Sec. 5, Alg. 3): pseudo-open-loop slopes, fitting of the reconstructed layers to deformable-
mirror (DM) actuator commands, and gain control.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): never imported by the GPU library.

Readings taken where the paper is silent (all listed in the design notes as well):

* DMs (Sec. 6, system table: actuators per side, altitude, spacing).  A DM is a square grid of
  ``n`` actuators with spacing ``d`` at altitude ``h``, actuator ``(a, b)`` at
  ``origin + ((b - (n-1)/2) d, (a - (n-1)/2) d)`` (the layer-grid convention); its surface is
  the bilinear interpolant of the commands, zero outside the grid (commands beyond the edge are
  zero).
* Interaction ``Gamma a`` of the pseudo-open-loop step (Alg. 3): read as the DM-to-sensor map
  ``H``: for sensor g, the sum over DMs of the surface at the cone-scaled, shifted node
  positions ``(1 - h_d / H_g) x + theta_g h_d`` (the propagation of Sec. 2 with the DMs as
  layers), then the Shack-Hartmann operator (zero on inactive subapertures).  Closed-loop
  measurements are the open-loop ones minus ``H a^(i-1)`` (two-step delay), so the
  pseudo-open-loop slopes ``s + H a^(i-1)`` recover them.
* Fitting ``a~ = F W^-1 c`` (Alg. 3; Sec. 6.1 for the two forms):
  - direct (the layers sit at the DM altitudes): the commands of DM d are layer d's function
    at the actuator positions;
  - least squares (more layers than DMs): the commands minimise
    ``sum_theta sum_x |sum_d a_d(x + theta h_d) - sum_l phi_l(x + theta h_l)|^2`` over a set of
    science directions theta and the pupil points x of a square sample grid (spacing
    ``D / (n_pts - 1)``, points inside the annulus); its normal equations are solved by
    ``fit_iter`` unpreconditioned CG iterations started from the previous frame's fitted
    commands (zero for the first frame).
* Gain control (Alg. 3): closed loop ``a^(i+1) = a^(i) + gain (a~ - a^(i-1))``, open loop
  ``a^(i+1) = (1 - gain) a^(i) + gain a~``.
"""
from __future__ import annotations

import numpy as np


def gain_update(a_prev, a_cur, a_fit, gain, closed):
    """Gain control of Alg. 3: the next commands from a^(i-1), a^(i) and the fitted a~."""
    if closed:
        return a_cur + gain * (a_fit - a_prev)
    return (1.0 - gain) * a_cur + gain * a_fit


class DmSpec:
    """One deformable mirror: ``n`` x ``n`` actuators of spacing ``spacing`` at ``height``."""

    def __init__(self, height, n, spacing, origin_x=0.0, origin_y=0.0):
        self.height, self.n, self.spacing = float(height), int(n), float(spacing)
        self.origin_x, self.origin_y = float(origin_x), float(origin_y)


def _grid_coord(p, origin, spacing, n):
    """Fractional grid coordinate of position p on an n-point grid centred at origin."""
    return (p - origin) / spacing + (n - 1) / 2.0


def bilinear_zero(img, u, v):
    """Bilinear interpolant of the n x n node values img at fractional coordinates (u: column,
    v: row), the nodes beyond the grid being zero."""
    n = img.shape[0]
    b0, a0 = np.floor(u).astype(np.int64), np.floor(v).astype(np.int64)
    fx, fy = u - b0, v - a0
    out = np.zeros(np.broadcast(u, v).shape)
    for da, wa in ((0, 1 - fy), (1, fy)):
        for db, wb in ((0, 1 - fx), (1, fx)):
            a, b = a0 + da, b0 + db
            ok = (a >= 0) & (a < n) & (b >= 0) & (b < n)
            out += np.where(ok, wa * wb * img[np.clip(a, 0, n - 1), np.clip(b, 0, n - 1)], 0.0)
    return out


def bilinear_zero_T(val, u, v, n):
    """Adjoint of :func:`bilinear_zero` in the node values: scatters val onto an n x n grid."""
    out = np.zeros((n, n))
    b0, a0 = np.floor(u).astype(np.int64), np.floor(v).astype(np.int64)
    fx, fy = u - b0, v - a0
    for da, wa in ((0, 1 - fy), (1, fy)):
        for db, wb in ((0, 1 - fx), (1, fx)):
            a, b = a0 + da, b0 + db
            ok = (a >= 0) & (a < n) & (b >= 0) & (b < n)
            np.add.at(out, (np.clip(a, 0, n - 1)[ok], np.clip(b, 0, n - 1)[ok]), (wa * wb * val)[ok])
    return out


class ClosedLoopOracle:
    """Alg. 3 around an :class:`oracle.fewha_oracle.AugmentedReconstructor`: pseudo-open-loop
    slopes, the frame solve, fitting and gain control."""

    def __init__(self, rec, dms, gain=0.4, closed=True, fit_dirs=None, n_pts=0, fit_iter=0):
        self.rec = rec
        self.sys = rec.sys
        self.dms = list(dms)
        self.gain = float(gain)
        self.closed = bool(closed)
        self.fit_iter = int(fit_iter)
        self.off = np.cumsum([0] + [d.n * d.n for d in self.dms])
        self.n_act = int(self.off[-1])
        spec = self.sys.spec
        if self.fit_iter == 0:
            if len(self.dms) != self.sys.L or any(abs(d.height - l.height) > 1e-9 for d, l in zip(self.dms, self.sys.layers)):
                raise ValueError("direct fitting needs one DM at the altitude of every layer")
        else:
            self.fit_dirs = np.asarray(fit_dirs, dtype=np.float64).reshape(-1, 2)
            t = (np.arange(n_pts) - (n_pts - 1) / 2.0) * spec.D / (n_pts - 1)
            X, Y = np.meshgrid(t, t, indexing="xy")
            r = np.hypot(X, Y)
            self.pupil = (r <= spec.D / 2.0) & (r >= spec.obstruction * spec.D / 2.0)
            self.px, self.py = X[self.pupil], Y[self.pupil]
        self.a_prev = np.zeros(self.n_act)     # a^(i-1)
        self.a_cur = np.zeros(self.n_act)      # a^(i)
        self.a_fit = np.zeros(self.n_act)      # the previous fitted commands (CG start)

    def split(self, a):
        return [a[self.off[k]:self.off[k + 1]].reshape(d.n, d.n) for k, d in enumerate(self.dms)]

    # --- H: DM commands -> slopes of every sensor (the pseudo-open-loop interaction)
    def dm_slopes(self, a):
        out = []
        for g, w in enumerate(self.sys.wfs):
            x = (np.arange(w.n_sub + 1) - w.n_sub / 2.0) * w.subap
            X, Y = np.meshgrid(x, x, indexing="xy")
            wf = np.zeros_like(X)
            for ad, d in zip(self.split(a), self.dms):
                sc = 1.0 - d.height / w.lgs_height if w.lgs_height > 0 else 1.0
                u = _grid_coord(sc * X + w.theta_x * d.height, d.origin_x, d.spacing, d.n)
                v = _grid_coord(sc * Y + w.theta_y * d.height, d.origin_y, d.spacing, d.n)
                wf += bilinear_zero(ad, u, v)
            out.append(self.sys.shack_hartmann(wf, g))
        return np.concatenate(out)

    def dm_slopes_T(self, s):
        acc = [np.zeros((d.n, d.n)) for d in self.dms]
        for g, (w, sg) in enumerate(zip(self.sys.wfs, self.sys.split_slopes(s))):
            wf = self.sys.shack_hartmann_T(sg, g)
            x = (np.arange(w.n_sub + 1) - w.n_sub / 2.0) * w.subap
            X, Y = np.meshgrid(x, x, indexing="xy")
            for k, d in enumerate(self.dms):
                sc = 1.0 - d.height / w.lgs_height if w.lgs_height > 0 else 1.0
                u = _grid_coord(sc * X + w.theta_x * d.height, d.origin_x, d.spacing, d.n)
                v = _grid_coord(sc * Y + w.theta_y * d.height, d.origin_y, d.spacing, d.n)
                acc[k] += bilinear_zero_T(wf, u, v, d.n)
        return np.concatenate([a.ravel() for a in acc])

    # --- fitting
    def _layers_at(self, phis, th):
        """sum_l phi_l(x + theta h_l) at the pupil points."""
        out = np.zeros(self.px.size)
        for ph, lay in zip(phis, self.sys.layers):
            u = _grid_coord(self.px + th[0] * lay.height, lay.origin_x, lay.spacing, lay.n)
            v = _grid_coord(self.py + th[1] * lay.height, lay.origin_y, lay.spacing, lay.n)
            out += bilinear_zero(ph, u, v)
        return out

    def _dms_at(self, a, th):
        out = np.zeros(self.px.size)
        for ad, d in zip(self.split(a), self.dms):
            u = _grid_coord(self.px + th[0] * d.height, d.origin_x, d.spacing, d.n)
            v = _grid_coord(self.py + th[1] * d.height, d.origin_y, d.spacing, d.n)
            out += bilinear_zero(ad, u, v)
        return out

    def _dms_at_T(self, val, th):
        acc = []
        for d in self.dms:
            u = _grid_coord(self.px + th[0] * d.height, d.origin_x, d.spacing, d.n)
            v = _grid_coord(self.py + th[1] * d.height, d.origin_y, d.spacing, d.n)
            acc.append(bilinear_zero_T(val, u, v, d.n).ravel())
        return np.concatenate(acc)

    def fit_normal(self, a):
        """sum_theta P_theta^T P_theta a: the matrix of the fitting's normal equations."""
        return sum(self._dms_at_T(self._dms_at(a, th), th) for th in self.fit_dirs)

    def fit_rhs(self, phis):
        return sum(self._dms_at_T(self._layers_at(phis, th), th) for th in self.fit_dirs)

    def fit(self, c):
        """a~ = F W^-1 c."""
        phis = self.sys.W_inv(c)
        if self.fit_iter == 0:
            out = []
            for ph, lay, d in zip(phis, self.sys.layers, self.dms):
                t = (np.arange(d.n) - (d.n - 1) / 2.0) * d.spacing
                X, Y = np.meshgrid(d.origin_x + t, d.origin_y + t, indexing="xy")
                out.append(bilinear_zero(ph, _grid_coord(X, lay.origin_x, lay.spacing, lay.n),
                                         _grid_coord(Y, lay.origin_y, lay.spacing, lay.n)).ravel())
            return np.concatenate(out)
        # unpreconditioned CG on the normal equations, from the previous fitted commands
        x = self.a_fit.copy()
        r = self.fit_rhs(phis) - self.fit_normal(x)
        p = r.copy()
        rr = r @ r
        for _ in range(self.fit_iter):
            q = self.fit_normal(p)
            pq = p @ q
            alpha = rr / pq if pq > 0 else 0.0
            x = x + alpha * p
            r = r - alpha * q
            rr_new = r @ r
            beta = rr_new / rr if rr > 0 else 0.0
            p = r + beta * p
            rr = rr_new
        return x

    # --- one frame of Alg. 3
    def step(self, s):
        """Slopes as measured (closed loop: after the DMs) -> the next DM commands."""
        s_ol = s + self.dm_slopes(self.a_prev) if self.closed else s
        c, info = self.rec.solve(s_ol)
        a_fit = self.fit(c)
        self.a_fit = a_fit
        a_next = gain_update(self.a_prev, self.a_cur, a_fit, self.gain, self.closed)
        self.a_prev, self.a_cur = self.a_cur, a_next
        return a_next, info
