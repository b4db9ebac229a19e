"""Seeded frozen-flow von Karman atmosphere and a Shack-Hartmann measurement simulator.

The simulator stands in for the end-to-end AO simulation the paper uses (its
MOST package is not available): it is the *telescope*, not the reconstructor.

* Each layer is a periodic FFT phase screen with the von Karman power spectrum
  ``0.023 r0_l^(-5/3) (f^2 + L0^-2)^(-11/6)`` and ``r0_l = r0 gamma_l^(-3/5)``,
  sampled at half the finest reconstruction-grid spacing.
* Frozen flow: at frame ``t`` layer ``l`` is shifted by ``wind_l * t * dt``.
* The wavefront seen by guide star ``g`` at pupil point ``x`` is the sum over
  layers of the screen at ``(1 - h/H) x + theta h`` (geometric optics).
* A subaperture measures the mean phase difference across it: the average over
  its edges (``q`` sub-samples each, trapezoid rule) of right-minus-left (x) and
  top-minus-bottom (y) phase.  Inactive subapertures read zero.
* Noise: Gaussian, standard deviation ``sigma_g = rms(noise-free frame-0
  slopes) / SNR`` per sensor; the inverse variance (times the mask) is the
  diagonal noise weighting handed to the reconstructor.
"""
from __future__ import annotations

import numpy as np

from .geometry import SystemSpec, WfsSpec, wfs_node_coords


def von_karman_screen(rng: np.random.Generator, n: int, dx: float, r0: float, L0: float) -> np.ndarray:
    fx = np.fft.fftfreq(n, dx)
    f2 = fx[None, :] ** 2 + fx[:, None] ** 2
    psd = 0.023 * r0 ** (-5.0 / 3.0) * (f2 + L0 ** -2) ** (-11.0 / 6.0)
    psd[0, 0] = 0.0
    df = 1.0 / (n * dx)
    c = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) * np.sqrt(psd) * df
    return np.real(np.fft.ifft2(c)) * (n * n)


class FrozenFlowAtmosphere:
    def __init__(self, spec: SystemSpec, seed: int):
        rng = np.random.default_rng(seed)
        self.dx = min(l.spacing for l in spec.layers) / 2.0
        extent = max(l.spacing * (l.n - 1) for l in spec.layers)
        n = 64
        while n * self.dx < 1.25 * extent:
            n *= 2
        self.n = n
        self.heights = np.array([l.height for l in spec.layers])
        self.winds = np.array([l.wind for l in spec.layers], dtype=float)
        self.screens = [von_karman_screen(rng, n, self.dx, spec.r0 * l.weight ** (-0.6), spec.L0)
                        for l in spec.layers]
        self.dt = spec.dt

    def sample(self, layer: int, x: np.ndarray, y: np.ndarray, t: int) -> np.ndarray:
        """Bilinear sample of the (periodic) screen of `layer` at frame t."""
        sx, sy = self.winds[layer] * (t * self.dt)
        u = (x - sx) / self.dx
        v = (y - sy) / self.dx
        u0 = np.floor(u)
        v0 = np.floor(v)
        fu = u - u0
        fv = v - v0
        n = self.n
        i0 = v0.astype(np.int64) % n
        j0 = u0.astype(np.int64) % n
        i1 = (i0 + 1) % n
        j1 = (j0 + 1) % n
        s = self.screens[layer]
        return ((1 - fv) * ((1 - fu) * s[i0, j0] + fu * s[i0, j1])
                + fv * ((1 - fu) * s[i1, j0] + fu * s[i1, j1]))


class SlopeSimulator:
    """Noise-free and noisy slopes of every WFS of `spec` for a frozen-flow atmosphere."""

    def __init__(self, spec: SystemSpec, atmosphere: FrozenFlowAtmosphere, q: int = 2):
        self.spec = spec
        self.atm = atmosphere
        self.q = q

    def _wavefront(self, w: WfsSpec, t: int) -> np.ndarray:
        q = self.q
        x = (np.arange(w.n_sub * q + 1) / q - w.n_sub / 2.0) * w.subap
        X, Y = np.meshgrid(x, x, indexing="xy")        # Y varies along rows
        psi = np.zeros_like(X)
        for l, h in enumerate(self.atm.heights):
            scale = 1.0 - h / w.lgs_height if w.lgs_height > 0 else 1.0
            psi += self.atm.sample(l, scale * X + w.theta_x * h, scale * Y + w.theta_y * h, t)
        return psi

    def clean_slopes(self, t: int) -> np.ndarray:
        q = self.q
        trap = np.full(q + 1, 1.0)
        trap[0] = trap[-1] = 0.5
        trap /= q
        out = []
        for w in self.spec.wfs:
            psi = self._wavefront(w, t)
            ns = w.n_sub
            # edge samples of every subaperture: rows i*q + 0..q, columns j*q and (j+1)*q
            idx = np.arange(ns)[:, None] * q + np.arange(q + 1)[None, :]     # (ns, q+1)
            left = psi[idx[:, None, :], (np.arange(ns) * q)[None, :, None]]       # (ns, ns, q+1)
            right = psi[idx[:, None, :], (np.arange(ns) * q + q)[None, :, None]]
            bottom = psi[(np.arange(ns) * q)[:, None, None], idx[None, :, :]]
            top = psi[(np.arange(ns) * q + q)[:, None, None], idx[None, :, :]]
            sx = ((right - left) * trap).sum(-1)
            sy = ((top - bottom) * trap).sum(-1)
            sx = np.where(w.mask, sx, 0.0)
            sy = np.where(w.mask, sy, 0.0)
            out.append(np.concatenate([sx.ravel(), sy.ravel()]))
        return out

    @staticmethod
    def elongation_geometry(w: WfsSpec):
        """Per subaperture: the radial unit vector (ex, ey) from the pupil centre and the
        variance factor k = 1 + (elongation r / R)^2 along it."""
        ns = w.n_sub
        c = (np.arange(ns) + 0.5 - ns / 2.0) * w.subap
        X, Y = np.meshgrid(c, c, indexing="xy")
        r = np.hypot(X, Y)
        ex = np.where(r > 0, X / np.where(r > 0, r, 1.0), 1.0)
        ey = np.where(r > 0, Y / np.where(r > 0, r, 1.0), 0.0)
        k = 1.0 + (w.elongation * r / (ns * w.subap / 2.0)) ** 2
        return ex.ravel(), ey.ravel(), k.ravel()

    def calibrate_noise(self, snr: float) -> None:
        """Set per-WFS sigma (from noise-free frame-0 slopes) and the inverse noise covariance:
        diagonal slope weights, and for an elongated LGS spot the 2x2 block per subaperture
        B = Sigma^-1, Sigma = sigma^2 (I + (k - 1) e e^T)."""
        for w, s in zip(self.spec.wfs, self.clean_slopes(0)):
            m = np.concatenate([w.mask.ravel(), w.mask.ravel()])
            rms = float(np.sqrt(np.mean(s[m] ** 2)))
            w.sigma = rms / snr
            if w.elongation > 0:
                ex, ey, k = self.elongation_geometry(w)
                a = (1.0 - 1.0 / k) / w.sigma ** 2
                mk = w.mask.ravel()
                bxx = np.where(mk, 1.0 / w.sigma ** 2 - a * ex * ex, 0.0)
                byy = np.where(mk, 1.0 / w.sigma ** 2 - a * ey * ey, 0.0)
                w.weight = np.concatenate([bxx, byy])
                w.cross_weight = np.where(mk, -a * ex * ey, 0.0)
            else:
                w.weight = np.where(m, 1.0 / w.sigma ** 2, 0.0)
                w.cross_weight = None

    def noisy_slopes(self, t: int, seed: int) -> np.ndarray:
        rng = np.random.default_rng([seed, t])
        parts = []
        for w, s in zip(self.spec.wfs, self.clean_slopes(t)):
            m = np.concatenate([w.mask.ravel(), w.mask.ravel()])
            z = rng.standard_normal(s.size)
            if w.elongation > 0:   # eta = sigma (z + (sqrt(k) - 1) (e . z) e)
                n2 = w.n_sub * w.n_sub
                ex, ey, k = self.elongation_geometry(w)
                ez = (np.sqrt(k) - 1.0) * (ex * z[:n2] + ey * z[n2:])
                z = np.concatenate([z[:n2] + ez * ex, z[n2:] + ez * ey])
            noisy = s + w.sigma * z
            if w.tt_jitter > 0:    # a global tip/tilt of this frame (LGS uplink jitter)
                a = w.sigma * w.tt_jitter * rng.standard_normal(2)
                n2 = w.n_sub * w.n_sub
                noisy = noisy + np.concatenate([np.full(n2, a[0]), np.full(n2, a[1])])
            parts.append(np.where(m, noisy, 0.0))
        return np.concatenate(parts)


def make_sequence(spec: SystemSpec, n_frames: int, seed: int, q: int = 2, start: int = 0):
    """Calibrate the noise weights of `spec` (in place) and return an (n_frames, S) float64
    array of consecutive noisy closed-form slope frames."""
    atm = FrozenFlowAtmosphere(spec, seed)
    sim = SlopeSimulator(spec, atm, q=q)
    sim.calibrate_noise(spec.snr)
    return np.stack([sim.noisy_slopes(start + t, seed) for t in range(n_frames)])
