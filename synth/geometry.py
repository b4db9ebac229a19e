"""System description: telescope pupil, guide-star wavefront sensors and layer grids.

Conventions (the paper leaves the discrete geometry open; these are the readings
used by every part of this repository):

* Wavefront sensor ``g`` has ``n_sub`` x ``n_sub`` square subapertures of side
  ``subap = D / n_sub``.  Its bilinear wavefront lives on ``(n_sub+1)^2`` nodes;
  node ``(i, j)`` (``i`` = row along y, ``j`` = column along x) sits at pupil
  coordinates ``((j - n_sub/2) * subap, (i - n_sub/2) * subap)`` (Sec. 2, the
  Shack-Hartmann model, and Fig. 1 of Sec. 3).
* A subaperture is active when at least half of its area lies in the annulus
  between the central obstruction and the pupil edge (16 x 16 supersampling).
* Layer ``l`` is a square grid of ``n = 2^J_l`` nodes per side with spacing
  ``spacing`` (d_l) centred at ``(origin_x, origin_y)``; node ``(a, b)`` sits at
  ``origin + ((b - (n-1)/2) d_l, (a - (n-1)/2) d_l)`` (Sec. 3, dual-domain
  discretisation).  The grid is fitted so that every projected guide-star
  footprint lies inside it with a margin of one cell:
  ``d_l = E_l / (n - 2)`` where ``E_l`` is the larger side of the bounding box of
  all projected WFS nodes at height ``h_l``.
* A natural guide star has ``lgs_height == 0``; a laser guide star at height H
  sees the layer point ``(1 - h/H) x + theta h`` (Sec. 2, cone effect).
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

ARCSEC = np.pi / 180.0 / 3600.0


@dataclass
class LayerSpec:
    height: float            # h_l [m]
    weight: float            # gamma_l, fraction of the turbulence strength
    n: int                   # grid side 2^J_l
    levels: int              # number of wavelet levels
    spacing: float = 0.0     # d_l [m]
    origin_x: float = 0.0    # grid centre [m]
    origin_y: float = 0.0
    wind: tuple = (0.0, 0.0)  # frozen-flow velocity [m/s] (simulator only)


@dataclass
class WfsSpec:
    n_sub: int
    subap: float             # d_s [m]
    theta_x: float           # guide-star direction [rad]
    theta_y: float
    lgs_height: float        # H [m]; 0 for a natural guide star
    mask: np.ndarray = None  # (n_sub, n_sub) bool, active subapertures
    weight: Optional[np.ndarray] = None  # 2 n_sub^2 slope weights (inverse noise variance incl. mask)
    sigma: float = 0.0       # slope noise standard deviation used by the simulator
    # laser-guide-star noise model (simulator and C_eta^-1): spot elongation, radial from the
    # launch axis at the pupil centre, raises the noise standard deviation along the radius
    # to sigma sqrt(1 + (elongation r / R)^2) at distance r (R = pupil radius); the inverse
    # covariance is then a 2x2 block per subaperture, whose off-diagonal is cross_weight
    elongation: float = 0.0
    cross_weight: Optional[np.ndarray] = None   # n_sub^2 (x, y) entries of the blocks, or None
    tt_filter: bool = False  # C_eta^-1 blind to this sensor's global tip/tilt
    tt_jitter: float = 0.0   # simulator: per-frame global tip/tilt of the slopes, in units of sigma


@dataclass
class SystemSpec:
    name: str
    D: float
    obstruction: float       # central obstruction diameter ratio
    layers: List[LayerSpec]
    wfs: List[WfsSpec]
    alpha: float = 2.0
    r0: float = 0.129        # Fried parameter [m] at 500 nm
    L0: float = 25.0         # outer scale [m]
    max_iter: int = 6
    recycle_k: int = 5
    recycle_mode: str = "galerkin"   # "galerkin" or "paper"
    project_all: bool = False
    rel_tol: float = 0.0
    precision: str = "fp64"          # "fp64" or "fp32"
    snr: float = 10.0
    dt: float = 2e-3                  # frame period [s]
    # frequency-weighted Jacobi: weight of the details of level l at [l - 1], of the scaling
    # coefficients at [levels]; None for the exact Jacobi preconditioner
    level_weight: Optional[Tuple[float, ...]] = None

    def copy(self, **changes) -> "SystemSpec":
        new = dataclasses.replace(self, **changes)
        if "layers" not in changes:
            new.layers = [dataclasses.replace(l) for l in self.layers]
        if "wfs" not in changes:
            new.wfs = [dataclasses.replace(w) for w in self.wfs]
        return new


def n_coeffs(spec: SystemSpec) -> int:
    return int(sum(l.n * l.n for l in spec.layers))


def n_slopes(spec: SystemSpec) -> int:
    return int(sum(2 * w.n_sub * w.n_sub for w in spec.wfs))


def wfs_node_coords(w: WfsSpec) -> np.ndarray:
    """1-D node coordinates (same along x and y), length n_sub + 1."""
    return (np.arange(w.n_sub + 1) - w.n_sub / 2.0) * w.subap


def subaperture_mask(n_sub: int, D: float, obstruction: float, supersample: int = 16) -> np.ndarray:
    d = D / n_sub
    t = (np.arange(supersample) + 0.5) / supersample
    edges = (np.arange(n_sub) - n_sub / 2.0) * d
    pts = (edges[:, None] + t[None, :] * d).ravel()          # n_sub*supersample sample coords
    yy, xx = np.meshgrid(pts, pts, indexing="ij")
    rr = np.hypot(xx, yy)
    inside = (rr <= D / 2.0) & (rr >= obstruction * D / 2.0)
    frac = inside.reshape(n_sub, supersample, n_sub, supersample).mean(axis=(1, 3))
    return frac >= 0.5


def _projected_extent(w: WfsSpec, h: float):
    x = wfs_node_coords(w)
    scale = 1.0 - h / w.lgs_height if w.lgs_height > 0 else 1.0
    xs = scale * x + w.theta_x * h
    ys = scale * x + w.theta_y * h
    return xs.min(), xs.max(), ys.min(), ys.max()


def fit_layer_grids(spec: SystemSpec) -> SystemSpec:
    """Set spacing/origin of every layer so that all footprints fit (one-cell margin)."""
    for lay in spec.layers:
        ext = np.array([_projected_extent(w, lay.height) for w in spec.wfs])
        x0, x1 = ext[:, 0].min(), ext[:, 1].max()
        y0, y1 = ext[:, 2].min(), ext[:, 3].max()
        E = max(x1 - x0, y1 - y0)
        lay.spacing = E / (lay.n - 2)
        lay.origin_x = 0.5 * (x0 + x1)
        lay.origin_y = 0.5 * (y0 + y1)
    return spec


def _winds(rng, speeds):
    ang = rng.uniform(0, 2 * np.pi, size=len(speeds))
    return [(float(s * np.cos(a)), float(s * np.sin(a))) for s, a in zip(speeds, ang)]


def config_small(seed: int = 1) -> SystemSpec:
    """8 m telescope, 3 NGS SH-WFS 40x40 (on-axis and +-1 arcmin), 3 layers at 0/4/12 km
    (weights 0.5/0.3/0.2) on 64x64 grids, db3 over 4 levels, r0 0.157 m, L0 25 m,
    10 PCG iterations, recycle dimension 5, FP64."""
    rng = np.random.default_rng(seed)
    D, ns = 8.0, 40
    mask = subaperture_mask(ns, D, 0.0)
    wfs = [WfsSpec(ns, D / ns, tx * ARCSEC, 0.0, 0.0, mask.copy()) for tx in (0.0, 60.0, -60.0)]
    winds = _winds(rng, [10.0, 15.0, 20.0])
    layers = [LayerSpec(h, g, 64, 4, wind=wv) for h, g, wv in
              zip((0.0, 4000.0, 12000.0), (0.5, 0.3, 0.2), winds)]
    spec = SystemSpec("small_ngs_fp64", D, 0.0, layers, wfs, alpha=2.0, r0=0.157, L0=25.0,
                      max_iter=10, recycle_k=5, precision="fp64")
    return fit_layer_grids(spec)


def config_elt_mcao(seed: int = 2, precision: str = "fp32", ground_n: int = 256,
                    other_n: int = 128) -> SystemSpec:
    """39 m ELT, 28 % central obstruction, 6 LGS (84x84 subapertures) on a 45 arcsec radius at
    90 km, 9 layers 0-20 km with weights decaying as exp(-h / 4 km), 256^2 ground grid and
    128^2 grids above, db3 over 6 levels, r0 0.129 m, alpha 2, 6 PCG iterations, k = 10."""
    rng = np.random.default_rng(seed)
    D, ns = 39.0, 84
    mask = subaperture_mask(ns, D, 0.28)
    wfs = []
    for az in np.arange(6) * 60.0:
        a = np.deg2rad(az)
        wfs.append(WfsSpec(ns, D / ns, 45.0 * ARCSEC * np.cos(a), 45.0 * ARCSEC * np.sin(a),
                           90000.0, mask.copy()))
    hs = np.array([0, 1, 2, 4, 6, 8, 12, 16, 20], dtype=float) * 1000.0
    gam = np.exp(-hs / 4000.0)
    gam /= gam.sum()
    speeds = np.linspace(5.0, 20.0, len(hs))
    winds = _winds(rng, speeds)
    layers = [LayerSpec(float(h), float(g), ground_n if i == 0 else other_n, 6, wind=wv)
              for i, (h, g, wv) in enumerate(zip(hs, gam, winds))]
    spec = SystemSpec("elt_mcao_" + precision, D, 0.28, layers, wfs, alpha=2.0, r0=0.129,
                      L0=25.0, max_iter=6, recycle_k=10, precision=precision)
    return fit_layer_grids(spec)


def config_elt_full(seed: int = 2, precision: str = "fp32") -> SystemSpec:
    """The ELT MCAO system of config_elt_mcao plus the three low-order natural guide stars of
    the paper's MCAO asterism (Sec. 6, system table and asterism figure): one 2x2 and two 1x1
    Shack-Hartmann sensors on an 80 arcsec radius triangle (azimuths 90, 210, 330 degrees).
    The layer grids are refitted so that the wider natural-star footprints fit."""
    spec = config_elt_mcao(seed=seed, precision=precision)
    D, obs = spec.D, spec.obstruction
    for ns, az in ((2, 90.0), (1, 210.0), (1, 330.0)):
        a = np.deg2rad(az)
        spec.wfs.append(WfsSpec(ns, D / ns, 80.0 * ARCSEC * np.cos(a), 80.0 * ARCSEC * np.sin(a), 0.0,
                                subaperture_mask(ns, D, obs)))
    spec.name = "elt_full_" + precision
    return fit_layer_grids(spec)


def elt_mcao_dms():
    """The three deformable mirrors of the paper's MCAO system (Sec. 6, system table), as
    (altitude [m], actuators per side, spacing [m]): 85 x 85 at 0 m with 0.5 m spacing,
    47 x 47 at 4 km and 53 x 53 at 12.7 km with 1 m spacing."""
    return [(0.0, 85, 0.5), (4000.0, 47, 1.0), (12700.0, 53, 1.0)]


def mcao_fit_directions():
    """The 5 x 5 grid of science directions of the MCAO asterism figure (Sec. 6): +-60 arcsec
    in steps of 30 arcsec, as (theta_x, theta_y) [rad], row by row."""
    return [(x * 30 * ARCSEC, y * 30 * ARCSEC) for y in range(-2, 3) for x in range(-2, 3)]


def config_elt_lgs_noise(seed: int = 2, precision: str = "fp32", elongation: float = 3.0,
                         tt_jitter: float = 5.0) -> SystemSpec:
    """The full ELT system (config_elt_full: 6 LGS + 3 NGS) with the laser-guide-star noise
    model: radially elongated spots (noise along the radius sqrt(1 + elongation^2) times larger
    at the pupil edge) and a per-frame tip/tilt jitter of the LGS slopes, which the
    reconstructor filters out of the LGS data (the NGS measure tip/tilt)."""
    spec = config_elt_full(seed=seed, precision=precision)
    for w in spec.wfs:
        if w.lgs_height > 0:
            w.elongation, w.tt_filter, w.tt_jitter = elongation, True, tt_jitter
    spec.name = "elt_lgs_noise_" + precision
    return spec


def config_tiny(seed: int = 3, n: int = 16, levels: int = 3, n_sub: int = 8) -> SystemSpec:
    """Two layers (0 and 6 km) on n x n grids and two 8x8 WFS (one NGS, one LGS at 90 km);
    small enough to assemble every operator densely."""
    rng = np.random.default_rng(seed)
    D = 4.0
    mask = subaperture_mask(n_sub, D, 0.2)
    wfs = [WfsSpec(n_sub, D / n_sub, 0.0, 0.0, 0.0, mask.copy()),
           WfsSpec(n_sub, D / n_sub, 20.0 * ARCSEC, -10.0 * ARCSEC, 90000.0, mask.copy())]
    layers = [LayerSpec(0.0, 0.6, n, levels, wind=(3.0, 1.0)),
              LayerSpec(6000.0, 0.4, n, levels, wind=(-2.0, 4.0))]
    spec = SystemSpec("tiny", D, 0.2, layers, wfs, alpha=2.0, r0=0.15, L0=25.0, max_iter=4,
                      recycle_k=3, precision="fp64")
    spec = fit_layer_grids(spec)
    for w in spec.wfs:   # seeded positive weights (inverse noise variance), zero where masked
        m = np.concatenate([w.mask.ravel(), w.mask.ravel()])
        w.weight = np.where(m, rng.uniform(0.5, 2.0, size=m.size), 0.0)
    return spec


def config_mixed(seed: int = 4) -> SystemSpec:
    """Edge-case mix: layers of different grid sizes and level counts (one transformed down
    to a 1x1 approximation), low-order 1x1 and 2x2 natural guide stars, a ragged 19x19
    laser-guide-star sensor."""
    rng = np.random.default_rng(seed)
    D = 6.0
    wfs = []
    for ns, th, H in ((19, (15.0, 10.0), 90000.0), (1, (-20.0, 5.0), 0.0), (2, (5.0, -25.0), 0.0),
                      (19, (0.0, 0.0), 0.0)):
        mask = subaperture_mask(ns, D, 0.1 if ns > 2 else 0.0)
        wfs.append(WfsSpec(ns, D / ns, th[0] * ARCSEC, th[1] * ARCSEC, H, mask))
    layers = [LayerSpec(0.0, 0.5, 32, 5), LayerSpec(3000.0, 0.3, 16, 4), LayerSpec(9000.0, 0.2, 32, 2)]
    spec = SystemSpec("mixed", D, 0.1, layers, wfs, alpha=1.5, r0=0.14, L0=30.0, max_iter=5,
                      recycle_k=7, precision="fp64")
    spec = fit_layer_grids(spec)
    for w in spec.wfs:
        m = np.concatenate([w.mask.ravel(), w.mask.ravel()])
        w.weight = np.where(m, rng.uniform(0.5, 2.0, size=m.size), 0.0)
    return spec


def config_random_instance(rng: np.random.Generator, precision: str = "fp32") -> SystemSpec:
    """One instance of a ragged batch: telescope 8-39 m, 20-84 subapertures, 3-9 layers,
    1-6 guide stars mixing NGS and LGS, grids the next power of two of E / d_s (<= 256)."""
    D = float(rng.uniform(8.0, 39.0))
    ns = int(rng.integers(20, 85))
    L = int(rng.integers(3, 10))
    G = int(rng.integers(1, 7))
    mask = subaperture_mask(ns, D, float(rng.choice([0.0, 0.28])))
    wfs = []
    for g in range(G):
        lgs = bool(rng.random() < 0.5)
        rad = (45.0 if lgs else 60.0) * ARCSEC * (0.0 if g == 0 and not lgs else 1.0)
        a = rng.uniform(0, 2 * np.pi)
        wfs.append(WfsSpec(ns, D / ns, rad * np.cos(a), rad * np.sin(a),
                           90000.0 if lgs else 0.0, mask.copy()))
    hs = np.sort(np.concatenate([[0.0], rng.uniform(500.0, 16000.0, size=L - 1)]))
    gam = np.exp(-hs / 4000.0)
    gam /= gam.sum()
    layers = []
    for h, gm in zip(hs, gam):
        ext = np.array([_projected_extent(w, h) for w in wfs])
        E = max(ext[:, 1].max() - ext[:, 0].min(), ext[:, 3].max() - ext[:, 2].min())
        n = 16
        while n < 256 and n - 2 < E / (D / ns):
            n *= 2
        lv = int(min(6, np.log2(n) - 1))
        layers.append(LayerSpec(float(h), float(gm), n, lv, wind=tuple(rng.uniform(-15, 15, 2))))
    spec = SystemSpec("random", D, 0.0, layers, wfs, alpha=2.0, r0=0.129, L0=25.0,
                      max_iter=200, recycle_k=10, rel_tol=1e-4, precision=precision)
    return fit_layer_grids(spec)
