"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds input generators only (models, wavelets, source mechanisms,
receiver layouts and the five named workloads); none of the finite-difference
method's arithmetic lives here.  Every random draw uses
``numpy.random.Generator(PCG64(seed))`` with ``seed = 1000 + workload index
(+ shot index)``.

Units are SI: m, s, kg/m^3, Pa, N m.  Arrays are float64 ``[nz, ny, nx]``
(x fastest, z down).  Positions are in grid units (x, y, z).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

# ---------------------------------------------------------------- wavelets


def ricker(f0: float, nt: int, dt: float, t0: Optional[float] = None, at_half: bool = True) -> np.ndarray:
    """Ricker wavelet sampled per step.

    Moment-tensor sources use it as the moment rate (unit peak, s^-1 scaled by M0
    in the mechanism) sampled at t = (n + 1/2) dt (``at_half``); force sources at
    t = n dt.  The delay defaults to t0 = 1.5 / f0.
    """
    if t0 is None:
        t0 = 1.5 / f0
    t = (np.arange(nt) + (0.5 if at_half else 0.0)) * dt - t0
    a = (np.pi * f0 * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


# ---------------------------------------------------------------- models


def homogeneous(shape_xyz: Sequence[int], vp: float = 3000.0, vs: float = 1732.0, rho: float = 2500.0):
    nx, ny, nz = shape_xyz
    r = np.full((nz, ny, nx), rho)
    mu = r * vs * vs
    lam = r * vp * vp - 2.0 * mu
    return lam, mu, r


def gaussian_field(shape_zyx, corr_len: float, h: float, rng: np.random.Generator) -> np.ndarray:
    """Unit-variance Gaussian-correlated field: white N(0,1) smoothed by a separable
    Gaussian of standard deviation corr_len / 2 (covariance ~ exp(-r^2 / corr_len^2)),
    renormalised to unit standard deviation and clipped to +-3."""
    from scipy.ndimage import gaussian_filter

    w = rng.standard_normal(size=shape_zyx, dtype=np.float32)
    g = gaussian_filter(w, sigma=(corr_len / 2.0) / h, mode="reflect")
    g = g.astype(np.float64)
    g /= g.std()
    return np.clip(g, -3.0, 3.0)


LAYER_VP = (1500.0, 2200.0, 2900.0, 3600.0, 4300.0, 5000.0)


def layered_perturbed(shape_xyz: Sequence[int], h: float, seed: int, pert: float = 0.05,
                      corr_len: float = 50.0, layers: Sequence[float] = LAYER_VP):
    """Six equal-thickness horizontal layers (vp increasing with depth), times
    (1 + pert * xi) with xi Gaussian-correlated; vs = vp / sqrt(3); Gardner density
    rho = 310 vp^0.25 (SI).  Returns (lam, mu, rho)."""
    nx, ny, nz = shape_xyz
    rng = np.random.Generator(np.random.PCG64(seed))
    k = np.arange(nz)
    layer = np.minimum(k * len(layers) // nz, len(layers) - 1)
    vp1d = np.asarray(layers)[layer]
    xi = gaussian_field((nz, ny, nx), corr_len, h, rng)
    vp = vp1d[:, None, None] * (1.0 + pert * xi)
    return elastic_from_vp(vp)


def elastic_from_vp(vp: np.ndarray):
    vs = vp / np.sqrt(3.0)
    rho = 310.0 * vp ** 0.25
    mu = rho * vs * vs
    lam = rho * vp * vp - 2.0 * mu
    return lam, mu, rho


def smoothed(lam, mu, rho, sigma_m: float, h: float):
    """Starting model: Gaussian smoothing (std sigma_m, reflect edges) of vp, vs and rho,
    then converted back to (lam, mu, rho)."""
    from scipy.ndimage import gaussian_filter

    vp = np.sqrt((lam + 2.0 * mu) / rho)
    vs = np.sqrt(mu / rho)
    s = sigma_m / h
    vp, vs, r = (gaussian_filter(a, sigma=s, mode="reflect") for a in (vp, vs, rho))
    mu2 = r * vs * vs
    return r * vp * vp - 2.0 * mu2, mu2, r


# ---------------------------------------------------------------- mechanisms


def explosion(m0: float = 1e15):
    return (m0, m0, m0, 0.0, 0.0, 0.0)


def random_mt(rng: np.random.Generator, scale: float = 1e15):
    """Symmetric moment tensor with independent N(0,1) * scale entries."""
    m = rng.standard_normal(6) * scale
    return tuple(float(v) for v in m)  # Mxx Myy Mzz Mxy Mxz Myz


def double_couple(strike: float, dip: float, rake: float, m0: float = 1e15):
    """Double couple from strike/dip/rake (radians); x north, y east, z down
    (Aki & Richards 2002, Box 4.4)."""
    s, d, r = strike, dip, rake
    mxx = -m0 * (np.sin(d) * np.cos(r) * np.sin(2 * s) + np.sin(2 * d) * np.sin(r) * np.sin(s) ** 2)
    mxy = m0 * (np.sin(d) * np.cos(r) * np.cos(2 * s) + 0.5 * np.sin(2 * d) * np.sin(r) * np.sin(2 * s))
    mxz = -m0 * (np.cos(d) * np.cos(r) * np.cos(s) + np.cos(2 * d) * np.sin(r) * np.sin(s))
    myy = m0 * (np.sin(d) * np.cos(r) * np.sin(2 * s) - np.sin(2 * d) * np.sin(r) * np.cos(s) ** 2)
    myz = -m0 * (np.cos(d) * np.cos(r) * np.sin(s) - np.cos(2 * d) * np.sin(r) * np.cos(s))
    mzz = m0 * np.sin(2 * d) * np.sin(r)
    return tuple(float(v) for v in (mxx, myy, mzz, mxy, mxz, myz))


# ---------------------------------------------------------------- receivers


def receiver_grid(xs: Sequence[float], ys: Sequence[float], z: float) -> np.ndarray:
    """[nrec, 3] positions: every (x, y) pair at depth z (x fastest)."""
    X, Y = np.meshgrid(np.asarray(xs, float), np.asarray(ys, float), indexing="xy")
    return np.stack([X.ravel(), Y.ravel(), np.full(X.size, float(z))], axis=1)


# ---------------------------------------------------------------- named workloads


@dataclass
class Shot:
    """One simulation: model, grid, time stepping, source and receivers."""

    name: str
    shape: Tuple[int, int, int]  # nx, ny, nz
    h: float
    dt: float
    nt: int
    lam: np.ndarray
    mu: np.ndarray
    rho: np.ndarray
    src_pos: Tuple[float, float, float]
    moment: Tuple[float, ...]
    force: Tuple[float, float, float]
    wavelet: np.ndarray
    rec_pos: np.ndarray
    sponge: Tuple[int, ...] = (20,) * 6
    alpha: float = 0.0
    free_surface: bool = False

    @property
    def cells(self) -> int:
        return int(np.prod(self.shape))


def c0(nt: int = 500) -> Shot:
    """64^3 homogeneous (vp 3000, vs 1732, rho 2500), h 10 m, dt 1 ms; explosion M0 1e15
    at the centre node, 10 Hz Ricker moment rate; 20-cell sponge; 16 receivers on a line."""
    shape = (64, 64, 64)
    lam, mu, rho = homogeneous(shape)
    rec = np.stack([np.arange(24, 40, dtype=float), np.full(16, 36.0), np.full(16, 38.0)], axis=1)
    return Shot("c0", shape, 10.0, 1e-3, nt, lam, mu, rho, (32.0, 32.0, 32.0), explosion(1e15),
                (0.0, 0.0, 0.0), ricker(10.0, nt, 1e-3), rec)


def c1(nt: int = 2000, shape=(256, 256, 256)) -> Shot:
    """256^3 six-layer model + 5 % Gaussian-correlated perturbation (50 m), h 10 m,
    dt 0.5 ms; random symmetric moment tensor at the centre, 12 Hz Ricker; 16 x 16
    receivers at z = 22 just under the 20-cell sponge."""
    seed = 1001
    lam, mu, rho = layered_perturbed(shape, 10.0, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 500))
    mt = random_mt(rng)
    nx, ny, nz = shape
    rec = receiver_grid(np.linspace(24, nx - 25, 16), np.linspace(24, ny - 25, 16), 22.0)
    return Shot("c1", tuple(shape), 10.0, 5e-4, nt, lam, mu, rho, (nx / 2, ny / 2, nz / 2), mt,
                (0.0, 0.0, 0.0), ricker(12.0, nt, 5e-4), rec)


def c2(nt: int = 4000, shape=(512, 512, 256)) -> Shot:
    """512 x 512 x 256, the same generator; free surface on top and a 30-cell sponge on
    the other five faces; seeded double couple (M0 1e15), 8 Hz Ricker, dt 0.6 ms;
    32 x 32 receivers at z = 1 under the surface."""
    seed = 1002
    lam, mu, rho = layered_perturbed(shape, 10.0, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 500))
    strike, dip, rake = rng.uniform(0, 2 * np.pi), rng.uniform(0.1, np.pi / 2), rng.uniform(-np.pi, np.pi)
    nx, ny, nz = shape
    rec = receiver_grid(np.linspace(34, nx - 35, 32), np.linspace(34, ny - 35, 32), 1.0)
    return Shot("c2", tuple(shape), 10.0, 6e-4, nt, lam, mu, rho, (nx / 2, ny / 2, nz / 2),
                double_couple(strike, dip, rake), (0.0, 0.0, 0.0), ricker(8.0, nt, 6e-4), rec,
                sponge=(30, 30, 30, 30, 0, 30), free_surface=True)


C3_SIZES = ((128, 128, 128), (192, 192, 128), (256, 256, 128))


def c3(nshots: int = 24, nt: int = 1500) -> List[Shot]:
    """24 shots with sizes drawn from {128^3, 192x192x128, 256x256x128}, each with its
    own seeded layered + perturbed model; explosions near the surface, 10 Hz Ricker;
    16 x 8 receivers at z = 22; dt 0.5 ms; 20-cell sponge."""
    base = 1003
    rng = np.random.Generator(np.random.PCG64(base))
    shots = []
    for s in range(nshots):
        shape = C3_SIZES[int(rng.integers(0, len(C3_SIZES)))]
        nx, ny, nz = shape
        lam, mu, rho = layered_perturbed(shape, 10.0, base + 1 + s)
        sx = float(rng.uniform(30, nx - 31))
        sy = float(rng.uniform(30, ny - 31))
        sz = float(22 + int(rng.integers(0, 4)))
        rec = receiver_grid(np.linspace(24, nx - 25, 16), np.linspace(24, ny - 25, 8), 22.0)
        shots.append(Shot(f"c3_{s}", shape, 10.0, 5e-4, nt, lam, mu, rho, (sx, sy, sz), explosion(1e15),
                          (0.0, 0.0, 0.0), ricker(10.0, nt, 5e-4), rec))
    return shots


def c4_models(shape=(256, 256, 256)):
    """True model = the 256^3 layered + perturbed generator; starting model = its
    Gaussian smoothing with a 200 m standard deviation."""
    true = layered_perturbed(shape, 10.0, 1001)
    start = smoothed(*true, sigma_m=200.0, h=10.0)
    return true, start


def c4_shots(lam, mu, rho, nt: int = 1500, shape=(256, 256, 256), nshots: int = 8) -> List[Shot]:
    """Eight explosions on a 4 x 2 grid at z = 24, 10 Hz Ricker, 16 x 16 receivers at
    z = 22, dt 0.5 ms, checkpoints every 50 steps (chosen by the caller)."""
    nx, ny, nz = shape
    xs = np.linspace(48, nx - 49, 4)
    ys = np.linspace(64, ny - 65, 2)
    rec = receiver_grid(np.linspace(24, nx - 25, 16), np.linspace(24, ny - 25, 16), 22.0)
    shots = []
    for s in range(nshots):
        sx, sy = float(xs[s % 4]), float(ys[(s // 4) % 2])
        shots.append(Shot(f"c4_{s}", tuple(shape), 10.0, 5e-4, nt, lam, mu, rho, (sx, sy, 24.0),
                          explosion(1e15), (0.0, 0.0, 0.0), ricker(10.0, nt, 5e-4), rec))
    return shots


def small_fd_case(seed: int = 1004, shape=(32, 32, 32), nt: int = 300):
    """32^3 FP64 finite-difference check: a perturbed two-layer model, 2 explosive shots,
    16 receivers, 6-cell sponge with alpha 0.05."""
    nx, ny, nz = shape
    rng = np.random.Generator(np.random.PCG64(seed))
    vp = np.where(np.arange(nz) < nz // 2, 2500.0, 3200.0)[:, None, None] * np.ones((nz, ny, nx))
    vp = vp * (1.0 + 0.03 * gaussian_field((nz, ny, nx), 30.0, 10.0, rng))
    lam, mu, rho = elastic_from_vp(vp)
    rec = receiver_grid(np.linspace(8, nx - 9, 4), np.linspace(8, ny - 9, 4), 8.0)
    srcs = [(11.3, 13.6, 10.2), (20.7, 17.1, 9.8)]
    return lam, mu, rho, srcs, rec
