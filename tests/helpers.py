"""Test-side helpers: staggered positions (Sec. 2.1.1), pinned-slot masks, discrete
energy, plane-wave modes and comparison metrics.  Independent of both the oracle
and the HIP library."""
from __future__ import annotations

import numpy as np

FIELDS = ("vx", "vy", "vz", "sxx", "syy", "szz", "sxy", "sxz", "syz")
# half-offset flags (x, y, z) per component, Sec. 2.1.1
STAG = np.array([
    [1, 0, 0], [0, 1, 0], [0, 0, 1],
    [0, 0, 0], [0, 0, 0], [0, 0, 0],
    [1, 1, 0], [1, 0, 1], [0, 1, 1],
])


def active_mask(comp: int, shape_xyz, periodic=(False, False, False)) -> np.ndarray:
    """Boolean [nz,ny,nx]: samples that are not pinned (a staggered axis has n-1)."""
    nx, ny, nz = shape_xyz
    m = np.ones((nz, ny, nx), dtype=bool)
    s = STAG[comp]
    if s[0] and not periodic[0]:
        m[:, :, nx - 1] = False
    if s[1] and not periodic[1]:
        m[:, ny - 1, :] = False
    if s[2] and not periodic[2]:
        m[nz - 1, :, :] = False
    return m


def coords(comp: int, shape_xyz, h):
    """(X, Y, Z) coordinates in metres of every sample of a component, [nz,ny,nx]; h is
    one spacing or (dx, dy, dz)."""
    nx, ny, nz = shape_xyz
    hx, hy, hz = (h, h, h) if np.ndim(h) == 0 else h
    s = STAG[comp]
    z, y, x = np.meshgrid((np.arange(nz) + 0.5 * s[2]) * hz, (np.arange(ny) + 0.5 * s[1]) * hy,
                          (np.arange(nx) + 0.5 * s[0]) * hx, indexing="ij")
    return x, y, z


def random_state(shape_xyz, rng, periodic=(False, False, False), vscale=1e-3, sscale=1e4) -> np.ndarray:
    nx, ny, nz = shape_xyz
    st = rng.standard_normal((9, nz, ny, nx))
    st[:3] *= vscale
    st[3:] *= sscale
    for c in range(9):
        st[c][~active_mask(c, shape_xyz, periodic)] = 0.0
    return st


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b.ravel())
    if nb == 0.0:
        return float(np.linalg.norm(a.ravel()))
    return float(np.linalg.norm((a - b).ravel()) / nb)


def discrete_energy(v_prev, state, lam, mu, rho, shape_xyz):
    """E^n = 1/2 sum rho_eff v^{n-1/2} . v^{n+1/2} + 1/2 sum sigma^n : C^{-1} sigma^n over
    active samples, with rho_eff the two-node mean and mu_eff the four-node mean
    (Sec. 2.2.1).  v_prev: [3,...] = v^{n-1/2}; state[:3] = v^{n+1/2}; state[3:] = sigma^n."""
    e = 0.0
    for c in range(3):
        ax = 2 - c  # numpy axis of x is 2
        r = rho.copy()
        rn = np.roll(rho, -1, axis=ax)
        reff = 0.5 * (r + rn)
        m = active_mask(c, shape_xyz)
        e += 0.5 * np.sum((reff * v_prev[c] * state[c])[m])
    sxx, syy, szz = state[3], state[4], state[5]
    # inverse of the isotropic normal block [[l+2m, l, l], [l, l+2m, l], [l, l, l+2m]]
    K = lam + 2.0 * mu / 3.0
    p = (sxx + syy + szz) / 3.0
    dxx, dyy, dzz = sxx - p, syy - p, szz - p
    e += 0.5 * np.sum(p * p / K + (dxx * dxx + dyy * dyy + dzz * dzz) / (2.0 * mu))
    for c, axes in ((6, (2, 1)), (7, (2, 0)), (8, (1, 0))):
        a0, a1 = axes
        m00 = mu
        m10 = np.roll(mu, -1, axis=a0)
        m01 = np.roll(mu, -1, axis=a1)
        m11 = np.roll(np.roll(mu, -1, axis=a0), -1, axis=a1)
        meff = ((m00 + m10) + (m01 + m11)) / 4.0
        m = active_mask(c, shape_xyz)
        e += 0.5 * np.sum((state[c] ** 2 / meff)[m])
    return e


def modified_wavenumber(k, h):
    """Fourier symbol of the Eq.(4) staggered derivative: (2/h)(9/8 sin(kh/2) - 1/24 sin(3kh/2))."""
    return (2.0 / h) * (9.0 / 8.0 * np.sin(k * h / 2.0) - 1.0 / 24.0 * np.sin(3.0 * k * h / 2.0))
