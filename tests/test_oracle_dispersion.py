"""Interior-scheme pin: in a periodic homogeneous box a discrete P or S plane wave is an
exact eigenmode of the staggered O(2,4) scheme, with sin(w dt/2) = (v dt/2) |K| where
K is the Eq.(4) modified wavenumber per axis (each axis with its own spacing).  Every
field, both operators, the staggering and the sign of each term enter; a dropped or
misplaced term, or a spacing taken from the wrong axis, fails."""
import numpy as np
import pytest

import oracle
from helpers import coords, modified_wavenumber

SHAPE = (16, 12, 10)
H = 10.0
ANISO = (10.0, 7.5, 12.5)  # dx, dy, dz
DT = 1e-3
LAM, MU, RHO = 2500.0 * (3000.0 ** 2 - 2 * 1732.0 ** 2), 2500.0 * 1732.0 ** 2, 2500.0


def spacing(h):
    return (h, h, h) if np.ndim(h) == 0 else tuple(h)


def mode(kvec, pol, t_v, t_s, omega, h=H):
    """Fields of Re(F e^{i(k.x - w t)}): v at time t_v, sigma at t_s."""
    Kv = np.array([modified_wavenumber(k, ha) for k, ha in zip(kvec, spacing(h))])
    wt = (2.0 / DT) * np.sin(omega * DT / 2.0)  # discrete time-derivative symbol
    V = pol
    S = np.zeros((3, 3), dtype=complex)
    kv = np.dot(Kv, V)
    for i in range(3):
        for j in range(3):
            S[i, j] = -(LAM * (i == j) * kv + MU * (Kv[i] * V[j] + Kv[j] * V[i])) / wt
    amp = [V[0], V[1], V[2], S[0, 0], S[1, 1], S[2, 2], S[0, 1], S[0, 2], S[1, 2]]
    nx, ny, nz = SHAPE
    st = np.zeros((9, nz, ny, nx))
    for c in range(9):
        x, y, z = coords(c, SHAPE, h)
        t = t_v if c < 3 else t_s
        ph = kvec[0] * x + kvec[1] * y + kvec[2] * z - omega * t
        st[c] = np.real(amp[c] * np.exp(1j * ph))
    return st


@pytest.mark.parametrize("h", [H, ANISO])
@pytest.mark.parametrize("wave", ["P", "S"])
@pytest.mark.parametrize("m", [(1, 0, 0), (0, 2, 1), (3, 2, 2), (5, 4, 3)])
def test_periodic_plane_wave(wave, m, h):
    nx, ny, nz = SHAPE
    hx, hy, hz = spacing(h)
    kvec = 2 * np.pi * np.array([m[0] / (nx * hx), m[1] / (ny * hy), m[2] / (nz * hz)])
    Kv = np.array([modified_wavenumber(k, ha) for k, ha in zip(kvec, (hx, hy, hz))])
    Kn = np.linalg.norm(Kv)
    if wave == "P":
        pol = Kv / Kn
        v = np.sqrt((LAM + 2 * MU) / RHO)
    else:
        a = np.cross(Kv / Kn, [0.3, -0.7, 0.64])
        pol = a / np.linalg.norm(a)
        v = np.sqrt(MU / RHO)
    omega = (2.0 / DT) * np.arcsin(DT * v * Kn / 2.0)
    nt = 37
    st0 = mode(kvec, pol, -DT / 2, 0.0, omega, h)
    want = mode(kvec, pol, (nt - 0.5) * DT, nt * DT, omega, h)
    cfg = oracle.Config(SHAPE, h, DT, nt, periodic=(True, True, True))
    shape = (nz, ny, nx)
    _, st = oracle.forward(cfg, np.full(shape, LAM), np.full(shape, MU), np.full(shape, RHO), state=st0)
    for c in range(9):
        scale = np.max(np.abs(want[c])) + np.max(np.abs(want[:3] if c < 3 else want[3:])) * 1e-3
        err = np.max(np.abs(st[c] - want[c]))
        assert err <= 1e-12 * scale, (c, err, scale)


def test_wrong_speed_fails():
    """Guard on the check itself: the continuum dispersion relation (no modified
    wavenumber) does not satisfy the scheme."""
    nx, ny, nz = SHAPE
    m = (3, 2, 2)
    kvec = 2 * np.pi * np.array([m[0] / (nx * H), m[1] / (ny * H), m[2] / (nz * H)])
    pol = kvec / np.linalg.norm(kvec)
    v = np.sqrt((LAM + 2 * MU) / RHO)
    omega = v * np.linalg.norm(kvec)
    nt = 37
    st0 = mode(kvec, pol, -DT / 2, 0.0, omega)
    want = mode(kvec, pol, (nt - 0.5) * DT, nt * DT, omega)
    cfg = oracle.Config(SHAPE, H, DT, nt, periodic=(True, True, True))
    shape = (nz, ny, nx)
    _, st = oracle.forward(cfg, np.full(shape, LAM), np.full(shape, MU), np.full(shape, RHO), state=st0)
    assert np.max(np.abs(st[0] - want[0])) > 1e-6 * np.max(np.abs(want[0]))


def test_spacing_from_the_wrong_axis_fails():
    """Guard: the anisotropic mode is not reproduced when the oracle is given the
    spacings in another order."""
    nx, ny, nz = SHAPE
    hx, hy, hz = ANISO
    m = (3, 2, 2)
    kvec = 2 * np.pi * np.array([m[0] / (nx * hx), m[1] / (ny * hy), m[2] / (nz * hz)])
    Kv = np.array([modified_wavenumber(k, ha) for k, ha in zip(kvec, ANISO)])
    pol = Kv / np.linalg.norm(Kv)
    v = np.sqrt((LAM + 2 * MU) / RHO)
    omega = (2.0 / DT) * np.arcsin(DT * v * np.linalg.norm(Kv) / 2.0)
    nt = 37
    st0 = mode(kvec, pol, -DT / 2, 0.0, omega, ANISO)
    want = mode(kvec, pol, (nt - 0.5) * DT, nt * DT, omega, ANISO)
    cfg = oracle.Config(SHAPE, (hy, hz, hx), DT, nt, periodic=(True, True, True))
    shape = (nz, ny, nx)
    _, st = oracle.forward(cfg, np.full(shape, LAM), np.full(shape, MU), np.full(shape, RHO), state=st0)
    assert np.max(np.abs(st[0] - want[0])) > 1e-6 * np.max(np.abs(want[0]))
