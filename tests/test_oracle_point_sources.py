"""Pins of the oracle's point operators against what the mathematics fixes.

* Point force (the force term f of Eq.(1), Sec. 2.1) against Stokes' full-space solution
  (Aki & Richards 2002 eq. 4.23, near field included), along z and along x.
* Off-diagonal moment-tensor sources (Eq.(7) of the paper gives the tensor; here pure
  Mxy and pure Mxz) against the general moment-tensor solution (Aki & Richards eq. 4.29:
  near, intermediate and far fields).
* Trilinear receivers (Sec. 2.4) reproduce fields linear in x, y, z exactly at
  off-sample points on each velocity component's own subgrid, and point injection is
  the transpose of that sampling at off-sample points, for every component.

The closed forms are checked first against each other and against quadrature, so that
a slip in writing one of them out cannot pass unnoticed: the moment-tensor field must
equal minus the spatial derivative of the force field, M = M0 I must give the
explosion, and the near-field integrals must match numerical quadrature.

Sources sit exactly on a sample of the component they drive and every receiver on a
sample of the component it is compared on, so no interpolation enters the closed-form
comparisons.  Homogeneous medium, no damping, and a window that ends before the first
return from the grid faces reaches any receiver.
"""
import numpy as np
import pytest
from scipy.integrate import quad

import oracle
import workloads as W
from oracle import analytic as A

VP, VS, RHO = 3000.0, 1732.0, 2500.0
F0 = 10.0
T0 = 1.2 / F0
# staggering offsets (grid units) of vx vy vz sxx syy szz sxy sxz syz, Sec. 2.1.1
STAG = [(0.5, 0, 0), (0, 0.5, 0), (0, 0, 0.5), (0, 0, 0), (0, 0, 0), (0, 0, 0), (0.5, 0.5, 0), (0.5, 0, 0.5),
        (0, 0.5, 0.5)]
DIRS = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1), (1, 1, 1), (1, -1, 1), (-1, 1, 1)]
DISTS = (100.0, 140.0)


def _closed_form_error(n, h, dt, nt, kind, value, comp):
    """rel-L2 of the oracle's receiver velocities against the closed form, over every
    receiver (each velocity component on its own samples, nine directions, two
    distances) and every sample of the window."""
    shape = (n, n, n)
    lam, mu, rho = W.homogeneous(shape, VP, VS, RHO)
    c = np.full(3, float(n // 2))
    spos = c + np.array(STAG[comp])
    cfg = oracle.Config(shape, h, dt, nt, sponge=(0,) * 6)
    if kind == "force":
        # force history sampled at n dt; the velocity field is 4.23 with its derivative
        wav = W.ricker(F0, nt, dt, t0=T0, at_half=False)
        src = oracle.Source(tuple(spos), force=value)
        hist, field = A.History(F0, T0, 1), A.force_field
    else:
        # moment rate sampled at (n + 1/2) dt; the velocity field is 4.29 with the rate
        wav = W.ricker(F0, nt, dt, t0=T0)
        src = oracle.Source(tuple(spos), moment=value)
        hist, field = A.History(F0, T0, 0), A.moment_field
    recs, comps = [], []
    for rc in range(3):
        st = np.array(STAG[rc])
        for d in DIRS:
            d = np.asarray(d, float) / np.linalg.norm(d)
            for r in DISTS:
                recs.append(np.round(c + d * r / h - st) + st)
                comps.append(rc)
    recs = np.array(recs)
    tr, _ = oracle.forward(cfg, lam, mu, rho, src, wav, recs)
    times = (np.arange(nt) + 0.5) * dt  # receivers record v^{n+1/2}
    num = den = 0.0
    for q, (p, rc) in enumerate(zip(recs, comps)):
        want = field((p - spos) * h, times, value, RHO, VP, VS, hist)[rc]
        num += np.sum((tr[q, rc] - want) ** 2)
        den += np.sum(want ** 2)
    return float(np.sqrt(num / den))


def _fine(kind, value, comp):
    # 10 m cells, 1 ms; the first face return reaches a receiver after (2 * 400 - 140) m / vp
    return _closed_form_error(80, 10.0, 1e-3, 220, kind, value, comp)


def _coarse(kind, value, comp):
    return _closed_form_error(40, 20.0, 2e-3, 110, kind, value, comp)


# ---------------------------------------------------------------- the closed forms


def test_near_field_integral_matches_quadrature():
    for order in (0, 1):
        h = A.History(F0, T0, order)
        for t in (0.05, 0.13, 0.2, 0.31):
            a, b = 0.03, 0.06
            want = quad(lambda tau: tau * h.g(t - tau), a, b, epsabs=1e-15, epsrel=1e-12)[0]
            got = A.near_integral(h, np.array([t]), a, b)[0]
            assert abs(got - want) <= 1e-10 * max(abs(want), 1e-12)


def test_moment_field_is_minus_gradient_of_force_field():
    """u^M_n = -M_pq d/dx_q u^{F = e_p}_n for the same history (the equivalent forces of
    a moment tensor), checked by central differences of the 4.23 implementation."""
    h = A.History(F0, T0, 0)
    t = np.linspace(0.0, 0.3, 301)
    M = np.array([[1.0, 0.3, -0.7], [0.3, -0.4, 0.5], [-0.7, 0.5, 0.9]]) * 1e15
    for x in (np.array([60.0, -45.0, 80.0]), np.array([-20.0, 130.0, 15.0])):
        got = A.moment_field(x, t, M, RHO, VP, VS, h)
        num = np.zeros_like(got)
        eps = 1e-3
        for p in range(3):
            for q in range(3):
                e = np.zeros(3)
                e[q] = eps
                F = np.zeros(3)
                F[p] = 1.0
                d = (A.force_field(x + e, t, F, RHO, VP, VS, h) - A.force_field(x - e, t, F, RHO, VP, VS, h)) / (2 * eps)
                num -= M[p, q] * d
        assert np.abs(got - num).max() <= 1e-7 * np.abs(got).max()


def test_isotropic_moment_field_is_the_explosion():
    h = A.History(F0, T0, 0)
    t = np.linspace(0.0, 0.3, 301)
    x = np.array([60.0, -45.0, 80.0])
    r = np.linalg.norm(x)
    got = A.moment_field(x, t, 1e15 * np.eye(3), RHO, VP, VS, h)
    want = A.explosion_vr(r, t, 1e15, RHO, VP, F0, T0)[None, :] * (x / r)[:, None]
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_force_velocity_is_time_derivative_of_displacement():
    x = np.array([60.0, -45.0, 80.0])
    F = np.array([0.2, -0.5, 1.0])
    t = np.linspace(0.0, 0.3, 301)
    v = A.force_field(x, t, F, RHO, VP, VS, A.History(F0, T0, 1))
    e = 1e-6
    u = lambda s: A.force_field(x, s, F, RHO, VP, VS, A.History(F0, T0, 0))
    assert np.abs(v - (u(t + e) - u(t - e)) / (2 * e)).max() <= 1e-7 * np.abs(v).max()


# ---------------------------------------------------------------- the oracle against them


def test_point_force_z_stokes_and_convergence():
    """Fz at a vz sample: < 1 % at 10 m, and the error falls >= 4x when h and dt halve."""
    fine = _fine("force", (0.0, 0.0, 1e9), 2)
    coarse = _coarse("force", (0.0, 0.0, 1e9), 2)
    assert fine < 0.01, fine
    assert coarse < 0.06, coarse
    assert coarse / fine >= 4.0, (coarse, fine)


def test_point_force_x_stokes():
    err = _fine("force", (1e9, 0.0, 0.0), 0)
    assert err < 0.01, err


@pytest.mark.parametrize("q,comp", [(3, 6), (4, 7)], ids=["Mxy", "Mxz"])
def test_off_diagonal_moment_closed_form_and_convergence(q, comp):
    """Pure Mxy at a sxy sample and pure Mxz at a sxz sample: the full 4.29 field (near,
    intermediate, far P and S) to < 1 % at 10 m, error falling >= 4x when h and dt halve.
    A flipped sign or a factor of two on the off-diagonal injection misses by >= 50 %."""
    m = [0.0] * 6
    m[q] = 1e15
    fine = _fine("moment", tuple(m), comp)
    coarse = _coarse("moment", tuple(m), comp)
    assert fine < 0.01, fine
    assert coarse < 0.06, coarse
    assert coarse / fine >= 4.0, (coarse, fine)


# ---------------------------------------------------------------- trilinear point operators


def _sample_coords(shape, comp):
    """True coordinates (grid units) of every storage slot of a component: (X, Y, Z) [nz, ny, nx]."""
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    s = STAG[comp]
    return x + s[0], y + s[1], z + s[2]


def _active_mask(shape, comp):
    nx, ny, nz = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    s = STAG[comp]
    return (x <= nx - 1 - (s[0] > 0)) & (y <= ny - 1 - (s[1] > 0)) & (z <= nz - 1 - (s[2] > 0))


COEF = [(0.7, -1.3, 2.1, 0.4), (-0.2, 0.9, 0.5, -1.7), (1.1, 0.3, -0.8, 2.6)]


def test_receivers_exact_on_linear_fields_off_sample():
    """One step from a state whose velocities are linear in the sample's true coordinate
    (stresses zero, no damping, no source, so the velocity pass leaves them unchanged):
    every receiver, at points off every subgrid, records a + b.p exactly for each
    component.  Wrong staggering offsets or wrong weights miss by O(1)."""
    shape = (12, 11, 10)
    nx, ny, nz = shape
    lam, mu, rho = W.homogeneous(shape)
    st = np.zeros((9, nz, ny, nx))
    for comp in range(3):
        X, Y, Z = _sample_coords(shape, comp)
        a, bx, by, bz = COEF[comp]
        st[comp] = np.where(_active_mask(shape, comp), a + bx * X + by * Y + bz * Z, 0.0)
    rng = np.random.Generator(np.random.PCG64(77))
    rec = np.column_stack([rng.uniform(2.2, nx - 3.2, 40), rng.uniform(2.2, ny - 3.2, 40),
                           rng.uniform(2.2, nz - 3.2, 40)])
    rec[:4] = [[4.25, 5.0, 3.5], [5.5, 5.5, 5.5], [6.0, 3.75, 4.0], [3.1, 6.9, 5.3]]
    cfg = oracle.Config(shape, 10.0, 1e-3, 1, sponge=(0,) * 6)
    tr, _ = oracle.forward(cfg, lam, mu, rho, None, None, rec, state=st)
    for comp in range(3):
        a, bx, by, bz = COEF[comp]
        want = a + bx * rec[:, 0] + by * rec[:, 1] + bz * rec[:, 2]
        np.testing.assert_allclose(tr[:, comp, 0], want, rtol=0, atol=1e-12)


def test_injection_is_transpose_of_sampling_off_sample():
    """One step from zero with a force (then a moment) source at an off-sample point, no
    damping: the injected field has total dt b F s / (dx dy dz) per component (moment:
    -dt M s / (dx dy dz)) and its first moments put it exactly at the source point on
    every component's subgrid, i.e. <inject(p), f> = f(p) for every linear f."""
    shape = (12, 11, 10)
    nx, ny, nz = shape
    lam, mu, rho = W.homogeneous(shape)
    h = (10.0, 12.0, 8.0)
    dt, s0 = 1e-4, 0.75
    vol = h[0] * h[1] * h[2]
    p = np.array([5.3, 4.7, 4.15])
    cfg = oracle.Config(shape, h, dt, 1, sponge=(0,) * 6)
    force = (2e9, -3e9, 5e9)
    _, st = oracle.forward(cfg, lam, mu, rho, oracle.Source(tuple(p), force=force), np.array([s0]))
    b = 1.0 / rho[0, 0, 0]
    for comp in range(3):
        X, Y, Z = _sample_coords(shape, comp)
        f = st[comp]
        tot = dt * b * force[comp] * s0 / vol
        assert f.sum() == pytest.approx(tot, rel=1e-13)
        for coord, want in zip((X, Y, Z), p):
            assert (f * coord).sum() / f.sum() == pytest.approx(want, rel=1e-13)
    moment = (1e15, -2e15, 3e15, 4e15, -5e15, 6e15)
    _, st = oracle.forward(cfg, lam, mu, rho, oracle.Source(tuple(p), moment=moment), np.array([s0]))
    for q in range(6):
        comp = 3 + q
        X, Y, Z = _sample_coords(shape, comp)
        f = st[comp]
        tot = -dt * moment[q] * s0 / vol
        assert f.sum() == pytest.approx(tot, rel=1e-13)
        for coord, want in zip((X, Y, Z), p):
            assert (f * coord).sum() / f.sum() == pytest.approx(want, rel=1e-13)
