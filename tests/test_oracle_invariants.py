"""Invariant pins of the oracle on small closed (zero-halo) boxes: discrete energy
conservation, force reciprocity, mirror and axis-permutation symmetry, linearity
and time-shift invariance, and stability at the von Neumann bound."""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import active_mask, discrete_energy, random_state, rel_l2


def hetero_model(shape, seed):
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    vp = 3000.0 * (1.0 + 0.2 * rng.random((nz, ny, nx)))
    return W.elastic_from_vp(vp)


def test_energy_conserved_without_damping():
    """E^n = 1/2 sum rho v^{n-1/2} v^{n+1/2} + 1/2 sum sigma C^-1 sigma is invariant
    (leapfrog with D- = -(D+)^T), heterogeneous model, random start."""
    shape = (11, 9, 13)
    lam, mu, rho = hetero_model(shape, 5)
    rng = np.random.default_rng(6)
    st = random_state(shape, rng, vscale=1e-3, sscale=1e4)
    cfg = oracle.Config(shape, 10.0, 1e-3, 1)
    energies = []
    for n in range(120):
        v_prev = st[:3].copy()
        _, st = oracle.forward(cfg, lam, mu, rho, state=st)
        # st now holds v^{n+1/2} and sigma^{n+1}; energy at step n uses sigma^n
        if n > 0:
            energies.append(discrete_energy(v_prev, np.concatenate([st[:3], s_prev]), lam, mu, rho, shape))
        s_prev = st[3:].copy()
    e = np.array(energies)
    assert np.max(np.abs(e - e[0])) <= 1e-12 * abs(e[0])


def test_energy_decays_with_damping():
    """With the sponge on, the discrete energy never grows and ends lower."""
    shape = (24, 22, 20)
    lam, mu, rho = hetero_model(shape, 7)
    rng = np.random.default_rng(8)
    st = random_state(shape, rng)
    cfg = oracle.Config(shape, 10.0, 1e-3, 1, sponge=(6,) * 6)
    e = []
    for n in range(60):
        v_prev = st[:3].copy()
        s_now = st[3:].copy()
        _, st = oracle.forward(cfg, lam, mu, rho, state=st)
        e.append(discrete_energy(v_prev, np.concatenate([st[:3], s_now]), lam, mu, rho, shape))
    e = np.array(e[1:])
    assert np.all(np.diff(e) <= 1e-12 * e[0])
    assert e[-1] < 0.9 * e[0]


def test_damping_leaves_interior_until_waves_arrive():
    """Fields far from the sponge are bitwise those of the undamped run until the
    stencil's domain of dependence (4 cells per step) carries the damping back."""
    shape = (60, 60, 60)
    lam, mu, rho = W.homogeneous(shape)
    src = oracle.Source((30.0, 30.0, 30.0), moment=W.explosion())
    nt = 8
    wav = np.ones(nt)
    c_damp = oracle.Config(shape, 10.0, 1e-3, nt, sponge=(10,) * 6)
    c_free = oracle.Config(shape, 10.0, 1e-3, nt)
    _, a = oracle.forward(c_damp, lam, mu, rho, src, wav)
    _, b = oracle.forward(c_free, lam, mu, rho, src, wav)
    inner = (slice(22, 38),) * 3
    for c in range(9):
        assert np.array_equal(a[c][inner], b[c][inner])
    # ... while inside the damping zone the two runs already differ
    assert not np.array_equal(a[3][:, :, :10], b[3][:, :, :10])


@pytest.mark.parametrize("ci,cj", [(0, 0), (0, 2), (1, 2), (2, 1)])
def test_force_reciprocity(ci, cj):
    """F_i at A -> v_j at B equals F_j at B -> v_i at A (no damping)."""
    shape = (14, 13, 12)
    lam, mu, rho = hetero_model(shape, 9)
    A = (4.3, 5.6, 4.8)
    B = (8.7, 6.2, 7.1)
    nt = 60
    wav = W.ricker(60.0, nt, 1e-3, at_half=False)
    cfg = oracle.Config(shape, 10.0, 1e-3, nt)
    f1 = [0.0, 0.0, 0.0]
    f1[ci] = 1e9
    f2 = [0.0, 0.0, 0.0]
    f2[cj] = 1e9
    t1, _ = oracle.forward(cfg, lam, mu, rho, oracle.Source(A, force=f1), wav, np.array([B]))
    t2, _ = oracle.forward(cfg, lam, mu, rho, oracle.Source(B, force=f2), wav, np.array([A]))
    a = t1[0, cj]
    b = t2[0, ci]
    assert np.max(np.abs(a)) > 0
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))


def test_mirror_symmetry():
    """Explosion at the centre of an odd homogeneous box: each field is even or odd
    under each axis mirror (staggered slot i <-> n-2-i, integer i <-> n-1-i)."""
    n = 25
    shape = (n, n, n)
    lam, mu, rho = W.homogeneous(shape)
    nt = 30
    cfg = oracle.Config(shape, 10.0, 1e-3, nt, sponge=(5,) * 6)
    src = oracle.Source((12.0, 12.0, 12.0), moment=W.explosion())
    _, st = oracle.forward(cfg, lam, mu, rho, src, W.ricker(25.0, nt, 1e-3))
    from helpers import STAG

    # parity under the mirror of axis a: -1 for the a-velocity and the shear stresses with index a
    odd = {0: {0, 6, 7}, 1: {1, 6, 8}, 2: {2, 7, 8}}
    for a in range(3):
        npax = 2 - a
        for c in range(9):
            f = st[c]
            if STAG[c][a]:
                core = np.take(f, np.arange(n - 1), axis=npax)
                mir = np.flip(core, axis=npax)
            else:
                core = f
                mir = np.flip(f, axis=npax)
            sign = -1.0 if c in odd[a] else 1.0
            scale = np.max(np.abs(core)) + 1e-300
            assert np.max(np.abs(core - sign * mir)) <= 1e-14 * scale, (a, c)


@pytest.mark.parametrize("h", [10.0, (10.0, 8.0, 12.0)])
def test_axis_permutation(h):
    """Swapping x and y in the model, source and spacing swaps the fields exactly (up to
    summation order): catches index mix-ups between axes, including a spacing taken
    from the wrong axis."""
    shape = (12, 15, 11)
    lam, mu, rho = hetero_model(shape, 11)
    nt = 25
    mt = (1.0e15, -0.4e15, 0.7e15, 0.3e15, -0.2e15, 0.5e15)  # xx yy zz xy xz yz
    pos = (5.3, 7.6, 4.9)
    wav = W.ricker(30.0, nt, 1e-3)
    sponge = (3, 4, 5, 2, 3, 6)
    hs = (h, h, h) if np.ndim(h) == 0 else h
    cfg = oracle.Config(shape, hs, 1e-3, nt, sponge=sponge)
    rec = np.array([[3.2, 9.1, 6.6], [8.4, 4.7, 2.2]])
    ta, a = oracle.forward(cfg, lam, mu, rho, oracle.Source(pos, moment=mt), wav, rec)
    T = lambda f: np.ascontiguousarray(np.swapaxes(f, 1, 2))
    shape_b = (15, 12, 11)
    sponge_b = (5, 2, 3, 4, 3, 6)
    cfg_b = oracle.Config(shape_b, (hs[1], hs[0], hs[2]), 1e-3, nt, sponge=sponge_b)
    mt_b = (mt[1], mt[0], mt[2], mt[3], mt[5], mt[4])
    tb, b = oracle.forward(cfg_b, T(lam), T(mu), T(rho), oracle.Source((pos[1], pos[0], pos[2]), moment=mt_b),
                           wav, rec[:, [1, 0, 2]])
    perm = [1, 0, 2, 4, 3, 5, 6, 8, 7]  # field of run a that maps to each field of run b
    for cb in range(9):
        want = T(a[perm[cb]])
        assert rel_l2(b[cb], want) <= 1e-13, cb
    np.testing.assert_allclose(tb[:, [1, 0, 2]], ta, rtol=1e-12, atol=1e-12 * np.max(np.abs(ta)))


def test_linearity_and_time_shift():
    shape = (20, 18, 16)
    lam, mu, rho = hetero_model(shape, 12)
    nt = 60
    cfg = oracle.Config(shape, 10.0, 1e-3, nt, sponge=(4,) * 6)
    rec = np.array([[5.5, 6.0, 7.25], [14.0, 9.5, 10.0]])
    m1 = (1e15, 2e14, -3e14, 4e14, 0.0, -1e14)
    m2 = (0.0, -5e14, 1e15, 0.0, 3e14, 2e14)
    pos = (9.4, 8.8, 7.3)
    wav = W.ricker(40.0, nt, 1e-3)
    t1, _ = oracle.forward(cfg, lam, mu, rho, oracle.Source(pos, moment=m1), wav, rec)
    t2, _ = oracle.forward(cfg, lam, mu, rho, oracle.Source(pos, moment=m2), wav, rec)
    m12 = tuple(2.5 * a - 1.5 * b for a, b in zip(m1, m2))
    t12, _ = oracle.forward(cfg, lam, mu, rho, oracle.Source(pos, moment=m12), wav, rec)
    assert rel_l2(t12, 2.5 * t1 - 1.5 * t2) <= 1e-13
    shift = 7
    wav_s = np.concatenate([np.zeros(shift), wav[:-shift]])
    ts, _ = oracle.forward(cfg, lam, mu, rho, oracle.Source(pos, moment=m1), wav_s, rec)
    assert np.array_equal(ts[:, :, :shift], np.zeros_like(ts[:, :, :shift]))
    assert rel_l2(ts[:, :, shift:], t1[:, :, :-shift]) <= 1e-13


@pytest.mark.parametrize("courant,stable", [(0.49, True), (0.50, False)])
def test_von_neumann_bound(courant, stable):
    """The 3D O(2,4) bound is 6/(7 sqrt 3) = 0.49487: the diagonal Nyquist mode grows
    just above it and stays bounded just below it (periodic box, random start)."""
    shape = (8, 8, 8)
    lam, mu, rho = W.homogeneous(shape)
    vp = np.sqrt((lam[0, 0, 0] + 2 * mu[0, 0, 0]) / rho[0, 0, 0])
    h = 10.0
    dt = courant * h / vp
    rng = np.random.default_rng(13)
    st0 = random_state(shape, rng, periodic=(True, True, True))
    cfg = oracle.Config(shape, h, dt, 400, periodic=(True, True, True))
    _, st = oracle.forward(cfg, lam, mu, rho, state=st0)
    growth = np.max(np.abs(st[:3])) / np.max(np.abs(st0[:3]))
    if stable:
        assert growth < 10.0
    else:
        assert growth > 1e6
