"""Pins of the oracle's free top surface (stress imaging with the second-order z
difference next to the surface): szz vanishes on the surface plane, and a laterally
uniform vertically incident P or S pulse doubles its particle velocity there."""
import numpy as np
import pytest

import oracle
import workloads as W

VP, VS, RHO = 3000.0, 1732.0, 2500.0
H, DT = 10.0, 1e-3


def plane_wave_state(kind, nz, z0_cells, width_cells, amp):
    """Upgoing pulse g(z + c t): v at t = -dt/2 and stresses at t = 0."""
    nx = ny = 4
    lam = RHO * VP * VP - 2 * RHO * VS * VS
    mu = RHO * VS * VS
    st = np.zeros((9, nz, ny, nx))
    zi = np.arange(nz) * H
    zh = (np.arange(nz) + 0.5) * H
    g = lambda z, t, c: amp * np.exp(-(((z + c * t) - z0_cells * H) / (width_cells * H)) ** 2)
    if kind == "P":
        c = VP
        st[2] = g(zh, -DT / 2, c)[:, None, None]  # vz at (i, j, k+1/2)
        szz = RHO * c * g(zi, 0.0, c)
        st[5] = szz[:, None, None]
        st[3] = st[4] = (lam / (lam + 2 * mu) * szz)[:, None, None]
    else:
        c = VS
        st[0] = g(zi, -DT / 2, c)[:, None, None]  # vx at (i+1/2, j, k)
        st[7] = (RHO * c * g(zh, 0.0, c))[:, None, None]  # sxz at (i+1/2, j, k+1/2)
    return st


@pytest.mark.parametrize("kind", ["P", "S"])
def test_surface_doubles_vertical_incidence(kind):
    nz = 320
    z0 = 200.0
    amp = 1e-3
    c = VP if kind == "P" else VS
    nt = int(1.15 * z0 * H / c / DT)
    shape = (4, 4, nz)
    lam, mu, rho = W.homogeneous(shape, VP, VS, RHO)
    st0 = plane_wave_state(kind, nz, z0, 8.0, amp)
    cfg = oracle.Config(shape, H, DT, nt, free_surface=True, periodic=(True, True, False),
                        sponge=(0, 0, 0, 0, 0, 0))
    rec = np.array([[1.0, 1.0, 0.5]]) if kind == "P" else np.array([[1.5, 1.0, 0.0]])
    tr, st = oracle.forward(cfg, lam, mu, rho, state=st0, rec_pos=rec)
    comp = 2 if kind == "P" else 0
    peak = np.max(np.abs(tr[0, comp]))
    assert abs(peak / (2 * amp) - 1.0) < 0.01, peak / amp
    # the arrival is at the expected time (pulse centre travels z0 from its start)
    n_peak = int(np.argmax(np.abs(tr[0, comp])))
    t_expect = z0 * H / c
    assert abs((n_peak + 0.5) * DT - t_expect) < 0.03 * t_expect
    assert np.all(st[5][0] == 0.0)


def test_szz_zero_on_surface_and_imaging_in_3d():
    shape = (24, 22, 20)
    lam, mu, rho = W.layered_perturbed(shape, 10.0, 77)
    nt = 60
    cfg = oracle.Config(shape, 10.0, 1e-3, nt, sponge=(5, 5, 5, 5, 0, 5), free_surface=True)
    src = oracle.Source((11.3, 10.6, 4.2), moment=W.double_couple(0.3, 1.1, -0.7))
    rec = np.array([[6.0, 7.0, 1.0], [15.5, 12.25, 1.0]])
    tr, st = oracle.forward(cfg, lam, mu, rho, src, W.ricker(25.0, nt, 1e-3), rec)
    assert np.all(st[5][0] == 0.0)
    assert np.max(np.abs(st[5][1])) > 0
    assert np.all(np.isfinite(st))
    # top sponge width is ignored with the free surface: same result when it is set
    cfg2 = oracle.Config(shape, 10.0, 1e-3, nt, sponge=(5, 5, 5, 5, 9, 5), free_surface=True)
    tr2, st2 = oracle.forward(cfg2, lam, mu, rho, src, W.ricker(25.0, nt, 1e-3), rec)
    assert np.array_equal(st, st2)


def test_free_surface_differs_from_closed_top():
    shape = (16, 16, 16)
    lam, mu, rho = W.homogeneous(shape)
    nt = 30
    src = oracle.Source((8.0, 8.0, 3.0), moment=W.explosion())
    wav = W.ricker(30.0, nt, 1e-3)
    _, a = oracle.forward(oracle.Config(shape, 10.0, 1e-3, nt, free_surface=True), lam, mu, rho, src, wav)
    _, b = oracle.forward(oracle.Config(shape, 10.0, 1e-3, nt), lam, mu, rho, src, wav)
    assert not np.allclose(a[2][:3], b[2][:3])
