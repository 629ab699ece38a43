"""Pins of the oracle's vacuum free surface (Sec. 2.5: low medium parameters above the
surface, second-order z differences next to it): a vertically incident P or S pulse
doubles at the effective surface half a cell above the first solid plane; the band of
second-order differences is what makes that accurate; the vacuum stays exactly free of
stress; the result agrees with the stress-imaging surface; mirror symmetry holds."""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import rel_l2
from test_oracle_free_surface import DT, H, RHO, VP, VS, plane_wave_state

KS = 10          # first solid node plane
RHO_VAC = 100.0  # vacuum density (lam = mu = 0 there)


def vacuum_model(shape, ks=KS):
    lam, mu, rho = W.homogeneous(shape, VP, VS, RHO)
    lam[:ks] = 0.0
    mu[:ks] = 0.0
    rho[:ks] = RHO_VAC
    return lam, mu, rho


def vertical_pulse(kind, band=KS):
    nz, z0, amp = 330, 210.0, 1e-3
    c = VP if kind == "P" else VS
    nt = int(1.15 * (z0 - KS) * H / c / DT)
    shape = (4, 4, nz)
    st0 = plane_wave_state(kind, nz, z0, 8.0, amp)
    st0[:, :KS] = 0.0
    cfg = oracle.Config(shape, H, DT, nt, periodic=(True, True, False), sponge=(0,) * 6, vacuum_top=band)
    zr = KS - 0.5  # effective surface
    rec = np.array([[1.0, 1.0, zr]]) if kind == "P" else np.array([[1.5, 1.0, zr]])
    tr, st = oracle.forward(cfg, *vacuum_model(shape), state=st0, rec_pos=rec)
    comp = 2 if kind == "P" else 0
    return tr[0, comp], amp, c, z0


@pytest.mark.parametrize("kind", ["P", "S"])
def test_vacuum_surface_doubles_vertical_incidence(kind):
    trace, amp, c, z0 = vertical_pulse(kind)
    assert abs(np.max(np.abs(trace)) / (2 * amp) - 1.0) < 0.01
    n_peak = int(np.argmax(np.abs(trace)))
    t_expect = (z0 - KS + 0.5) * H / c
    assert abs((n_peak + 0.5) * DT - t_expect) < 0.03 * t_expect


def test_second_order_band_makes_it_accurate():
    """The P doubling is exact to 1e-3 with the second-order band and off by several per
    cent with the fourth-order stencil reaching into the vacuum."""
    with_band, amp, _, _ = vertical_pulse("P")
    without, _, _, _ = vertical_pulse("P", band=0)
    assert abs(np.max(np.abs(with_band)) / (2 * amp) - 1.0) < 1e-3
    assert abs(np.max(np.abs(without)) / (2 * amp) - 1.0) > 0.03


def test_vacuum_stays_stress_free():
    shape = (24, 22, 26)
    lam, mu, rho = vacuum_model(shape, ks=6)
    nt = 80
    cfg = oracle.Config(shape, 10.0, 1e-3, nt, sponge=(5, 5, 5, 5, 0, 5), vacuum_top=6)
    src = oracle.Source((11.3, 10.6, 12.2), moment=W.double_couple(0.3, 1.1, -0.7))
    _, st = oracle.forward(cfg, lam, mu, rho, src, W.ricker(25.0, nt, 1e-3))
    assert np.all(st[3:6, :6] == 0.0)    # normal stresses at vacuum nodes
    assert np.all(st[6, :6] == 0.0)      # sxy at vacuum planes
    assert np.all(st[7:9, :5] == 0.0)    # sxz, syz between two vacuum planes
    assert np.max(np.abs(st[7, 5])) > 0  # ... but not at the plane straddling the surface
    assert np.all(np.isfinite(st))


def test_vacuum_agrees_with_stress_imaging():
    """A buried explosion recorded near the surface: the vacuum surface (effective surface
    half a cell above the first solid plane) against stress imaging on the same medium."""
    nt, ks = 150, 6
    wav = W.ricker(20.0, nt, 1e-3)
    shape_i = (40, 40, 34)
    rec_i = np.array([[x, 20.0, 1.0] for x in (12.0, 16.0, 24.0, 28.0)])
    cfg_i = oracle.Config(shape_i, 10.0, 1e-3, nt, sponge=(8, 8, 8, 8, 0, 8), free_surface=True)
    tri, _ = oracle.forward(cfg_i, *W.homogeneous(shape_i, VP, VS, RHO),
                            oracle.Source((20.0, 20.0, 10.0), moment=W.explosion(1e15)), wav, rec_i)
    shape_v = (40, 40, 40)
    cfg_v = oracle.Config(shape_v, 10.0, 1e-3, nt, sponge=(8, 8, 8, 8, 0, 8), vacuum_top=ks)
    shift = np.array([0.0, 0.0, ks - 0.5])
    trv, _ = oracle.forward(cfg_v, *vacuum_model(shape_v, ks),
                            oracle.Source(tuple(np.array([20.0, 20.0, 10.0]) + shift), moment=W.explosion(1e15)),
                            wav, rec_i + shift)
    assert rel_l2(trv[:, 2], tri[:, 2]) < 0.08   # vertical
    assert rel_l2(trv[:, 1], tri[:, 1]) < 0.10   # transverse (small)


def test_vacuum_mirror_symmetry():
    shape = (21, 18, 24)
    lam, mu, rho = vacuum_model(shape, ks=5)
    nt = 60
    cfg = oracle.Config(shape, 10.0, 1e-3, nt, sponge=(4, 4, 4, 4, 0, 4), vacuum_top=5)
    _, st = oracle.forward(cfg, lam, mu, rho, oracle.Source((10.0, 8.3, 11.4), moment=W.explosion(1e15)),
                           W.ricker(25.0, nt, 1e-3))
    # x -> 20 - x: vx (at x + 1/2) is odd about the centre, the other fields even
    vx = st[0][:, :, :20]
    assert np.max(np.abs(vx + vx[:, :, ::-1])) <= 1e-12 * np.max(np.abs(vx))
    szz = st[5]
    assert np.max(np.abs(szz - szz[:, :, ::-1])) <= 1e-12 * np.max(np.abs(szz))


def ridge_model(shape, depth=6, height=3):
    """A ridge along y, symmetric about x = (nx - 1) / 2: the first solid plane rises from
    `depth` to `depth - height` at the centre."""
    nx, ny, nz = shape
    x = np.arange(nx)
    ks_col = depth - np.round(height * np.exp(-((x - (nx - 1) / 2) / 3.0) ** 2)).astype(int)
    ks = np.broadcast_to(ks_col[None, :], (ny, nx)).astype(np.int32)
    lam, mu, rho = W.homogeneous(shape, VP, VS, RHO)
    z = np.arange(nz)[:, None, None]
    vac = z < ks[None, :, :]
    lam[vac] = 0.0
    mu[vac] = 0.0
    rho[vac] = RHO_VAC
    return (lam, mu, rho), ks


def test_flat_topography_equals_the_plane():
    shape = (18, 16, 22)
    lam, mu, rho = vacuum_model(shape, ks=5)
    nt = 50
    src = oracle.Source((8.3, 7.6, 11.4), moment=W.double_couple(0.3, 1.1, -0.7))
    wav = W.ricker(25.0, nt, 1e-3)
    a = oracle.forward(oracle.Config(shape, 10.0, 1e-3, nt, sponge=(4, 4, 4, 4, 0, 4), vacuum_top=5),
                       lam, mu, rho, src, wav)[1]
    b = oracle.forward(oracle.Config(shape, 10.0, 1e-3, nt, sponge=(4, 4, 4, 4, 0, 4), vacuum_top=5,
                                     vacuum_map=np.full((16, 18), 5, np.int32)), lam, mu, rho, src, wav)[1]
    assert np.array_equal(a, b)


def test_topography_mirror_symmetry_and_stress_free_vacuum():
    shape = (21, 14, 24)
    (lam, mu, rho), ks = ridge_model(shape)
    nt = 70
    cfg = oracle.Config(shape, 10.0, 1e-3, nt, sponge=(4, 4, 4, 4, 0, 4), vacuum_top=int(ks.max()), vacuum_map=ks)
    _, st = oracle.forward(cfg, lam, mu, rho, oracle.Source((10.0, 6.6, 12.4), moment=W.explosion(1e15)),
                           W.ricker(25.0, nt, 1e-3))
    assert np.all(np.isfinite(st))
    vx = st[0][:, :, :20]
    assert np.max(np.abs(vx + vx[:, :, ::-1])) <= 1e-12 * np.max(np.abs(vx))
    for c in (1, 2, 3, 5):
        f = st[c]
        assert np.max(np.abs(f - f[:, :, ::-1])) <= 1e-12 * np.max(np.abs(f)), c
    z = np.arange(shape[2])[:, None, None]
    vac = z < ks[None, :, :]
    assert np.all(st[3][vac] == 0.0) and np.all(st[4][vac] == 0.0) and np.all(st[5][vac] == 0.0)
    # the ridge changes the wavefield against a flat surface at its foot
    flat = oracle.Config(shape, 10.0, 1e-3, nt, sponge=(4, 4, 4, 4, 0, 4), vacuum_top=int(ks.max()))
    (l2, m2, r2) = vacuum_model(shape, ks=int(ks.max()))
    _, st2 = oracle.forward(flat, l2, m2, r2, oracle.Source((10.0, 6.6, 12.4), moment=W.explosion(1e15)),
                            W.ricker(25.0, nt, 1e-3))
    assert rel_l2(st[2], st2[2]) > 1e-3
