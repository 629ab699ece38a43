"""Closed-form pin of the whole forward pass: an explosion (M = M0 I) in a homogeneous
full space against the analytic radial velocity (near- and far-field terms), and the
error's fall when h and dt are halved together."""
import numpy as np

import oracle
import workloads as W
from oracle.analytic import explosion_vr

VP, VS, RHO = 3000.0, 1732.0, 2500.0
F0 = 15.0
M0 = 1e15


def run(n, h, dt, nt, sponge, dists):
    """n: nodes per axis (int) or (nx, ny, nz); h: one spacing or (dx, dy, dz)."""
    shape = (n, n, n) if np.ndim(n) == 0 else tuple(n)
    hs = np.array((h, h, h) if np.ndim(h) == 0 else h, float)
    lam, mu, rho = W.homogeneous(shape, VP, VS, RHO)
    c = np.array([m // 2 for m in shape], float)
    cfg = oracle.Config(shape, tuple(hs), dt, nt, sponge=(sponge,) * 6)
    wav = W.ricker(F0, nt, dt)  # moment rate at (n + 1/2) dt
    rec = []
    for ax in range(3):
        for r in dists:
            p = c.copy()
            p[ax] = c[ax] + r / hs[ax]  # on the radial component's own samples
            rec.append(p)
    rec = np.array(rec, float)
    tr, _ = oracle.forward(cfg, lam, mu, rho, oracle.Source(tuple(c), moment=W.explosion(M0)), wav, rec)
    times = (np.arange(nt) + 0.5) * dt  # receivers record v^{n+1/2}
    num = den = 0.0
    for q, p in enumerate(rec):
        d = (p - c) * hs
        r = np.linalg.norm(d)
        want = explosion_vr(r, times, M0, RHO, VP, F0, 1.5 / F0)[None, :] * (d / r)[:, None]
        num += np.sum((tr[q] - want) ** 2)
        den += np.sum(want ** 2)
    return np.sqrt(num / den)


def test_explosion_closed_form_and_convergence():
    # window ends before returns from the grid edges reach the receivers
    coarse = run(48, 20.0, 2e-3, 100, 10, [110.0, 150.0, 190.0])
    fine = run(96, 10.0, 1e-3, 200, 20, [105.0, 145.0, 185.0])
    assert coarse < 0.05
    assert fine < 0.01
    assert coarse / fine >= 4.0


def test_explosion_closed_form_anisotropic_cells():
    """Cells of 10 x 10 x 8 m: the point source injects per cell volume dx dy dz and each
    derivative divides by its own axis' spacing; the closed form holds to the accuracy of
    the isotropic 10 m grid along all three axes (a cube volume, or a spacing from the
    wrong axis, misses by tens of percent)."""
    err = run((96, 96, 120), (10.0, 10.0, 8.0), 1e-3, 200, 20, [105.0, 145.0, 185.0])
    assert err < 0.01
