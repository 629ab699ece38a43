"""Pins of the oracle's tangent-linear (Born) forward: the derivative of the traces along a
model perturbation against central finite differences of the forward pass, the
dot-product identity with the (independently written) store-all adjoint gradient
<J dm, r> = <dm, J^T r>, and the background traces equal to the forward's."""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import rel_l2

NT, DT = 120, 1e-3
SHAPE = (24, 22, 20)
SPONGE, ALPHA = (5,) * 6, 0.05


def setup(h=10.0):
    nx, ny, nz = SHAPE
    rng = np.random.Generator(np.random.PCG64(808))
    vp = np.where(np.arange(nz) < nz // 2, 2500.0, 3200.0)[:, None, None] * np.ones((nz, ny, nx))
    vp = vp * (1.0 + 0.03 * W.gaussian_field((nz, ny, nx), 30.0, 10.0, rng))
    model = W.elastic_from_vp(vp)
    cfg = oracle.Config(SHAPE, h, DT, NT, sponge=SPONGE, alpha=ALPHA)
    rec = W.receiver_grid(np.linspace(7, nx - 8, 3), np.linspace(7, ny - 8, 3), 6.0)
    dm = [a * rng.standard_normal(a.shape) * 0.1 for a in model]
    return cfg, model, dm, rec, rng


SOURCES = {
    "moment": (oracle.Source((11.3, 10.6, 9.2), moment=(1e15, -3e14, 5e14, 2e14, -1e14, 4e14)), True),
    "force": (oracle.Source((12.7, 9.1, 10.8), force=(3e9, -2e9, 4e9)), False),
}


@pytest.mark.parametrize("kind", ["moment", "force"])
@pytest.mark.parametrize("which", [0, 1, 2, None])
def test_born_matches_central_differences(kind, which):
    cfg, model, dm, rec, _ = setup()
    src, at_half = SOURCES[kind]
    wav = W.ricker(25.0, NT, DT, at_half=at_half)
    if which is not None:
        dm = [d if p == which else np.zeros_like(d) for p, d in enumerate(dm)]
    tr, dtr = oracle.born(cfg, *model, *dm, src, wav, rec)
    eps = 1e-4
    plus = [m + eps * d for m, d in zip(model, dm)]
    minus = [m - eps * d for m, d in zip(model, dm)]
    fd = (oracle.forward(cfg, *plus, src, wav, rec)[0] - oracle.forward(cfg, *minus, src, wav, rec)[0]) / (2 * eps)
    assert rel_l2(dtr, fd) <= 1e-6, rel_l2(dtr, fd)
    assert np.array_equal(tr, oracle.forward(cfg, *model, src, wav, rec)[0])


@pytest.mark.parametrize("h", [10.0, (10.0, 12.0, 8.0)])
@pytest.mark.parametrize("kind", ["moment", "force"])
def test_born_is_the_transpose_of_the_gradient(kind, h):
    cfg, model, dm, rec, rng = setup(h)
    src, at_half = SOURCES[kind]
    wav = W.ricker(25.0, NT, DT, at_half=at_half)
    _, dtr = oracle.born(cfg, *model, *dm, src, wav, rec)
    r = rng.standard_normal(dtr.shape)
    gl, gm, gr, _ = oracle.gradient(cfg, *model, src, wav, rec, r)
    lhs = float(np.sum(dtr * r))
    rhs = float(np.sum(dm[0] * gl) + np.sum(dm[1] * gm) + np.sum(dm[2] * gr))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs), (lhs, rhs)
