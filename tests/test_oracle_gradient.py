"""Pins of the oracle's store-all discrete adjoint: the adjoint-state dot-product
identity <P x0, r> = <x0, P^T r> (sources off, sponge on), and the model gradient
of J = 1/2 |d - d_obs|^2 against central finite differences of the forward pass."""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import random_state

NT = 160
DT = 1e-3
H = 10.0
SPONGE = (6,) * 6
ALPHA = 0.05


def fd_setup(h=H):
    lam, mu, rho, srcs, rec = W.small_fd_case(nt=NT)
    shape = (lam.shape[2], lam.shape[1], lam.shape[0])
    cfg = oracle.Config(shape, h, DT, NT, sponge=SPONGE, alpha=ALPHA)
    wav = W.ricker(25.0, NT, DT)
    # observed data from a model with a slow blob
    nz, ny, nx = lam.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    blob = np.exp(-((x - 16) ** 2 + (y - 15) ** 2 + (z - 17) ** 2) / 20.0)
    vp = np.sqrt((lam + 2 * mu) / rho) * (1.0 - 0.04 * blob)
    lt, mt, rt = W.elastic_from_vp(vp)
    return cfg, (lam, mu, rho), (lt, mt, rt), srcs, rec, wav


def misfit_and_grad(cfg, model, srcs_obs, rec, wav, srcs):
    lam, mu, rho = model
    J = 0.0
    g = [np.zeros_like(lam) for _ in range(3)]
    for src, dobs in zip(srcs, srcs_obs):
        tr, _ = oracle.forward(cfg, lam, mu, rho, src, wav, rec)
        J += oracle.misfit(tr, dobs)
        gl, gm, gr, _ = oracle.gradient(cfg, lam, mu, rho, src, wav, rec, tr - dobs)
        g[0] += gl
        g[1] += gm
        g[2] += gr
    return J, g


def misfit_only(cfg, model, srcs_obs, rec, wav, srcs):
    lam, mu, rho = model
    J = 0.0
    for src, dobs in zip(srcs, srcs_obs):
        tr, _ = oracle.forward(cfg, lam, mu, rho, src, wav, rec)
        J += oracle.misfit(tr, dobs)
    return J


@pytest.mark.parametrize("kind,h", [("moment", H), ("force", H), ("force", (10.0, 12.0, 8.0))])
def test_gradient_matches_central_differences(kind, h):
    cfg, model, true, src_pos, rec, wav = fd_setup(h)
    if kind == "moment":
        srcs = [oracle.Source(p, moment=W.explosion(1e15)) for p in src_pos]
    else:
        srcs = [oracle.Source(p, force=(3e9, -2e9, 4e9)) for p in src_pos]
        wav = W.ricker(25.0, NT, DT, at_half=False)
    d_obs = [oracle.forward(cfg, *true, s, wav, rec)[0] for s in srcs]
    J0, g = misfit_and_grad(cfg, model, d_obs, rec, wav, srcs)
    assert J0 > 0
    rng = np.random.default_rng(21)
    nz, ny, nx = model[0].shape
    for p in range(3):
        for direction in ("random", "cell"):
            d = np.zeros_like(model[p])
            if direction == "random":
                d = rng.standard_normal(d.shape) * model[p]
            else:
                d[14, 17, 13] = model[p][14, 17, 13]
            eps = 1e-5
            plus = [m.copy() for m in model]
            minus = [m.copy() for m in model]
            plus[p] += eps * d
            minus[p] -= eps * d
            fd = (misfit_only(cfg, plus, d_obs, rec, wav, srcs) - misfit_only(cfg, minus, d_obs, rec, wav, srcs)) / (2 * eps)
            an = float(np.sum(g[p] * d))
            assert abs(fd - an) <= 1e-6 * abs(an), (p, direction, fd, an)


@pytest.mark.parametrize("h", [H, (10.0, 8.0, 12.0)])
def test_adjoint_state_dot_product(h):
    """Sources off, random initial state x0 and random residual r:
    <P x0, r> = <x0, P^T r> where P^T r is the adjoint of the initial state."""
    shape = (18, 16, 14)
    rng = np.random.default_rng(22)
    lam, mu, rho = W.elastic_from_vp(3000.0 * (1 + 0.2 * rng.random((14, 16, 18))))
    nt = 50
    cfg = oracle.Config(shape, h, DT, nt, sponge=(4, 5, 3, 4, 5, 3))
    x0 = random_state(shape, rng)
    rec = np.array([[4.2, 5.5, 6.1], [12.7, 9.3, 3.3], [8.0, 8.0, 8.0]])
    d, _ = oracle.forward(cfg, lam, mu, rho, None, None, rec, state=x0)
    r = rng.standard_normal(d.shape)
    _, _, _, adj = oracle.gradient(cfg, lam, mu, rho, None, None, rec, r, state0=x0)
    lhs = float(np.sum(d * r))
    rhs = float(np.sum(x0 * adj))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
