"""Coarse medium grid: the HIP trilinear upsampler against the oracle's, and a forward
run on an upsampled model against the oracle on the oracle-upsampled model."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from gpu_cases import compare, gpu_run, oracle_run

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype,tol", [(torch.float32, 1e-6), (torch.float64, 1e-14)])
@pytest.mark.parametrize("mshape,nshape", [((5, 4, 3), (37, 29, 23)), ((7, 7, 7), (7, 7, 7)), ((1, 3, 2), (9, 8, 5)),
                                           ((33, 17, 9), (64, 64, 32))])
def test_upsample_matches_oracle(dtype, tol, mshape, nshape):
    from paper_2112_15071_amd import upsample

    rng = np.random.default_rng(sum(mshape) + sum(nshape))
    mx, my, mz = mshape
    c = 2000.0 + 500.0 * rng.random((mz, my, mx))
    print(f"[upsample] {mshape} -> {nshape} {dtype}", flush=True)
    got = upsample(torch.as_tensor(c, dtype=dtype, device="cuda"), nshape).double().cpu().numpy()
    want = oracle.upsample(c if dtype == torch.float64 else c.astype(np.float32).astype(np.float64), nshape)
    assert got.shape == want.shape
    assert np.max(np.abs(got - want)) <= tol * np.max(np.abs(want))


def test_forward_on_a_coarse_medium():
    """Medium on a 9 x 8 x 6 node grid, simulated on 37 x 29 x 23 nodes."""
    import dataclasses

    from paper_2112_15071_amd import upsample

    lam_c, mu_c, rho_c = W.layered_perturbed((9, 8, 6), 40.0, 55)
    fine = (37, 29, 23)
    up_o = [oracle.upsample(a, fine) for a in (lam_c, mu_c, rho_c)]
    up_g = [upsample(torch.as_tensor(a, dtype=torch.float64, device="cuda"), fine).cpu().numpy()
            for a in (lam_c, mu_c, rho_c)]
    for a, b in zip(up_o, up_g):
        assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))
    rng = np.random.default_rng(55)
    nt = 120
    rec = np.array([[5.25, 6.5, 3.0], [30.6, 20.1, 4.0], [17.0, 14.0, 11.5]])
    shot = W.Shot("coarse", fine, 10.0, 5e-4, nt, *up_o, (18.4, 13.7, 9.6), W.random_mt(rng), (0.0, 0.0, 0.0),
                  W.ricker(40.0, nt, 5e-4), rec, sponge=(5,) * 6)
    ref = oracle_run(shot)
    for dtype, tol in ((torch.float32, 1e-4), (torch.float64, 1e-12)):
        got = gpu_run(dataclasses.replace(shot, lam=up_g[0], mu=up_g[1], rho=up_g[2]), dtype)
        compare(got, ref, tol, f"coarse medium {dtype}")


# ------------------------------------------------------------------ coarse medium read in the kernels

def coarse_shot(free_surface, h=10.0, seed=57):
    """Medium on 9 x 8 x 6 coarse nodes over a ragged 37 x 29 x 23 grid (no coarse node
    spacing divides the fine one), moment and force sources."""
    lam_c, mu_c, rho_c = W.layered_perturbed((9, 8, 6), 40.0, seed)
    rng = np.random.default_rng(seed)
    nt = 140
    rec = np.array([[5.25, 6.5, 1.0], [30.6, 20.1, 4.0], [17.0, 14.0, 11.5], [9.9, 21.3, 18.2]])
    sponge = (5, 6, 4, 5, 0 if free_surface else 5, 6)
    return W.Shot("coarse", (37, 29, 23), h, 5e-4, nt, lam_c, mu_c, rho_c, (18.4, 13.7, 6.6), W.random_mt(rng),
                  (2e10, -1e10, 3e10), W.ricker(40.0, nt, 5e-4), rec, sponge=sponge, free_surface=free_surface)


def coarse_oracle(shot, coarse_reading=True):
    cfg = oracle.Config(shot.shape, shot.h, shot.dt, shot.nt, sponge=shot.sponge, free_surface=shot.free_surface,
                        coarse=tuple(reversed(shot.lam.shape)) if coarse_reading else None)
    model = (shot.lam, shot.mu, shot.rho) if coarse_reading else tuple(oracle.upsample(a, shot.shape)
                                                                     for a in (shot.lam, shot.mu, shot.rho))
    return oracle.forward(cfg, *model, oracle.Source(shot.src_pos, moment=shot.moment, force=shot.force),
                          shot.wavelet, shot.rec_pos)


TILES = [("tile", 4, 4), ("tile", 8, 5), ("tile", 16, 32), ("tile", 4, 6, 128), ("tile", 8, 9, 128),
         ("tile", 4, 7, 256), ("tile", 4, 23, 256)]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("free_surface,h", [(False, 10.0), (True, 10.0), (False, (10.0, 12.0, 8.0))])
def test_coarse_medium_in_kernel_matches_oracle(dtype, free_surface, h):
    """The step kernels reading the coarse medium by trilinear samples at every value's own
    position (rho at the velocity samples, lambda and mu at the nodes, mu at the shear
    samples) against the oracle's same reading, through every tile shape."""
    from test_gpu_forward import fp64_ok

    shot = coarse_shot(free_surface, h)
    ref = coarse_oracle(shot)
    for kern in TILES:
        if dtype == torch.float64 and not fp64_ok(kern):
            continue
        print(f"[coarse] {dtype} fs={free_surface} h={h} {kern}", flush=True)
        got = gpu_run(shot, dtype, kernel=kern, grid=shot.shape)
        compare(got, ref, 1e-4 if dtype == torch.float32 else 1e-12, f"coarse medium in-kernel {kern}")


def test_coarse_reading_differs_from_the_setup_reading():
    """The two readings of one coarse medium agree to a fraction of a per cent on this
    smooth model but not to rounding: they differ where a node mean straddles a coarse
    node."""
    shot = coarse_shot(False)
    tr_in, _ = gpu_run(shot, torch.float64, kernel=("tile", 8, 5), grid=shot.shape)
    tr_setup, _ = coarse_oracle(shot, coarse_reading=False)
    for c in range(3):
        d = np.linalg.norm(tr_in[:, c] - tr_setup[:, c]) / np.linalg.norm(tr_setup[:, c])
        assert 1e-9 < d < 5e-2, (c, d)


def test_coarse_medium_refusals():
    from paper_2112_15071_amd import Simulator, _abi

    shot = coarse_shot(False)
    sim = Simulator(shot.lam, shot.mu, shot.rho, shot.h, shot.dt, shot.nt, sponge=shot.sponge, grid=shot.shape)
    with pytest.raises(_abi.FD3DError):
        sim.set_kernel("cell", 8, 32)
    with pytest.raises(_abi.FD3DError):
        sim.set_kernel("fused", 4, 8)
    with pytest.raises(_abi.FD3DError):  # the gradient's checkpointed forward
        sim.forward_ckpt(sim.grad_workspace(10), shot.src_pos, shot.moment, wavelet=shot.wavelet,
                         rec_pos=shot.rec_pos)
    sim.close()
    with pytest.raises(_abi.FD3DError):  # coarse medium with the vacuum surface
        Simulator(shot.lam, shot.mu, shot.rho, shot.h, shot.dt, shot.nt, grid=shot.shape, vacuum_top=3)
