"""Vacuum free surface on the GPU (Sec. 2.5): every tile and cell kernel against the
oracle on a ragged grid with a vacuum layer, cubic and anisotropic cells, moment and
force sources; the model check accepts lam = mu = 0 only with the option; the fused
kernel, the gradient and the Born forward refuse the option; batched runs equal single
runs."""
import dataclasses

import numpy as np
import pytest
import torch

import workloads as W
from gpu_cases import compare, gpu_run, oracle_run
from test_gpu_forward import KERNELS, TOL, fp64_ok

pytestmark = pytest.mark.gpu

KS = 5


def vacuum_shot(force=False, h=10.0, seed=41):
    shape = (37, 29, 23)
    lam, mu, rho = W.layered_perturbed(shape, 10.0, seed)
    lam[:KS] = 0.0
    mu[:KS] = 0.0
    rho[:KS] = 0.04 * rho[KS:].min()
    nt = 160
    rng = np.random.Generator(np.random.PCG64(seed))
    f = (2e10, -1e10, 3e10) if force else (0.0, 0.0, 0.0)
    rec = np.array([[5.25, 6.5, KS + 0.5], [30.6, 20.1, KS + 1.0], [17.0, 14.0, 11.5], [9.9, 21.3, 18.2]])
    return W.Shot("vacuum", shape, h, 5e-4, nt, lam, mu, rho, (18.4, 13.7, 10.6), W.random_mt(rng), f,
                  W.ricker(40.0, nt, 5e-4), rec, sponge=(6, 5, 4, 7, 0, 6))


def run_oracle(shot):
    import oracle

    cfg = oracle.Config(shot.shape, shot.h, shot.dt, shot.nt, sponge=shot.sponge, vacuum_top=KS)
    src = oracle.Source(shot.src_pos, moment=shot.moment, force=shot.force)
    return oracle.forward(cfg, shot.lam, shot.mu, shot.rho, src, shot.wavelet, shot.rec_pos)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("force,h", [(False, 10.0), (True, 10.0), (True, (10.0, 12.0, 8.0))])
def test_vacuum_matches_oracle(dtype, force, h):
    shot = vacuum_shot(force, h)
    ref = run_oracle(shot)
    for kern in KERNELS:
        if kern[0] == "fused" or (dtype == torch.float64 and not fp64_ok(kern)):
            continue
        print(f"[vacuum] {dtype} force={force} h={h} {kern}", flush=True)
        compare(gpu_run(shot, dtype, kernel=kern, vacuum_top=KS), ref, TOL[dtype], f"vacuum {kern}")


def test_vacuum_option_checks():
    from paper_2112_15071_amd import Simulator, _abi

    shot = vacuum_shot()
    with pytest.raises(_abi.FD3DError) as e:  # lam + 2 mu = 0 without the option
        Simulator(shot.lam, shot.mu, shot.rho, shot.h, shot.dt, shot.nt, sponge=shot.sponge)
    assert e.value.code == _abi.FD3D_EMODEL
    sim = Simulator(shot.lam, shot.mu, shot.rho, shot.h, shot.dt, shot.nt, sponge=shot.sponge, vacuum_top=KS)
    with pytest.raises(_abi.FD3DError):
        sim.set_kernel("fused", 4, 8, 64)
    gws = sim.grad_workspace(10)
    with pytest.raises(_abi.FD3DError):
        sim.gradient(gws, torch.zeros((4, 3, shot.nt), device="cuda"),
                     *[torch.zeros(shot.lam.shape, device="cuda") for _ in range(3)],
                     src_pos=shot.src_pos, moment=shot.moment, wavelet=shot.wavelet, rec_pos=shot.rec_pos)
    with pytest.raises(_abi.FD3DError):
        sim.born(*[np.zeros_like(shot.lam) for _ in range(3)], src_pos=shot.src_pos, moment=shot.moment,
                 wavelet=shot.wavelet, rec_pos=shot.rec_pos)
    with pytest.raises(_abi.FD3DError):
        Simulator(shot.lam, shot.mu, shot.rho, shot.h, shot.dt, shot.nt, sponge=shot.sponge, vacuum_top=23)
    sim.close()


def test_batched_vacuum_equals_single():
    from paper_2112_15071_amd import Simulator
    from paper_2112_15071_amd.batch import BatchSimulator

    shots = [vacuum_shot(False, 10.0, 41), vacuum_shot(True, 10.0, 42)]
    singles = []
    for s in shots:
        sim = Simulator(s.lam, s.mu, s.rho, s.h, s.dt, s.nt, sponge=s.sponge, vacuum_top=KS)
        sim.set_kernel("tile", 8, 8, 64)
        singles.append(sim.forward(s.src_pos, s.moment, s.force, s.wavelet, s.rec_pos).cpu().numpy())
        sim.close()
    sims = [Simulator(s.lam, s.mu, s.rho, s.h, s.dt, s.nt, sponge=s.sponge, vacuum_top=KS) for s in shots]
    batch = BatchSimulator(sims)
    batch.set_kernel(64, 8)
    trs = batch.forward([dict(src_pos=s.src_pos, moment=s.moment, force=s.force, wavelet=s.wavelet,
                              rec_pos=s.rec_pos) for s in shots], use_graph=True)
    torch.cuda.synchronize()
    for a, b in zip(trs, singles):
        assert np.array_equal(a.cpu().numpy(), b)
    batch.close()
    for s in sims:
        s.close()


def hill_shot(seed=43):
    """The ragged grid with a hill: first solid plane 7 at the edges rising to 3."""
    shot = vacuum_shot(True, 10.0, seed)
    nx, ny, nz = shot.shape
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    ks = (7 - np.round(4 * np.exp(-(((x - 17.0) / 6.0) ** 2 + ((y - 13.0) / 5.0) ** 2)))).astype(np.int32)
    lam, mu, rho = W.layered_perturbed(shot.shape, 10.0, seed)
    vac = np.arange(nz)[:, None, None] < ks[None, :, :]
    rho_vac = 0.04 * rho[~vac].min()
    lam[vac], mu[vac], rho[vac] = 0.0, 0.0, rho_vac
    return dataclasses.replace(shot, lam=lam, mu=mu, rho=rho), ks


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_topography_matches_oracle(dtype):
    import oracle

    shot, ks = hill_shot()
    cfg = oracle.Config(shot.shape, shot.h, shot.dt, shot.nt, sponge=shot.sponge, vacuum_top=int(ks.max()),
                        vacuum_map=ks)
    ref = oracle.forward(cfg, shot.lam, shot.mu, shot.rho, oracle.Source(shot.src_pos, moment=shot.moment,
                                                                          force=shot.force),
                         shot.wavelet, shot.rec_pos)
    for kern in KERNELS:
        if kern[0] == "fused" or (dtype == torch.float64 and not fp64_ok(kern)):
            continue
        print(f"[topography] {dtype} {kern}", flush=True)
        compare(gpu_run(shot, dtype, kernel=kern, vacuum_map=ks), ref, TOL[dtype], f"topography {kern}")


def test_topography_checks():
    from paper_2112_15071_amd import Simulator, _abi

    shot, ks = hill_shot()
    bad = ks.copy()
    bad[3, 4] = 0
    with pytest.raises(_abi.FD3DError):
        Simulator(shot.lam, shot.mu, shot.rho, shot.h, shot.dt, shot.nt, sponge=shot.sponge, vacuum_map=bad)
    bad[3, 4] = shot.shape[2]
    with pytest.raises(_abi.FD3DError):
        Simulator(shot.lam, shot.mu, shot.rho, shot.h, shot.dt, shot.nt, sponge=shot.sponge, vacuum_map=bad)
