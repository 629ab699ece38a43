"""The forward entry point that allocates nothing (fd3d_forward_static: the whole workspace
in the library's static device scratch) against the existing path (fd3d_create on a
caller workspace + fd3d_forward + fd3d_get_state): identical traces and final state, bit
for bit, on two calls in a row whose second grid is smaller (the scratch keeps the first
call's contents), then again after a larger call, in FP32 and FP64; the first call also
against the FP64 oracle; grids beyond the scratch are refused with FD3D_EWS."""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_cases import compare, oracle_run

pytestmark = pytest.mark.gpu


def shot(shape, seed, nt=90):
    lam, mu, rho = W.layered_perturbed(shape, 10.0, seed)
    rng = np.random.Generator(np.random.PCG64(seed))
    nx, ny, nz = shape
    pos = (nx / 2 + 0.3, ny / 2 - 0.4, nz / 2 + 0.2)
    rec = np.stack([rng.uniform(3, nx - 4, 9), rng.uniform(3, ny - 4, 9), rng.uniform(2, nz - 4, 9)], axis=1)
    return W.Shot(f"static{seed}", shape, 10.0, 5e-4, nt, lam, mu, rho, pos, W.random_mt(rng), (1e10, -2e10, 5e9),
                  W.ricker(40.0, nt, 5e-4), rec, sponge=(5,) * 6)


def with_context(s, dtype):
    from paper_2112_15071_amd import Simulator

    sim = Simulator(s.lam, s.mu, s.rho, s.h, s.dt, s.nt, dtype=dtype, sponge=s.sponge)
    tr = sim.forward(s.src_pos, s.moment, s.force, s.wavelet, s.rec_pos).clone()
    st = sim.state()
    torch.cuda.synchronize()
    sim.close()
    return tr, st


def static(s, dtype):
    from paper_2112_15071_amd import forward_static

    dev = torch.device("cuda")
    lam, mu, rho = (torch.as_tensor(a, dtype=dtype, device=dev).contiguous() for a in (s.lam, s.mu, s.rho))
    wav = torch.as_tensor(s.wavelet, dtype=dtype, device=dev)
    nx, ny, nz = s.shape
    tr = torch.full((len(s.rec_pos), 3, s.nt), float("nan"), dtype=dtype, device=dev)
    st = torch.full((9, nz, ny, nx), float("nan"), dtype=dtype, device=dev)
    forward_static(lam, mu, rho, s.h, s.dt, s.nt, s.src_pos, s.moment, s.force, wav, s.rec_pos, dtype=dtype,
                   sponge=s.sponge, traces=tr, state=st)
    return tr, st


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_static_forward_equals_forward(dtype):
    big, small, mid = shot((60, 52, 44), 611), shot((37, 29, 23), 612), shot((48, 40, 36), 613)
    for k, s in enumerate((big, small, mid)):
        print(f"[static] call {k}: {s.shape} {dtype}", flush=True)
        got = static(s, dtype)
        want = with_context(s, dtype)
        assert torch.isfinite(got[0]).all() and torch.isfinite(got[1]).all(), k
        assert torch.equal(got[0], want[0]), k
        assert torch.equal(got[1], want[1]), k
        if k == 0:
            compare((got[0].double().cpu().numpy(), got[1].double().cpu().numpy()), oracle_run(s),
                    1e-4 if dtype == torch.float32 else 1e-12, f"static forward {dtype}")


def test_static_forward_refuses_grids_beyond_the_scratch():
    from paper_2112_15071_amd import _abi, forward_static

    dev = torch.device("cuda")
    n = 128  # 128^3 FP32 needs ~151 MB of workspace
    lam, mu, rho = (torch.full((n, n, n), v, device=dev) for v in (7.5e9, 7.5e9, 2500.0))
    with pytest.raises(_abi.FD3DError) as e:
        forward_static(lam, mu, rho, 10.0, 1e-3, 4, sponge=0)
    assert e.value.code == _abi.FD3D_EWS and "static scratch" in str(e.value)
