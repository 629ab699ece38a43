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
