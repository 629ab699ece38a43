"""GPU tests of the C ABI's contract: error codes, state copy, resume, determinism."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def small(nt=40, shape=(24, 20, 18)):
    lam, mu, rho = W.layered_perturbed(shape, 10.0, 77)
    return lam, mu, rho, nt


def test_cfl_rejected():
    from paper_2112_15071_amd import Simulator
    from paper_2112_15071_amd._abi import FD3DError, FD3D_ECFL

    lam, mu, rho, nt = small()
    sim = Simulator(lam, mu, rho, 10.0, 5e-4, nt)
    vpmax, vsmin, rmin, dtmax = sim.info()
    assert abs(dtmax - 6 / (7 * np.sqrt(3)) * 10.0 / vpmax) < 1e-12 * dtmax
    assert abs(vpmax - np.sqrt((lam + 2 * mu) / rho).max()) < 1e-3 * vpmax
    sim.close()
    with pytest.raises(FD3DError) as e:
        Simulator(lam, mu, rho, 10.0, dtmax * 1.001, nt)
    assert e.value.code == FD3D_ECFL
    Simulator(lam, mu, rho, 10.0, dtmax * 0.999, nt).close()


@pytest.mark.parametrize("bad", ["rho", "mu", "nan"])
def test_bad_model_rejected(bad):
    from paper_2112_15071_amd import Simulator
    from paper_2112_15071_amd._abi import FD3DError, FD3D_EMODEL

    lam, mu, rho, nt = small()
    if bad == "rho":
        rho = rho.copy(); rho[3, 4, 5] = 0.0
    elif bad == "mu":
        mu = mu.copy(); mu[1, 2, 3] = -1.0
    else:
        lam = lam.copy(); lam[5, 5, 5] = np.nan
    with pytest.raises(FD3DError) as e:
        Simulator(lam, mu, rho, 10.0, 5e-4, nt)
    assert e.value.code == FD3D_EMODEL


def test_out_of_range_taps_rejected():
    from paper_2112_15071_amd import Simulator
    from paper_2112_15071_amd._abi import FD3DError, FD3D_ERANGE

    lam, mu, rho, nt = small()
    sim = Simulator(lam, mu, rho, 10.0, 5e-4, nt)
    w = W.ricker(25.0, nt, 5e-4)
    with pytest.raises(FD3DError) as e:
        sim.forward((5, 5, 5), W.explosion(), (0, 0, 0), w, [[22.9, 5.0, 5.0]])  # vx tap at slot nx-1
    assert e.value.code == FD3D_ERANGE
    with pytest.raises(FD3DError) as e:
        sim.forward((-0.5, 5, 5), W.explosion(), (0, 0, 0), w, [[5.0, 5.0, 5.0]])
    assert e.value.code == FD3D_ERANGE
    sim.forward((5, 5, 5), W.explosion(), (0, 0, 0), w, [[22.4, 5.0, 5.0]])  # last active vx slot
    sim.close()


def test_workspace_too_small():
    from paper_2112_15071_amd import _abi, make_opts

    lam, mu, rho, nt = small()
    nz, ny, nx = lam.shape
    dev = [torch.as_tensor(a, dtype=torch.float32, device="cuda") for a in (lam, mu, rho)]
    o = make_opts(torch.float32, 5)
    need = _abi.fd3d_workspace_bytes(nx, ny, nz, o)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    with pytest.raises(_abi.FD3DError) as e:
        _abi.fd3d_create(nx, ny, nz, *(t.data_ptr() for t in dev), 10.0, 5e-4, nt, o, ws.data_ptr(), need - 1,
                         torch.cuda.current_stream().cuda_stream)
    assert e.value.code == _abi.FD3D_EWS


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("fused", [False, True])
def test_resume_and_determinism(dtype, fused):
    """m steps, export, import, nt - m steps == nt straight, bitwise; reruns are bitwise.
    With the fused kernel the state swaps buffers every step (17 is odd)."""
    from paper_2112_15071_amd import Simulator

    lam, mu, rho, nt = small(nt=50)
    w = W.ricker(30.0, nt, 5e-4)
    src = ((11.3, 9.7, 8.2), (1e15, -3e14, 2e14, 5e14, -1e14, 3e14), (1e9, 0, -2e9))
    rec = [[5.5, 6.0, 7.25], [14.0, 9.5, 10.0]]

    def make(n):
        sim = Simulator(lam, mu, rho, 10.0, 5e-4, n, dtype=dtype, sponge=4)
        if fused:
            sim.set_kernel("fused", 4, 8, 64)
        return sim

    full = make(nt)
    t_full = full.forward(*src, w, rec).clone()
    s_full = full.state()
    t_again = full.forward(*src, w, rec).clone()
    assert torch.equal(t_full, t_again)
    assert torch.equal(s_full, full.state())
    m = 17
    a = make(m)
    ta = a.forward(*src, w[:m], rec)
    b = make(nt - m)
    b.set_state(a.state())
    tb = b.forward(*src, w[m:], rec, keep_state=True)
    assert torch.equal(torch.cat([ta, tb], dim=2), t_full)
    assert torch.equal(b.state(), s_full)
    for s in (full, a, b):
        s.close()


def test_set_state_pins_last_slot():
    from paper_2112_15071_amd import Simulator

    lam, mu, rho, nt = small(nt=1)
    sim = Simulator(lam, mu, rho, 10.0, 5e-4, nt)
    nz, ny, nx = lam.shape
    st = torch.ones((9, nz, ny, nx), device="cuda")
    sim.set_state(st)
    got = sim.state()
    assert torch.all(got[0][:, :, nx - 1] == 0) and torch.all(got[0][:, :, : nx - 1] == 1)
    assert torch.all(got[6][:, ny - 1, :] == 0) and torch.all(got[6][:, :, nx - 1] == 0)
    assert torch.all(got[8][nz - 1] == 0) and torch.all(got[3] == 1)
    sim.close()


def test_check_finite_flags_blow_up():
    """A state near the FP32 maximum overflows within a few steps; the debug check
    reports it.  From zero state the same context runs clean."""
    from paper_2112_15071_amd import Simulator
    from paper_2112_15071_amd._abi import FD3DError, FD3D_ENONFINITE

    lam, mu, rho, nt = small(nt=5)
    sim = Simulator(lam, mu, rho, 10.0, 5e-4, nt, check_finite=True)
    nz, ny, nx = lam.shape
    st = torch.full((9, nz, ny, nx), 3e38, device="cuda")
    sim.set_state(st)
    with pytest.raises(FD3DError) as e:
        sim.forward(None, rec_pos=None, keep_state=True)
    assert e.value.code == FD3D_ENONFINITE
    sim.forward(None, rec_pos=None)  # from zero: finite
    sim.close()
