"""Field storage (fd3d_opts.layout): separate arrays and interleaved rows run the same
arithmetic on the same samples, so every entry point gives bitwise equal results in both.
The oracle parity of each entry point is tested elsewhere on the layout the library picks
(interleaved rows on the small grids, separate arrays on the 512 x 512 planes); here each
path is run in both layouts on ragged grids and compared bit for bit."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import workloads as W
from helpers import random_state

pytestmark = pytest.mark.gpu

H, DT = 10.0, 5e-4
LAYOUTS = ("separate", "rows")


def model(shape, seed=21):
    return W.layered_perturbed(shape, H, seed)


def shot(shape, nt, seed=5):
    nx, ny, nz = shape
    rng = np.random.Generator(np.random.PCG64(seed))
    rec = np.stack([rng.uniform(3, nx - 4, 12), rng.uniform(3, ny - 4, 12), rng.uniform(2, nz - 4, 12)], axis=1)
    return dict(src_pos=(nx / 2 + 0.3, ny / 2 - 0.2, nz / 2 + 0.45), moment=W.random_mt(rng, 1e15),
                force=(2e9, -1e9, 3e9), wavelet=W.ricker(40.0, nt, DT, t0=0.006), rec_pos=rec)


def sims(lam, mu, rho, nt, dtype, **kw):
    from paper_2112_15071_amd import Simulator

    out = {lay: Simulator(lam, mu, rho, H, DT, nt, dtype=dtype, layout=lay, **kw) for lay in LAYOUTS}
    for lay, s in out.items():
        assert s.layout() == lay
    return out


def close(d):
    for s in d.values():
        s.close()


def test_auto_layout_choice():
    from paper_2112_15071_amd import Simulator

    lam, mu, rho = model((40, 36, 30))
    s = Simulator(lam, mu, rho, H, DT, 4)
    assert s.layout() == "rows"  # a whole-depth sweep of 9 rows fits one buffer window
    s.close()


KERNELS = [None, ("tile", 8, 16, 64), ("tile", 4, 8, 128), ("cell", 4, 8, 64), ("fused", 4, 16, 64)]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("fs", [False, True])
@pytest.mark.parametrize("kernel", KERNELS)
def test_forward_equal_in_both_layouts(dtype, fs, kernel):
    shape, nt = (70, 44, 38), 48
    print(f"[layout] forward {shape} x {nt} {dtype} fs={fs} kernel={kernel}", flush=True)
    lam, mu, rho = model(shape)
    d = sims(lam, mu, rho, nt, dtype, sponge=6, free_surface=fs)
    out = {}
    for lay, s in d.items():
        if kernel is not None:
            s.set_kernel(*kernel)
        tr = s.forward(**shot(shape, nt))
        out[lay] = (tr.clone(), s.state())
    torch.cuda.synchronize()
    a, b = out["separate"], out["rows"]
    assert float(a[0].abs().max()) > 0.0
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    close(d)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_state_roundtrip_and_continuation(dtype):
    shape, nt = (45, 38, 33), 20
    print(f"[layout] set/get state and continuation {shape} {dtype}", flush=True)
    lam, mu, rho = model(shape)
    st0 = random_state(shape, np.random.default_rng(3))
    d = sims(lam, mu, rho, nt, dtype, sponge=5)
    out = {}
    for lay, s in d.items():
        s.set_state(st0)
        got = s.state().double().cpu().numpy()
        assert np.array_equal(got, st0.astype(np.float32 if dtype == torch.float32 else np.float64)), lay
        tr = s.forward(**shot(shape, nt), keep_state=True)
        out[lay] = (tr.clone(), s.state())
    torch.cuda.synchronize()
    assert torch.equal(out["separate"][0], out["rows"][0]) and torch.equal(out["separate"][1], out["rows"][1])
    close(d)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("kernel", [None, ("cell", 4, 8, 64)])
def test_gradient_equal_in_both_layouts(dtype, kernel):
    lam, mu, rho, srcs, rec = W.small_fd_case(shape=(34, 31, 29), nt=60)
    nt = 60
    print(f"[layout] gradient 34x31x29 x {nt} {dtype} kernel={kernel}", flush=True)
    shots = [dict(src_pos=srcs[0], moment=W.explosion(1e15), wavelet=W.ricker(25.0, nt, 1e-3), rec_pos=rec),
             dict(src_pos=srcs[1], force=(3e9, -2e9, 4e9), wavelet=W.ricker(25.0, nt, 1e-3), rec_pos=rec)]
    from paper_2112_15071_amd import Simulator

    out = {}
    for lay in LAYOUTS:
        s = Simulator(lam, mu, rho, H, 1e-3, nt, dtype=dtype, sponge=6, sponge_alpha=0.05, layout=lay)
        if kernel is not None:
            s.set_kernel(*kernel)
        gws = s.grad_workspace(9)
        g = [torch.zeros(lam.shape, dtype=dtype, device="cuda") for _ in range(3)]
        Js = []
        for sh in shots:
            obs = torch.zeros((rec.shape[0], 3, nt), dtype=dtype)
            tr, j = s.gradient(gws, obs, *g, **sh)
            Js.append(j.clone())
        out[lay] = (torch.cat(Js), g, s.adjoint_state(gws))
        torch.cuda.synchronize()
        s.close()
    a, b = out["separate"], out["rows"]
    assert float(a[0].min()) > 0.0
    assert torch.equal(a[0], b[0])
    for p in range(3):
        assert float(a[1][p].abs().max()) > 0.0
        assert torch.equal(a[1][p], b[1][p]), p
    assert torch.equal(a[2], b[2])


@pytest.mark.parametrize("kernel", [None, ("cell", 4, 8, 64)])
def test_born_equal_in_both_layouts(kernel):
    shape, nt = (40, 37, 33), 40
    print(f"[layout] born {shape} x {nt} kernel={kernel}", flush=True)
    lam, mu, rho = model(shape)
    rng = np.random.default_rng(9)
    dm = [0.01 * a * rng.standard_normal(a.shape) for a in (lam, mu, rho)]
    d = sims(lam, mu, rho, nt, torch.float32, sponge=5)
    out = {}
    for lay, s in d.items():
        if kernel is not None:
            s.set_kernel(*kernel)
        tr, dtr = s.born(*dm, **shot(shape, nt))
        out[lay] = (tr.clone(), dtr.clone())
    torch.cuda.synchronize()
    assert float(out["rows"][1].abs().max()) > 0.0
    assert torch.equal(out["separate"][0], out["rows"][0]) and torch.equal(out["separate"][1], out["rows"][1])
    close(d)


def test_coarse_medium_equal_in_both_layouts():
    from paper_2112_15071_amd import Simulator

    grid, coarse, nt = (48, 40, 36), (10, 9, 8), 30
    print(f"[layout] coarse medium {coarse} on {grid} x {nt}", flush=True)
    lam, mu, rho = model(coarse, seed=4)
    out = {}
    for lay in LAYOUTS:
        s = Simulator(lam, mu, rho, H, DT, nt, sponge=5, grid=grid, layout=lay)
        assert s.layout() == lay
        tr = s.forward(**shot(grid, nt))
        out[lay] = (tr.clone(), s.state())
        torch.cuda.synchronize()
        s.close()
    assert torch.equal(out["separate"][0], out["rows"][0]) and torch.equal(out["separate"][1], out["rows"][1])


@pytest.mark.parametrize("kernel", [None, ("cell", 4, 8, 64)])
def test_vacuum_equal_in_both_layouts(kernel):
    shape, nt, ks = (44, 40, 36), 30, 6
    print(f"[layout] vacuum surface at plane {ks}, kernel={kernel}", flush=True)
    lam, mu, rho = model(shape)
    lam, mu, rho = lam.copy(), mu.copy(), rho.copy()
    lam[:ks], mu[:ks], rho[:ks] = 0.0, 0.0, 0.05 * rho[ks:].min()
    d = sims(lam, mu, rho, nt, torch.float32, sponge=(5, 5, 5, 5, 0, 5), vacuum_top=ks)
    out = {}
    for lay, s in d.items():
        if kernel is not None:
            s.set_kernel(*kernel)
        sh = shot(shape, nt)
        sh["src_pos"] = (22.3, 19.6, 14.2)
        sh["rec_pos"] = np.array([[10.0 + 2 * r, 12.0, ks + 1.0] for r in range(8)])
        tr = s.forward(**sh)
        out[lay] = (tr.clone(), s.state())
    torch.cuda.synchronize()
    assert torch.equal(out["separate"][0], out["rows"][0]) and torch.equal(out["separate"][1], out["rows"][1])
    close(d)


def test_batch_with_mixed_layouts_equals_single_shots():
    """A batch whose shots use different layouts (each shot's launch descriptor carries its
    own strides): forward through the graph and the batched gradient, each shot equal to
    its single-shot run."""
    from paper_2112_15071_amd import Simulator
    from paper_2112_15071_amd.batch import BatchSimulator

    nt = 24
    shapes = [(40, 36, 30), (48, 40, 32), (40, 36, 30)]
    lays = ["rows", "separate", "separate"]
    print(f"[layout] batch {shapes} {lays} x {nt}", flush=True)
    mods = [model(s, seed=30 + k) for k, s in enumerate(shapes)]
    shots = [shot(s, nt, seed=40 + k) for k, s in enumerate(shapes)]
    ref = []
    for m, sh, lay in zip(mods, shots, lays):
        s = Simulator(*m, H, DT, nt, sponge=5, layout=lay)
        ref.append((s.forward(**sh).clone(), s.state()))
        torch.cuda.synchronize()
        s.close()
    bs = [Simulator(*m, H, DT, nt, sponge=5, layout=lay) for m, lay in zip(mods, lays)]
    batch = BatchSimulator(bs)
    trs = batch.forward(shots, use_graph=True)
    torch.cuda.synchronize()
    for k, s in enumerate(bs):
        assert torch.equal(trs[k], ref[k][0]), k
        assert torch.equal(s.state(), ref[k][1]), k
    # batched gradient (lockstep) against per-shot gradients
    obs = [torch.zeros_like(t) for t in trs]
    g_b = [[torch.zeros(m[0].shape, dtype=torch.float32, device="cuda") for _ in range(3)] for m in mods]
    _, misfit = batch.gradient(shots, obs, [g[0] for g in g_b], [g[1] for g in g_b], [g[2] for g in g_b],
                               ckpt_every=8)
    torch.cuda.synchronize()
    for k, (m, sh, lay) in enumerate(zip(mods, shots, lays)):
        s = Simulator(*m, H, DT, nt, sponge=5, layout=lay)
        gws = s.grad_workspace(8)
        g = [torch.zeros(m[0].shape, dtype=torch.float32, device="cuda") for _ in range(3)]
        _, j = s.gradient(gws, obs[k], *g, **sh)
        torch.cuda.synchronize()
        assert torch.equal(j, misfit[k:k + 1]), k
        for p in range(3):
            assert torch.equal(g[p], g_b[k][p]), (k, p)
        s.close()
    batch.close()
    for s in bs:
        s.close()


def test_batch_shots_over_one_model_share_its_copy():
    """Shots created over the same model tensors (interleaved rows: each context holds a
    copy) read the first shot's copy inside a batch; a shot over other tensors keeps its
    own.  Forward and gradient of every shot equal its single-shot run."""
    from paper_2112_15071_amd import Simulator
    from paper_2112_15071_amd.batch import BatchSimulator

    nt, shape = 24, (44, 40, 34)
    print(f"[layout] batch over one shared model {shape} x {nt}", flush=True)
    shared = [torch.as_tensor(a, dtype=torch.float32, device="cuda") for a in model(shape, seed=50)]
    other = [torch.as_tensor(a, dtype=torch.float32, device="cuda") for a in model(shape, seed=51)]
    mods = [shared, shared, other, shared]
    shots = [shot(shape, nt, seed=60 + k) for k in range(4)]
    ref = []
    for m, sh in zip(mods, shots):
        s = Simulator(*m, H, DT, nt, sponge=5)
        assert s.layout() == "rows"
        tr = s.forward(**sh).clone()
        gws = s.grad_workspace(8)
        g = [torch.zeros(shape[::-1], dtype=torch.float32, device="cuda") for _ in range(3)]
        _, j = s.gradient(gws, torch.zeros_like(tr), *g, **sh)
        torch.cuda.synchronize()
        ref.append((tr, j.clone(), g))
        s.close()
    bs = [Simulator(*m, H, DT, nt, sponge=5) for m in mods]
    batch = BatchSimulator(bs)
    trs = batch.forward(shots, use_graph=True)
    torch.cuda.synchronize()
    for k in range(4):
        assert torch.equal(trs[k], ref[k][0]), k
    g_b = [[torch.zeros(shape[::-1], dtype=torch.float32, device="cuda") for _ in range(3)] for _ in mods]
    _, misfit = batch.gradient(shots, [torch.zeros_like(t) for t in trs], [g[0] for g in g_b],
                               [g[1] for g in g_b], [g[2] for g in g_b], ckpt_every=8)
    torch.cuda.synchronize()
    for k in range(4):
        assert torch.equal(misfit[k:k + 1], ref[k][1]), k
        for p in range(3):
            assert torch.equal(g_b[k][p], ref[k][2][p]), (k, p)
    batch.close()
    for s in bs:
        s.close()
