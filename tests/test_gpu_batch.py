"""Batched stepping: many uneven shots in one persistent launch per pass, eager or
replayed from one hipGraph, give per-shot results identical to single-shot runs with the
same tile shape (and so the oracle's)."""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_cases import compare, oracle_run
from helpers import rel_l2

pytestmark = pytest.mark.gpu

SHAPES = [(40, 36, 28), (52, 33, 30), (37, 29, 23), (64, 40, 32)]
NT, DT = 80, 5e-4


def make_shots(seed, fs=False):
    shots = []
    for s, shape in enumerate(SHAPES):
        rng = np.random.Generator(np.random.PCG64(seed + s))
        lam, mu, rho = W.layered_perturbed(shape, 10.0, seed + 10 + s)
        nx, ny, nz = shape
        pos = (float(rng.uniform(8, nx - 9)), float(rng.uniform(8, ny - 9)), float(rng.uniform(6, nz - 7)))
        rec = np.stack([rng.uniform(3, nx - 4, 5), rng.uniform(3, ny - 4, 5), rng.uniform(1, nz - 4, 5)], axis=1)
        sponge = (5, 5, 5, 5, 0 if fs else 5, 5)
        shots.append(W.Shot(f"b{s}", shape, 10.0, DT, NT, lam, mu, rho, pos, W.random_mt(rng),
                            tuple(rng.standard_normal(3) * 1e9), W.ricker(40.0, NT, DT), rec, sponge=sponge,
                            free_surface=fs))
    return shots


def sims_for(shots, dtype=torch.float32):
    from paper_2112_15071_amd import Simulator

    return [Simulator(s.lam, s.mu, s.rho, s.h, s.dt, s.nt, dtype=dtype, sponge=s.sponge,
                      free_surface=s.free_surface) for s in shots]


def desc(s, scale=1.0):
    return dict(src_pos=s.src_pos, moment=tuple(scale * m for m in s.moment), force=s.force, wavelet=s.wavelet,
                rec_pos=s.rec_pos)


def shot_tile(shape, tile, tile2=None):
    """The tile shape a batch gives a shot: the second shape when it covers the rows with
    fewer idle columns."""
    if tile2 and tile2[0]:
        pad = lambda tx: -(-shape[0] // tx) * tx
        if pad(tile2[0]) < pad(tile[0]):
            return tile2
    return tile


def single_runs(shots, tile, scale=1.0, dtype=torch.float32, tile2=None):
    out = []
    for sim, s in zip(sims_for(shots, dtype), shots):
        t = shot_tile(s.shape, tile, tile2)
        sim.set_kernel("tile", t[1], sim.kernel()["zchunk"], t[0])
        tr = sim.forward(**desc(s, scale))
        out.append((tr.double().cpu().numpy(), sim.state().double().cpu().numpy()))
        sim.close()
    return out


@pytest.mark.parametrize("fs", [False, True])
@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_equals_single_shots(fs, use_graph):
    from paper_2112_15071_amd.batch import BatchSimulator

    shots = make_shots(500 + int(fs), fs)
    tile = (64, 8)
    ref = single_runs(shots, tile)
    sims = sims_for(shots)
    batch = BatchSimulator(sims)
    batch.set_kernel(*tile)
    print(f"[batch] fs={fs} graph={use_graph}", flush=True)
    trs = batch.forward([desc(s) for s in shots], use_graph=use_graph)
    torch.cuda.synchronize()
    for k, (sim, tr) in enumerate(zip(sims, trs)):
        assert np.array_equal(tr.double().cpu().numpy(), ref[k][0]), k
        assert np.array_equal(sim.state().double().cpu().numpy(), ref[k][1]), k
    # one shot against the oracle as well
    compare((trs[2].double().cpu().numpy(), sims[2].state().double().cpu().numpy()), oracle_run(shots[2]), 1e-4,
            "batched shot 2")
    batch.close()
    for s in sims:
        s.close()


def test_batch_autotune_then_forward():
    """After the batch autotuner (which runs sourceless steps on every shot), a batched
    forward on the chosen tile shape and grid mode equals single-shot runs."""
    from paper_2112_15071_amd.batch import BatchSimulator

    shots = make_shots(600)
    sims = sims_for(shots)
    batch = BatchSimulator(sims)
    best = batch.autotune(steps=3, cache=False)
    print(f"[batch] autotune -> {best['tile_x']}x{best['tile_y']} wg={best['workgroups']}", flush=True)
    assert best["ms_per_step"] > 0
    trs = batch.forward([desc(s) for s in shots], use_graph=True)
    torch.cuda.synchronize()
    ref = single_runs(shots, (best["tile_x"], best["tile_y"]), tile2=(best["tile2_x"], best["tile2_y"]))
    for k, (sim, tr) in enumerate(zip(sims, trs)):
        assert np.array_equal(tr.double().cpu().numpy(), ref[k][0]), k
        assert np.array_equal(sim.state().double().cpu().numpy(), ref[k][1]), k
    batch.close()
    for s in sims:
        s.close()


PAIR_SHAPES = [(128, 20, 18), (64, 24, 20), (192, 18, 16), (100, 22, 19)]


@pytest.mark.parametrize("pair,use_graph", [(((128, 8), (64, 16)), True), (((256, 4), (64, 16)), False),
                                            (((256, 4), (128, 8)), True), (((128, 4), (64, 8)), False)])
def test_batch_two_tile_shapes(pair, use_graph):
    """Rows of 128, 64, 192 and 100 samples in one batch with two tile shapes: each shot
    takes the shape with fewer idle columns and equals its single-shot run."""
    from paper_2112_15071_amd.batch import BatchSimulator

    shots = []
    for s, shape in enumerate(PAIR_SHAPES):
        rng = np.random.Generator(np.random.PCG64(1300 + s))
        lam, mu, rho = W.layered_perturbed(shape, 10.0, 1310 + s)
        nx, ny, nz = shape
        pos = (float(rng.uniform(8, nx - 9)), float(rng.uniform(6, ny - 7)), float(rng.uniform(6, nz - 7)))
        rec = np.stack([rng.uniform(3, nx - 4, 4), rng.uniform(3, ny - 4, 4), rng.uniform(2, nz - 4, 4)], axis=1)
        shots.append(W.Shot(f"p{s}", shape, 10.0, DT, 60, lam, mu, rho, pos, W.random_mt(rng),
                            tuple(rng.standard_normal(3) * 1e9), W.ricker(40.0, 60, DT), rec, sponge=(4,) * 6))
    tile, tile2 = pair
    ref = single_runs(shots, tile, tile2=tile2)
    sims = sims_for(shots)
    batch = BatchSimulator(sims)
    batch.set_kernel(*tile, tile2=tile2)
    print(f"[batch] pair {tile} + {tile2} graph={use_graph}", flush=True)
    trs = batch.forward([desc(s) for s in shots], use_graph=use_graph)
    torch.cuda.synchronize()
    for k, (sim, tr) in enumerate(zip(sims, trs)):
        assert np.array_equal(tr.double().cpu().numpy(), ref[k][0]), k
        assert np.array_equal(sim.state().double().cpu().numpy(), ref[k][1]), k
    batch.close()
    for s in sims:
        s.close()


def test_one_workgroup_per_tile_equals_persistent():
    from paper_2112_15071_amd.batch import BatchSimulator

    shots = make_shots(650)
    out = []
    for wg in (8, 4096):  # 8 workgroups: many tiles each; 4096: one tile each
        sims = sims_for(shots)
        batch = BatchSimulator(sims)
        batch.set_kernel(64, 8, wg)
        trs = batch.forward([desc(s) for s in shots], use_graph=False)
        torch.cuda.synchronize()
        out.append([(t.cpu(), s.state().cpu()) for t, s in zip(trs, sims)])
        batch.close()
        for s in sims:
            s.close()
    for (ta, sa), (tb, sb) in zip(*out):
        assert torch.equal(ta, tb) and torch.equal(sa, sb)


def test_graph_replays_with_new_sources():
    """Replays of the captured graph, with eager work and synchronisation in between,
    each match eager single-shot runs for the sources of that replay."""
    from paper_2112_15071_amd.batch import BatchSimulator

    shots = make_shots(700)
    tile = (64, 8)
    sims = sims_for(shots)
    batch = BatchSimulator(sims)
    batch.set_kernel(*tile)
    for rep, scale in enumerate((1.0, -0.5, 2.0)):
        trs = batch.forward([desc(s, scale) for s in shots], use_graph=True)
        torch.cuda.synchronize()
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        ref = single_runs(shots, tile, scale)
        for k, (sim, tr) in enumerate(zip(sims, trs)):
            assert np.array_equal(tr.double().cpu().numpy(), ref[k][0]), (rep, k)
            assert np.array_equal(sim.state().double().cpu().numpy(), ref[k][1]), (rep, k)
        del junk
    batch.close()
    for s in sims:
        s.close()


def early_c3(nt):
    """The 24-shot uneven batch at full size with wavelets that peak within a truncated
    run and four extra receivers 4-6 cells from each source, so traces are non-zero."""
    import dataclasses

    out = []
    for s in W.c3(nt=nt):
        near = np.asarray(s.src_pos) + np.array([[4.3, 0.2, -1.5], [-5.1, 1.4, 0.5], [0.7, 4.6, 2.25],
                                                 [-1.2, -5.3, -2.75]])
        out.append(dataclasses.replace(s, wavelet=W.ricker(10.0, nt, s.dt, t0=0.004),
                                       rec_pos=np.concatenate([s.rec_pos, near])))
    return out


def test_full_size_uneven_batch_truncated():
    """The 24-shot uneven batch at full size (128^3 .. 256x256x128), 12 steps, lockstep
    with the batch's default tile shape: every shot equals its single-shot run."""
    from paper_2112_15071_amd import Simulator
    from paper_2112_15071_amd.batch import BatchSimulator

    nt = 12
    shots = early_c3(nt)
    print(f"[batch] 24 uneven shots x {nt}", flush=True)
    sims = [Simulator(s.lam, s.mu, s.rho, s.h, s.dt, nt, sponge=s.sponge) for s in shots]
    batch = BatchSimulator(sims)
    trs = batch.forward([desc(s) for s in shots], use_graph=True)
    torch.cuda.synchronize()
    tile = (128, 4)  # the batch default for these widths
    for k, s in enumerate(shots):
        one = Simulator(s.lam, s.mu, s.rho, s.h, s.dt, nt, sponge=s.sponge)
        one.set_kernel("tile", tile[1], one.kernel()["zchunk"], tile[0])
        tr = one.forward(**desc(s))
        assert float(tr.abs().max()) > 0, k
        assert torch.equal(tr, trs[k]), k
        assert torch.equal(one.state(), sims[k].state()), k
        one.close()
    batch.close()
    for s in sims:
        s.close()


def test_full_size_uneven_batch_bench_schedule():
    """The 24-shot batch at full size in the benchmark's configuration: the batch tuner
    (per-shape kernels, batched tile shapes, cache-blocked group budgets) decides the
    launches, then a 192 MiB group budget (the benchmark's pick on MI355X) is run as well;
    16 steps replayed twice from the graph.  Every shot equals its single-shot run with its
    own tuned kernel bit for bit, and one shot of each size matches the oracle."""
    from paper_2112_15071_amd import Simulator
    from paper_2112_15071_amd.batch import BatchSimulator

    nt = 16
    shots = early_c3(nt)
    sims = [Simulator(s.lam, s.mu, s.rho, s.h, s.dt, nt, sponge=s.sponge) for s in shots]
    batch = BatchSimulator(sims)
    tune = batch.autotune(steps=3, cache=False)
    print(f"[batch] bench schedule: tuned group budget {tune['group_mib']} MiB, tiles "
          f"{tune['tile_x']}x{tune['tile_y']} + {tune['tile2_x']}x{tune['tile2_y']}", flush=True)
    ref = []
    for k, s in enumerate(shots):
        one = Simulator(s.lam, s.mu, s.rho, s.h, s.dt, nt, sponge=s.sponge)
        kern = sims[k].kernel()
        one.set_kernel(kern["variant"], kern["tile_y"], kern["zchunk"], kern["tile_x"])
        ref.append((one.forward(**desc(s)).clone(), one.state()))
        one.close()
    for budget in (None, 192 << 20):
        if budget is not None:
            batch.set_schedule(budget)
        for rep in range(2):
            trs = batch.forward([desc(s) for s in shots], use_graph=True)
            torch.cuda.synchronize()
            for k in range(len(shots)):
                assert torch.equal(trs[k], ref[k][0]), (budget, rep, k)
                assert torch.equal(sims[k].state(), ref[k][1]), (budget, rep, k)
    seen = set()
    for k, s in enumerate(shots):
        if s.shape in seen:
            continue
        seen.add(s.shape)
        print(f"[batch] bench schedule: shot {k} {s.shape} against the oracle", flush=True)
        compare((ref[k][0].double().cpu().numpy(), ref[k][1].double().cpu().numpy()), oracle_run(s), 1e-4,
                f"batched shot {k} {s.shape}")
    batch.close()
    for s in sims:
        s.close()


GSHAPES = [(32, 32, 32), (36, 30, 28), (40, 34, 30)]


def grad_shots(seed, nt):
    shots = []
    for s, shape in enumerate(GSHAPES):
        rng = np.random.Generator(np.random.PCG64(seed + s))
        lam, mu, rho = W.layered_perturbed(shape, 10.0, seed + 20 + s)
        nx, ny, nz = shape
        pos = (float(rng.uniform(8, nx - 9)), float(rng.uniform(8, ny - 9)), float(rng.uniform(6, nz - 7)))
        rec = np.stack([rng.uniform(4, nx - 5, 6), rng.uniform(4, ny - 5, 6), np.full(6, 6.0)], axis=1)
        shots.append(W.Shot(f"g{s}", shape, 10.0, DT, nt, lam, mu, rho, pos, W.explosion(1e15),
                            tuple(rng.standard_normal(3) * 1e9), W.ricker(40.0, nt, DT), rec, sponge=(6,) * 6))
    return shots


@pytest.mark.parametrize("tile2", [None, (64, 8)])
def test_batched_gradient_equals_per_shot(tile2):
    """Every shot's gradient equals its single-shot gradient bitwise; with tile2 the batch
    runs 128x4 + 64x8 and every (narrow) shot takes the second shape."""
    from paper_2112_15071_amd.batch import BatchSimulator

    nt, k = 60, 7
    shots = grad_shots(900, nt)
    rng = np.random.default_rng(5)
    d_obs = [torch.as_tensor(rng.standard_normal((len(s.rec_pos), 3, nt)) * 1e-6, dtype=torch.float32) for s in shots]
    tile = (64, 8)
    ref = []
    for s, obs in zip(shots, d_obs):
        sim = sims_for([s])[0]
        sim.set_kernel("tile", tile[1], sim.kernel()["zchunk"], tile[0])
        g = [torch.zeros(s.lam.shape, dtype=torch.float32, device="cuda") for _ in range(3)]
        tr, J = sim.gradient(sim.grad_workspace(k), obs, *g, **desc(s))
        ref.append((tr.cpu(), J.cpu(), [x.cpu() for x in g]))
        sim.close()
    sims = sims_for(shots)
    batch = BatchSimulator(sims)
    if tile2:
        batch.set_kernel(128, 4, tile2=tile2)
    else:
        batch.set_kernel(*tile)
    gl = [torch.zeros(s.lam.shape, dtype=torch.float32, device="cuda") for s in shots]
    gm = [torch.zeros_like(x) for x in gl]
    gr = [torch.zeros_like(x) for x in gl]
    print("[batch-grad] 3 shots", flush=True)
    trs, J = batch.gradient([desc(s) for s in shots], d_obs, gl, gm, gr, ckpt_every=k)
    torch.cuda.synchronize()
    for q in range(3):
        assert torch.equal(trs[q].cpu(), ref[q][0]), q
        assert torch.equal(J[q:q + 1].cpu(), ref[q][1]), q
        for a, b in zip((gl[q], gm[q], gr[q]), ref[q][2]):
            assert torch.equal(a.cpu(), b), q
    batch.close()
    for s in sims:
        s.close()


@pytest.mark.parametrize("dtype,tol", [(torch.float32, 1e-5), (torch.float64, 1e-12)])
def test_batched_gradient_dot_product(dtype, tol):
    """Per shot, sources off, start from a random state x0, d_obs = 0 (so the residual is
    d = P x0): <d, d> = <x0, P^T d> with P^T d the adjoint of the initial state."""
    from paper_2112_15071_amd.batch import BatchSimulator
    from helpers import random_state

    nt, k = 40, 9
    shots = grad_shots(950, nt)
    rng = np.random.default_rng(6)
    sims = sims_for(shots, dtype)
    x0 = []
    for sim, s in zip(sims, shots):
        sim.set_state(torch.as_tensor(random_state(s.shape, rng), dtype=dtype))
        x0.append(sim.state().double().cpu().numpy())
    batch = BatchSimulator(sims)
    d_obs = [torch.zeros((len(s.rec_pos), 3, nt), dtype=dtype) for s in shots]
    g = [torch.zeros(s.lam.shape, dtype=dtype, device="cuda") for s in shots]
    gws = [sim.grad_workspace(k) for sim in sims]
    nosrc = [dict(src_pos=None, rec_pos=s.rec_pos) for s in shots]
    trs, J = batch.gradient(nosrc, d_obs, g, [torch.zeros_like(x) for x in g], [torch.zeros_like(x) for x in g],
                            ckpt_every=k, gws=gws, keep_state=True)
    for q, sim in enumerate(sims):
        d = trs[q].double().cpu().numpy()
        adj = sim.adjoint_state(gws[q]).double().cpu().numpy()
        lhs, rhs = float(np.sum(d * d)), float(np.sum(x0[q] * adj))
        assert lhs > 0 and abs(lhs - rhs) <= tol * abs(lhs), (q, lhs, rhs)
    batch.close()
    for s in sims:
        s.close()


@pytest.mark.parametrize("use_graph", [False, True])
def test_cache_blocked_groups_equal_single_shots(use_graph):
    """The cache-blocked schedule (shots sorted by working set, cut into groups within a
    byte budget, each group stepped through all its steps before the next) gives every
    shot its single-shot result.  Budget 4 MB on these shots (1.2, 1.9, 2.5 and 3.9 MB of
    fields and model): groups {2, 0}, {1}, {3}; the first two launch with their shots' own
    tile shapes, shot 3 (cell kernel) with the batch's shape."""
    from paper_2112_15071_amd.batch import BatchSimulator

    shots = make_shots(700)
    ref = single_runs(shots, (64, 8))
    sims = sims_for(shots)
    for sim, kern in zip(sims, [("tile", 8, 64), ("tile", 4, 64), ("tile", 8, 64), ("cell", 8, 32)]):
        sim.set_kernel(kern[0], kern[1], sim.kernel()["zchunk"], kern[2])
    batch = BatchSimulator(sims)
    batch.set_kernel(128, 4)
    batch.set_schedule(4 << 20)
    print(f"[batch] cache-blocked groups graph={use_graph}", flush=True)
    for rep in range(2):
        trs = batch.forward([desc(s) for s in shots], use_graph=use_graph)
        torch.cuda.synchronize()
        for k, (sim, tr) in enumerate(zip(sims, trs)):
            assert np.array_equal(tr.double().cpu().numpy(), ref[k][0]), (rep, k)
            assert np.array_equal(sim.state().double().cpu().numpy(), ref[k][1]), (rep, k)
    # back to lockstep on the same batch
    batch.set_schedule(0)
    trs = batch.forward([desc(s) for s in shots], use_graph=use_graph)
    torch.cuda.synchronize()
    for k, tr in enumerate(trs):
        assert np.array_equal(tr.double().cpu().numpy(), ref[k][0]), k
    batch.close()
    for s in sims:
        s.close()


@pytest.mark.parametrize("group_bytes", [0, 4 << 20])
def test_many_receivers_batch_equals_single_shots(group_bytes):
    """Receiver counts of 700, 1, 350 and 45 per shot: the batched stress launches sample
    3288 items over four 1024-thread workgroups, with shot boundaries inside a workgroup, in
    the lockstep schedule and in cache-blocked groups; every shot equals its single-shot run
    (whose stress launch samples its own receivers, 2100 items over three workgroups)."""
    import dataclasses

    from paper_2112_15071_amd.batch import BatchSimulator

    shots = make_shots(720)
    rng = np.random.default_rng(72)
    for q, m in enumerate((700, 1, 350, 45)):
        nx, ny, nz = shots[q].shape
        rec = np.stack([rng.uniform(3, nx - 4, m), rng.uniform(3, ny - 4, m), rng.uniform(1, nz - 4, m)], axis=1)
        shots[q] = dataclasses.replace(shots[q], rec_pos=rec)
    tile = (128, 8)
    ref = single_runs(shots, tile)
    sims = sims_for(shots)
    batch = BatchSimulator(sims)
    batch.set_kernel(*tile)
    batch.set_schedule(group_bytes)
    print(f"[batch] many receivers, group bytes {group_bytes}", flush=True)
    for use_graph in (False, True):
        trs = batch.forward([desc(s) for s in shots], use_graph=use_graph)
        torch.cuda.synchronize()
        for k, (sim, tr) in enumerate(zip(sims, trs)):
            assert tr.shape[0] == len(shots[k].rec_pos)
            assert np.array_equal(tr.double().cpu().numpy(), ref[k][0]), (use_graph, k)
            assert np.array_equal(sim.state().double().cpu().numpy(), ref[k][1]), (use_graph, k)
    # the shot with the most receivers against the oracle as well
    compare((trs[0].double().cpu().numpy(), sims[0].state().double().cpu().numpy()), oracle_run(shots[0]), 1e-4,
            "batched shot 0, 700 receivers")
    batch.close()
    for s in sims:
        s.close()
