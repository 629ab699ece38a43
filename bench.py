"""Benchmark of the elastic FD hot path on one MI355X.

Headline (``value``): forward throughput in Gcell-steps/s on the 256^3 six-layer +
5 % Gaussian-perturbed model (h 10 m, dt 0.5 ms, 2000 steps), random moment-tensor
source, 12 Hz Ricker, 256 receivers, 20-cell sponge, FP32.  A "step" is one time step of
the whole forward path: velocity pass (force source, damping), then the stress pass
(moment source, damping) whose launch also samples the receivers.

Also reported (same JSON line):
  batched  -- the 24-shot uneven batch (128^3 .. 256x256x128, 1500 steps): per-shot loop
              vs one persistent launch per pass replayed from a hipGraph (Gcell-steps/s);
  gradient -- the 8-shot 256^3 FWI gradient (1500 steps, checkpoints every 50): per-shot
              loop vs batched waves (shots/s), each with the kernel configuration its
              gradient tuner picks;
  roofline -- the dominant forward kernel's algorithmic bytes / its HIP-event duration;
  c2_forward -- the 512x512x256 free-surface workload (300 steps);
  stream_copy_gbs -- a plain 1 GiB device copy (read + write GB/s), the practical ceiling;
  born     -- the tangent-linear (Born) forward on the 256^3 model, 300 steps;
  levels   -- the paper's Table 5 level sweep (64x64x32 .. 512^3, anisotropic cells) on
              its case-study medium (seven layers under 30 km of air: vacuum surface),
              upsampled from one coarse grid to every level, 100 timed steps per level;
  cpu_baseline -- the FP64 oracle on a bounded sample on this host's cores (and, as
              one_core, on a single core over an eighth of the steps).

    python bench.py [--steps 2000] [--warmup 100] [--gpus 1] [--no-batch] [--no-grad] [--no-levels]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# algorithmic (compulsory) bytes per cell per launch, FP32: every input field read once
# and every updated field written once
BYTES_PER_CELL = {
    "velocity": 4 * (6 + 3 + 1 + 3),  # read 6 stress, 3 velocity, rho; write 3 velocity
    "stress": 4 * (3 + 6 + 2 + 6),  # read 3 velocity, 6 stress, lambda, mu; write 6 stress
    "fused": 4 * (6 + 3 + 3 + 9),  # read 6 stress, 3 velocity, rho, lambda, mu; write 9
}


def step_bytes(kern):
    """Algorithmic bytes per cell and time step of the forward path with this kernel."""
    if kern["variant"] == "fused":
        return BYTES_PER_CELL["fused"]
    return BYTES_PER_CELL["velocity"] + BYTES_PER_CELL["stress"]
# gradient, per shot and time step: forward with checkpoints (120), segment recompute
# storing v^{n+1/2} and sigma^n (156), the four adjoint passes: stress-A 27 fields,
# velocity-A 12, velocity-B 19, stress-B 15 (292)
GRAD_BYTES_PER_CELL_STEP = 120 + 156 + 4 * (27 + 12 + 19 + 15)
# measured counter calibration (plain 1 GiB copy): FETCH_SIZE reads 0.5x, WRITE_SIZE 1.0x
FETCH_FACTOR, WRITE_FACTOR = 2.0, 1.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sync():
    import torch

    torch.cuda.synchronize()


def shot_desc(s):
    return dict(src_pos=s.src_pos, moment=s.moment, force=s.force, wavelet=s.wavelet, rec_pos=s.rec_pos)


def measured_traffic(kern, dom):
    """HBM bytes per launch of the dominant forward kernel from the committed counter
    table (rocprofv3 FETCH_SIZE / WRITE_SIZE, copy-calibrated), or None when the table
    has no entry for this kernel configuration or the kernel sources changed since."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "forward_tile_hbm_traffic.json")
    try:
        with open(path) as f:
            table = json.load(f)
        h = hashlib.sha256()
        for src in table["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        if h.hexdigest() != table["sources_sha256"]:
            return None
        key = f"{kern['variant']},{kern['tile_x']},{kern['tile_y']},{kern['zchunk']}"
        return table["kernels"][key][dom]["hbm_bytes"]
    except (OSError, KeyError, ValueError):
        return None


def bench_forward(K, Wm, kernel=None):
    import torch

    import workloads as W
    from paper_2112_15071_amd import Simulator, _abi

    dev = torch.device("cuda:0")
    log(f"[bench] 256^3 workload: steps {K}, warmup {Wm}")
    shot = W.c1(nt=max(K, Wm))
    nx, ny, nz = shot.shape
    cells = nx * ny * nz
    lam, mu, rho = (torch.as_tensor(a, dtype=torch.float32).to(dev) for a in (shot.lam, shot.mu, shot.rho))
    wav = torch.as_tensor(shot.wavelet, dtype=torch.float32).to(dev)
    kw = dict(dtype=torch.float32, sponge=shot.sponge, device=dev)
    sim = Simulator(lam, mu, rho, shot.h, shot.dt, K, **kw)
    if kernel:
        variant, tx, ty, zc = kernel.split(",")
        sim.set_kernel(variant, int(ty), int(zc), int(tx))
        log(f"[bench] kernel {sim.kernel()} (given)")
    else:
        tune = sim.autotune(steps=20)
        log(f"[bench] kernel {sim.kernel()} (autotune {'cached' if tune['cached'] else 'run'})")
    if Wm > 0:
        warm = Simulator(lam, mu, rho, shot.h, shot.dt, Wm, **kw)
        k = sim.kernel()
        warm.set_kernel(k["variant"], k["tile_y"], k["zchunk"], k["tile_x"])
        warm.forward(shot.src_pos, shot.moment, shot.force, wav[:Wm], shot.rec_pos)
        sync()
        warm.close()
    traces = torch.empty((shot.rec_pos.shape[0], 3, K), dtype=torch.float32, device=dev)
    sync()
    t0 = time.perf_counter()
    sim.forward(shot.src_pos, shot.moment, shot.force, wav[:K], shot.rec_pos, traces=traces)
    sync()
    elapsed = time.perf_counter() - t0
    gcs = cells * K / elapsed / 1e9
    log(f"[bench] forward {elapsed:.3f} s -> {gcs:.2f} Gcell-steps/s")
    # the same run again with per-kernel HIP events on the launch stream
    _abi.fd3d_profile(sim.ctx, True)
    sim.forward(shot.src_pos, shot.moment, shot.force, wav[:K], shot.rec_pos, traces=traces)
    ms, launches = _abi.fd3d_profile_read(sim.ctx)
    sync()
    _abi.fd3d_profile(sim.ctx, False)
    names = ("velocity", "record", "stress", "fused")
    per = {names[i]: ms[i] / launches[i] for i in range(4) if launches[i] > 0}
    if "fused" in per:
        dom = "fused"
    else:
        dom = "stress" if per["stress"] >= per["velocity"] else "velocity"
    bytes_launch = BYTES_PER_CELL[dom] * cells
    achieved = bytes_launch / (per[dom] * 1e-3) / 1e9
    both = step_bytes(sim.kernel()) * cells * K / (elapsed * 1e9)
    log(f"[bench] avg kernel ms {per}; dominant {dom} {achieved:.0f} GB/s; whole step {both:.0f} GB/s")
    kern = sim.kernel()
    sim.close()
    return shot, dict(gcs=gcs, elapsed=elapsed, per=per, dom=dom, achieved=achieved, bytes_launch=bytes_launch,
                      both=both, kernel=kern, traffic=measured_traffic(kern, dom))


def bench_c2(K=300):
    """The 512 x 512 x 256 free-surface workload (30-cell sponge on five faces), K steps."""
    import torch

    import workloads as W
    from paper_2112_15071_amd import Simulator

    dev = torch.device("cuda:0")
    log(f"[bench] 512x512x256 free-surface workload: {K} steps")
    shot = W.c2(nt=K)
    lam, mu, rho = (torch.as_tensor(a, dtype=torch.float32).to(dev) for a in (shot.lam, shot.mu, shot.rho))
    wav = torch.as_tensor(shot.wavelet, dtype=torch.float32).to(dev)
    sim = Simulator(lam, mu, rho, shot.h, shot.dt, K, sponge=shot.sponge, free_surface=True, device=dev)
    sim.autotune(steps=10)
    traces = torch.empty((shot.rec_pos.shape[0], 3, K), dtype=torch.float32, device=dev)
    sim.forward(shot.src_pos, shot.moment, shot.force, wav, shot.rec_pos, traces=traces)  # warm-up
    sync()
    t0 = time.perf_counter()
    sim.forward(shot.src_pos, shot.moment, shot.force, wav, shot.rec_pos, traces=traces)
    sync()
    el = time.perf_counter() - t0
    kern = sim.kernel()
    sim.close()
    gcs = shot.cells * K / el / 1e9
    gbs = step_bytes(kern) * shot.cells * K / el / 1e9
    log(f"[bench] c2: {el:.3f} s -> {gcs:.2f} Gcell-steps/s, {gbs:.0f} GB/s")
    return dict(gcs=round(gcs, 3), steps=K, seconds=round(el, 4), kernel=kern, hbm_gbs_whole_step=round(gbs, 1),
                hbm_frac_whole_step=round(gbs / HBM_PEAK_GBS, 4))


def stream_copy_ceiling(reps=20):
    """Device-to-device copy of 1 GiB with torch, timed with HIP events on the current
    stream: read + write bytes per second (the practical HBM ceiling of a plain stream)."""
    import torch

    n = 1 << 28
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    gbs = 2 * 4 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    log(f"[bench] 1 GiB device copy: {gbs:.0f} GB/s")
    return round(gbs, 1)


def bench_batch():
    import torch

    import workloads as W
    from paper_2112_15071_amd import Simulator
    from paper_2112_15071_amd.batch import BatchSimulator

    log("[bench] 24-shot uneven batch, 1500 steps")
    shots = W.c3()
    cells_steps = sum(s.cells * s.nt for s in shots)
    sims = [Simulator(s.lam, s.mu, s.rho, s.h, s.dt, s.nt, sponge=s.sponge) for s in shots]
    batch = BatchSimulator(sims)
    tune = batch.autotune(steps=10)
    descs = [shot_desc(s) for s in shots]
    traces = [torch.empty((len(s.rec_pos), 3, s.nt), device="cuda") for s in shots]
    # plain per-shot loop (each shot with its own tuned kernel)
    for sim, d, tr in zip(sims, descs, traces):
        sim.forward(**d, traces=tr)
    sync()
    t0 = time.perf_counter()
    for sim, d, tr in zip(sims, descs, traces):
        sim.forward(**d, traces=tr)
    sync()
    t_loop = time.perf_counter() - t0
    batch.forward(descs, use_graph=True, traces=traces)  # capture + first replay
    sync()
    t0 = time.perf_counter()
    batch.forward(descs, use_graph=True, traces=traces)
    sync()
    t_graph = time.perf_counter() - t0
    log(f"[bench] batch: loop {t_loop:.3f} s, graph {t_graph:.3f} s (group budget {tune['group_mib']} MiB)")
    t_lock = t_graph
    if tune["group_mib"]:
        # the lockstep schedule with the same tile shapes, for comparison
        batch.set_schedule(0)
        batch.forward(descs, use_graph=True, traces=traces)
        sync()
        t0 = time.perf_counter()
        batch.forward(descs, use_graph=True, traces=traces)
        sync()
        t_lock = time.perf_counter() - t0
        log(f"[bench] batch lockstep: graph {t_lock:.3f} s")
    batch.close()
    for s in sims:
        s.close()
    return dict(loop_gcs=round(cells_steps / t_loop / 1e9, 3), batched_gcs=round(cells_steps / t_graph / 1e9, 3),
                loop_s=round(t_loop, 3), batched_s=round(t_graph, 3), speedup=round(t_loop / t_graph, 3),
                lockstep_gcs=round(cells_steps / t_lock / 1e9, 3), group_mib=tune["group_mib"],
                tile=[tune["tile_x"], tune["tile_y"]], tile2=[tune["tile2_x"], tune["tile2_y"]],
                workgroups=tune["workgroups"], cell_steps=cells_steps)


# Born (tangent-linear) forward, per cell and step, with the tile kernels: the background's
# and the perturbation's forward passes (120 each), plus what the source terms add to the
# background's passes: the velocity pass reads drho and the perturbation's velocity and
# writes it (7 values), the stress pass reads dlam, dmu and the perturbation's stress and
# writes it (14 values)
BORN_BYTES_PER_CELL_STEP = 120 + 120 + 4 * (1 + 2 * 3) + 4 * (2 + 2 * 6)


def bench_born(K=300):
    """Born forward on the 256^3 workload's model with a smooth 2 % perturbation of lam,
    mu and rho, K steps (after a warm-up run of the same length)."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2112_15071_amd import Simulator

    dev = torch.device("cuda:0")
    shot = W.c1(nt=K)
    nx, ny, nz = shot.shape
    model = [torch.as_tensor(a, dtype=torch.float32, device=dev) for a in (shot.lam, shot.mu, shot.rho)]
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    blob = np.exp(-((x - nx / 2) ** 2 + (y - ny / 2) ** 2 + (z - nz / 2) ** 2) / (2 * 20.0 ** 2))
    dm = [m * torch.as_tensor(0.02 * blob, dtype=torch.float32, device=dev) for m in model]
    sim = Simulator(*model, shot.h, shot.dt, K, sponge=shot.sponge, device=dev)
    sim.autotune(steps=10)
    args = dict(src_pos=shot.src_pos, moment=shot.moment, force=shot.force, wavelet=shot.wavelet[:K],
                rec_pos=shot.rec_pos)
    sim.born(*dm, **args)
    sync()
    t0 = time.perf_counter()
    sim.born(*dm, **args)
    sync()
    el = time.perf_counter() - t0
    cells = nx * ny * nz
    gbs = BORN_BYTES_PER_CELL_STEP * cells * K / el / 1e9
    log(f"[bench] born: {K} steps in {el:.3f} s -> {cells * K / el / 1e9:.2f} Gcell-steps/s, {gbs:.0f} GB/s")
    kern = sim.kernel()
    sim.close()
    return dict(gcs=round(cells * K / el / 1e9, 3), ms_per_step=round(el / K * 1e3, 4), steps=K, kernel=kern,
                bytes_per_cell_step=BORN_BYTES_PER_CELL_STEP, hbm_gbs=round(gbs, 1))


# The paper's levels of detail (Table 5): grid (nx, ny, nz), cell size (km per axis), dt (s),
# time steps of the full simulation.
TABLE5 = [
    ((64, 64, 32), (6.67, 10.61, 3.75), 0.1, 1700),
    ((64, 64, 64), (6.67, 10.61, 1.87), 0.1, 1700),
    ((128, 64, 64), (3.33, 10.61, 1.87), 0.1, 1700),
    ((128, 128, 64), (3.33, 5.30, 1.87), 0.1, 1700),
    ((128, 128, 128), (3.33, 5.30, 0.93), 0.05, 3400),
    ((256, 128, 128), (1.66, 5.30, 0.93), 0.05, 3400),
    ((256, 256, 128), (1.66, 2.65, 0.93), 0.05, 3400),
    ((256, 256, 256), (1.66, 2.65, 0.46), 0.01, 17000),
    ((512, 256, 256), (0.83, 2.65, 0.46), 0.01, 17000),
    ((512, 512, 256), (0.83, 1.32, 0.46), 0.01, 17000),
    ((512, 512, 512), (0.83, 1.32, 0.23), 0.01, 17000),
]


# The paper's layered medium (its table of medium parameters, case-study section): depth
# of each layer's top below the surface in km, vp and vs in km/s, density in g/cm^3.
MEDIUM_LAYERS = [(0.0, 4.90, 2.816, 2.50), (3.0, 5.40, 3.103, 2.60), (5.0, 6.00, 3.448, 2.70),
                 (7.0, 6.90, 3.966, 2.80), (20.0, 7.60, 4.368, 3.10), (26.0, 7.80, 4.483, 3.26),
                 (34.0, 8.00, 4.598, 3.30)]
LEVEL_BOX_KM = (427.03, 679.36, 120.0)  # the simulated box; its top 30 km lie above the surface
LEVEL_AIR_KM = 30.0
RHO_VACUUM = 100.0  # kg/m^3 above the surface, with lam = mu = 0


def level_medium(mshape):
    """The layered medium on a coarse node grid spanning the box (solid values continued
    up into the air, which each level then replaces by vacuum): lam, mu, rho [nz, ny, nx]."""
    import numpy as np

    mx, my, mz = mshape
    depth = np.linspace(0.0, LEVEL_BOX_KM[2], mz) - LEVEL_AIR_KM
    vp, vs, rho = (np.empty(mz) for _ in range(3))
    for top, a, b, r in MEDIUM_LAYERS:
        sel = depth >= top if top > 0.0 else np.ones(mz, dtype=bool)
        vp[sel], vs[sel], rho[sel] = a * 1e3, b * 1e3, r * 1e3
    mu = rho * vs * vs
    lam = rho * vp * vp - 2.0 * mu
    return [np.broadcast_to(a[:, None, None], (mz, my, mx)).copy() for a in (lam, mu, rho)]


def bench_levels(K=100):
    """The Table 5 level sweep on the paper's case-study medium: its seven crustal layers
    given on a coarse 64 x 64 x 128 node grid over the 427 x 679 x 120 km box are upsampled
    on the GPU to every level's grid, and the top 30 km (the air above the surface) are set
    to vacuum with the vacuum free surface below them.  Each level runs with its own
    anisotropic cells and dt (explosion at 10 km depth, 16 receivers one plane below the
    surface, 10-cell sponge on the other faces), K timed steps after autotuning: the single-shot forward (one
    launch per pass) and the same steps replayed from a hipGraph (a one-shot batch whose one
    group uses the shot's own tuned kernel), which removes the host launch cost on the small
    levels."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2112_15071_amd import Simulator, upsample
    from paper_2112_15071_amd.batch import BatchSimulator

    dev = torch.device("cuda:0")
    coarse = [torch.as_tensor(a, dtype=torch.float32, device=dev) for a in level_medium((64, 64, 128))]
    out = []
    for lev, (shape, dp, dt, nt_full) in enumerate(TABLE5):
        nx, ny, nz = shape
        lam, mu, rho = (upsample(c, shape) for c in coarse)
        ks = int(round(LEVEL_AIR_KM / dp[2]))  # first solid plane
        lam[:ks] = 0.0
        mu[:ks] = 0.0
        rho[:ks] = RHO_VACUUM
        h = tuple(v * 1e3 for v in dp)
        # sponge on the side and bottom faces; the top face is the vacuum surface
        sim = Simulator(lam, mu, rho, h, dt, K, sponge=(10, 10, 10, 10, 0, 10), device=dev, vacuum_top=ks)
        sim.autotune(steps=5)
        src = (nx / 2, ny / 2, ks + 10.0 / dp[2])
        rec = W.receiver_grid(np.linspace(12, nx - 13, 4), np.linspace(12, ny - 13, 4), ks + 1.0)
        wav = torch.as_tensor(W.ricker(0.05 if lev < 3 else 0.1, K, dt), dtype=torch.float32, device=dev)
        traces = torch.empty((len(rec), 3, K), dtype=torch.float32, device=dev)
        sim.forward(src, W.explosion(1e15), (0.0, 0.0, 0.0), wav, rec, traces=traces)
        sync()
        t0 = time.perf_counter()
        sim.forward(src, W.explosion(1e15), (0.0, 0.0, 0.0), wav, rec, traces=traces)
        sync()
        el = time.perf_counter() - t0
        batch = BatchSimulator([sim])
        batch.set_schedule(1 << 50)  # one group: the shot's own kernel shape
        desc = [dict(src_pos=src, moment=W.explosion(1e15), wavelet=wav, rec_pos=rec)]
        batch.forward(desc, use_graph=True, traces=[traces])  # capture + first replay
        sync()
        t0 = time.perf_counter()
        batch.forward(desc, use_graph=True, traces=[traces])
        sync()
        el_g = time.perf_counter() - t0
        batch.close()
        cells = nx * ny * nz
        best = min(el, el_g)
        st = sim.state()
        finite = bool(torch.isfinite(st).all()) and bool(torch.isfinite(traces).all()) and float(st.abs().max()) > 0.0
        del st
        row = dict(level=lev, grid=list(shape), cell_m=list(h), dt=dt, vacuum_planes=ks, state_finite=finite,
                   steps_timed=K,
                   gcs=round(cells * K / el / 1e9, 3), gcs_graph=round(cells * K / el_g / 1e9, 3),
                   ms_per_step=round(best / K * 1e3, 4), full_run_s=round(best / K * nt_full, 2), kernel=sim.kernel())
        log(f"[bench] level {lev} {shape}: {row['gcs']} Gcell-steps/s ({row['gcs_graph']} from a graph), "
            f"{row['ms_per_step']} ms/step, {nt_full} steps in {row['full_run_s']} s, state finite and nonzero: {finite}")
        out.append(row)
        sim.close()
        del lam, mu, rho
    return out


def bench_gradient(wave=4, nshots=8):
    import numpy as np
    import torch

    import workloads as W
    from paper_2112_15071_amd import Simulator
    from paper_2112_15071_amd.batch import BatchSimulator

    log(f"[bench] FWI gradient: {nshots} shots, 256^3, 1500 steps, checkpoints every 50")
    (tl, tm, tr_), start = W.c4_models()
    dev = torch.device("cuda:0")
    true = [torch.as_tensor(a, dtype=torch.float32, device=dev) for a in (tl, tm, tr_)]
    model = [torch.as_tensor(a, dtype=torch.float32, device=dev) for a in start]
    shots = W.c4_shots(*start)[:nshots]
    k = 50
    # observed data from the true model
    obs_sim = Simulator(*true, 10.0, 5e-4, 1500, sponge=20, device=dev)
    obs_sim.autotune(steps=10)
    d_obs = [obs_sim.forward(**shot_desc(s)).clone() for s in shots]
    sync()
    obs_sim.close()
    del true
    # per-shot loop through one gradient workspace
    sim = Simulator(*model, 10.0, 5e-4, 1500, sponge=20, device=dev)
    sim.autotune(steps=10)
    # the gradient's own kernel choice (its adjoint passes can rank tile shapes unlike the forward)
    gt = sim.autotune_gradient(shot_desc(shots[0]))
    log(f"[bench] gradient kernel {sim.kernel()} (tried {gt['tried']})")
    gws = sim.grad_workspace(k)
    g_loop = [torch.zeros_like(model[0]) for _ in range(3)]
    sync()
    t0 = time.perf_counter()
    J_loop = 0.0
    for s, o in zip(shots, d_obs):
        _, j = sim.gradient(gws, o, *g_loop, **shot_desc(s))
        J_loop = J_loop + j
    sync()
    t_loop = time.perf_counter() - t0
    kern = sim.kernel()
    sim.close()
    del gws
    torch.cuda.empty_cache()
    log(f"[bench] gradient loop {t_loop:.2f} s")
    # batched waves sharing the model and the gradient arrays
    wave = min(wave, len(shots))
    sims = [Simulator(*model, 10.0, 5e-4, 1500, sponge=20, device=dev) for _ in range(wave)]
    for x in sims:
        x.set_kernel(kern["variant"], kern["tile_y"], kern["zchunk"], kern["tile_x"])
    batch = BatchSimulator(sims)
    bt = batch.autotune_gradient([shot_desc(s) for s in shots[:wave]])
    log(f"[bench] batched gradient tile {bt['tile']}, z chunk {bt['zchunk']} (tried {bt['tried']})")
    gws_b = [x.grad_workspace(k) for x in sims]
    g_b = [torch.zeros_like(model[0]) for _ in range(3)]
    sync()
    t0 = time.perf_counter()
    J_b = 0.0
    for w0 in range(0, len(shots), wave):
        grp = shots[w0:w0 + wave]
        _, J = batch.gradient([shot_desc(s) for s in grp], d_obs[w0:w0 + wave], *g_b, ckpt_every=k, gws=gws_b)
        J_b = J_b + J.sum()
    sync()
    t_b = time.perf_counter() - t0
    log(f"[bench] gradient batched {t_b:.2f} s")
    diff = max(float((a - b).abs().max() / b.abs().max()) for a, b in zip(g_b, g_loop))
    batch.close()
    for x in sims:
        x.close()
    del gws_b
    torch.cuda.empty_cache()
    n = len(shots)
    return dict(loop_shots_per_s=round(n / t_loop, 4), batched_shots_per_s=round(n / t_b, 4),
                loop_s=round(t_loop, 2), batched_s=round(t_b, 2), speedup=round(t_loop / t_b, 3), wave=wave,
                loop_kernel=kern, batch_tile=bt["tile"], batch_zchunk=bt["zchunk"],
                misfit=float(J_loop), max_rel_diff_batched_vs_loop=diff,
                bytes_per_cell_step_per_shot=GRAD_BYTES_PER_CELL_STEP)


def counters_run(kernels, K):
    """Forward steps on the 256^3 workload with each kernel configuration in turn, then
    three copies of 1 GiB with torch (a plain copy kernel of known size, which calibrates
    the HBM byte counters).  Meant to run under rocprofv3 --pmc."""
    import torch

    import workloads as W
    from paper_2112_15071_amd import Simulator

    dev = torch.device("cuda:0")
    shot = W.c1(nt=K)
    lam, mu, rho = (torch.as_tensor(a, dtype=torch.float32).to(dev) for a in (shot.lam, shot.mu, shot.rho))
    wav = torch.as_tensor(shot.wavelet, dtype=torch.float32).to(dev)
    for spec in kernels:
        variant, tx, ty, zc = spec.split(",")
        sim = Simulator(lam, mu, rho, shot.h, shot.dt, K, dtype=torch.float32, sponge=shot.sponge, device=dev)
        sim.set_kernel(variant, int(ty), int(zc), int(tx))
        log(f"[counters] {spec}: {K} steps")
        sim.forward(shot.src_pos, shot.moment, shot.force, wav[:K], shot.rec_pos)
        sync()
        sim.close()
    a = torch.ones(1 << 28, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    sync()
    log("[counters] 3 x 1 GiB copies done")


def cpu_baseline(shot, ns):
    import oracle

    oracle.build(force=False)
    cfg = oracle.Config(shot.shape, shot.h, shot.dt, ns, sponge=shot.sponge)
    src = oracle.Source(shot.src_pos, moment=shot.moment, force=shot.force)
    log(f"[bench] oracle baseline: {ns} steps at full size on {oracle.get_threads()} threads")
    t0 = time.perf_counter()
    oracle.forward(cfg, shot.lam, shot.mu, shot.rho, src, shot.wavelet[:ns], shot.rec_pos)
    dt = time.perf_counter() - t0
    cells = int(shot.cells)
    # the same oracle on one core, over fewer steps (the cost per step is constant)
    threads = oracle.get_threads()
    ns1 = max(1, ns // 8)
    oracle.set_threads(1)
    try:
        log(f"[bench] oracle baseline: {ns1} steps at full size on 1 thread")
        t1 = time.perf_counter()
        cfg1 = oracle.Config(shot.shape, shot.h, shot.dt, ns1, sponge=shot.sponge)
        oracle.forward(cfg1, shot.lam, shot.mu, shot.rho, src, shot.wavelet[:ns1], shot.rec_pos)
        dt1 = time.perf_counter() - t1
    finally:
        oracle.set_threads(threads)
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), cpu)
    except OSError:
        pass
    return {"value": round(cells * ns / dt / 1e9, 5), "unit": "Gcell-steps/s", "cores": oracle.get_threads(),
            "kind": "oracle", "cpu": cpu,
            "sample": f"FP64 oracle on the 256^3 workload at full size, first {ns} of 2000 steps ({dt:.1f} s)",
            "one_core": {"value": round(cells * ns1 / dt1 / 1e9, 5), "steps": ns1, "seconds": round(dt1, 2)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--cpu-steps", type=int, default=24, help="oracle steps for the CPU baseline sample (0: skip)")
    ap.add_argument("--no-c2", action="store_true", help="skip the 512x512x256 free-surface section")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--no-levels", action="store_true", help="skip the Table 5 level sweep")
    ap.add_argument("--no-born", action="store_true", help="skip the Born (tangent-linear) section")
    ap.add_argument("--kernel", metavar="VARIANT,TX,TY,ZC", default=None,
                    help="forward kernel configuration (default: autotuned, cached per grid)")
    ap.add_argument("--grad-shots", type=int, default=8, help="shots of the gradient section (profiling runs: fewer)")
    ap.add_argument("--counters", metavar="VARIANT,TX,TY,ZC", action="append", default=[],
                    help="counter-collection run: --steps forward steps per kernel given (repeatable), then a "
                         "1 GiB device copy that calibrates FETCH_SIZE / WRITE_SIZE; prints no JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU path is not built.",
              file=sys.stderr)
        sys.exit(2)

    if args.counters:
        counters_run(args.counters, args.steps)
        return
    shot, f = bench_forward(args.steps, args.warmup, args.kernel)
    copy_gbs = stream_copy_ceiling()
    c2 = None if args.no_c2 else bench_c2()
    batch = None if args.no_batch else bench_batch()
    grad = None if args.no_grad else bench_gradient(nshots=args.grad_shots)
    levels = None if args.no_levels else bench_levels()
    born = None if args.no_born else bench_born()
    cpu = cpu_baseline(shot, args.cpu_steps) if args.cpu_steps > 0 else None
    nx, ny, nz = shot.shape
    out = {
        "metric": "FD Gcell-steps/s (forward, 256^3, FP32)",
        "value": round(f["gcs"], 3),
        "unit": "Gcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f["elapsed"] / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "256^3 six-layer + 5% Gaussian-correlated perturbation, h 10 m, dt 0.5 ms, random MT "
                        "source, 12 Hz Ricker, 256 receivers, 20-cell Cerjan sponge, O(2,4) velocity-stress",
            "grid": [nx, ny, nz],
            "cells": int(shot.cells),
            "time_steps": args.steps,
            "kernel": f["kernel"],
            "hbm_gbs_whole_step": round(f["both"], 1),
            "hbm_frac_whole_step": round(f["both"] / HBM_PEAK_GBS, 4),
            "bytes_per_cell_step": step_bytes(f["kernel"]),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": f["dom"],
            "achieved": round(f["achieved"], 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(f["achieved"] / HBM_PEAK_GBS, 4),
            "traffic": f["traffic"],
            "avg_kernel_ms": {k: round(v, 5) for k, v in f["per"].items()},
            "bytes_per_launch": f["bytes_launch"],
        },
        "stream_copy_gbs": copy_gbs,
        "c2_forward": c2,
        "batched_forward": batch,
        "gradient": grad,
        "levels": levels,
        "born": born,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
