"""Benchmark of the elastic FD hot path on one MI355X.

Headline (``value``): forward throughput in Gcell-steps/s on the 256^3 six-layer +
5 % Gaussian-perturbed model (h 10 m, dt 0.5 ms, random moment-tensor source, 12 Hz
Ricker, 256 receivers, 20-cell sponge, FP32), over exactly ``--steps`` time steps, the
median of five timed runs.  A "step" is one time step of the whole forward path: the
velocity pass (force source, damping), then the stress pass (moment source, damping)
whose launch also samples the receivers.  Each timed run starts from a zero state that
is set before the clock starts.

Also reported (same JSON line; a section that fails records {"error": ...} and the line
is still printed):
  c1_full  -- the same workload over its full 2000 steps (median of 3);
  roofline -- the dominant forward kernel's algorithmic bytes / its HIP-event duration,
              both passes separately, and the whole step;
  c2_forward -- the 512x512x256 free-surface workload over 1000 of its 4000 steps
              (median of 3; the cost per step does not depend on the step);
  stream_copy_gbs -- a plain 1 GiB device copy (read + write GB/s);
  batched_forward -- the 24-shot uneven batch (128^3 .. 256x256x128, 1500 steps):
              per-shot loop vs cache-blocked groups replayed from a hipGraph (median of 3
              each), and the lockstep schedule once;
  gradient -- the 8-shot 256^3 FWI gradient (1500 steps, checkpoints every 50): per-shot
              loop vs batched waves (shots/s, with the median per-shot and per-wave
              times), each with the kernel configuration its gradient tuner picks, and
              the fraction of the HBM roofline at the bytes the kernels move;
  levels   -- the paper's Table 5 level sweep (64x64x32 .. 512^3, anisotropic cells) on
              its case-study medium (seven layers under 30 km of air: vacuum surface),
              upsampled from one coarse grid to every level, 100 timed steps per level;
  born     -- the tangent-linear (Born) forward on the 256^3 model, 300 steps;
  coarse_medium -- a medium given on a 64^3 node grid over the 256^3 box: upsampled once
              to the nodes (set-up reading) vs sampled inside the step kernels at every
              value's own position (in-kernel reading), 300 steps each;
  paper_table6 -- the paper's own GLSL and CPU totals per level, with their hardware
              (context only, not a target);
  cpu_baseline -- the FP64 oracle on a bounded sample on this host's cores (and, as
              one_core, on a single core over an eighth of the steps).

    python bench.py [--steps 20] [--warmup 5] [--gpus 1] [--no-c2] [--no-batch] [--no-grad]
                    [--no-levels] [--no-born] [--no-coarse] [--cpu-steps 24]
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time
import traceback

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
# (120: its velocity pass writes v^{n+1/2} into the segment slot instead of over the
# state), the adjoint passes: stress-M 36 fields (the adjoint stress update of the step
# after and stress-A of this step: A_s, Y, stored v, lambda, mu and 5 accumulators read;
# A_s, X and the accumulators written), velocity-A 22 (X, Y, v^{n+1/2}, rho and g_b read,
# Y and g_b written): 232
GRAD_BYTES_PER_CELL_STEP = 120 + 120 + 4 * (36 + 22)
# the design figure with eight staggered-point accumulators and no hand-over fields
# between the adjoint passes (forward 120 + recompute 120 + adjoint 232)
GRAD_BYTES_DESIGN = 120 + 120 + 232
# the same adjoint with a recompute that also stores sigma^n (156: the form whose buoyancy
# gradient reads D_S sigma^n), the usual figure for a checkpointed elastic adjoint
GRAD_BYTES_SIGMA_STORED = 120 + 156 + 232
# measured counter calibration (plain 1 GiB copy): FETCH_SIZE reads 0.5x, WRITE_SIZE 1.0x
FETCH_FACTOR, WRITE_FACTOR = 2.0, 1.0

# The paper's Table 6: total time of one simulation per level of detail, its GLSL shaders
# on the Vega iGPU of a Ryzen 7 4700U notebook (24 GB DDR4) against its NumPy/OpenBLAS
# CPU implementation on the same notebook; grids and step counts from its Table 5.
# (level, (nx, ny, nz), steps, CPU seconds, GPU seconds)
PAPER_TABLE6 = [
    (0, (64, 64, 32), 1700, 10, 3),
    (1, (64, 64, 64), 1700, 40, 4),
    (2, (128, 64, 64), 1700, 113, 7),
    (3, (128, 128, 64), 1700, 221, 18),
    (4, (128, 128, 128), 3400, 850, 122),
    (5, (256, 128, 128), 3400, 1666, 136),
    (6, (256, 256, 128), 3400, 3502, 295),
    (7, (256, 256, 256), 17000, 36210, 2890),
    (8, (512, 256, 256), 17000, 73950, 5100),
    (9, (512, 512, 256), 17000, 158270, 14450),
    (10, (512, 512, 512), 17000, 372470, 29750),
]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sync():
    import torch

    torch.cuda.synchronize()


def median_time(fn, reps, prep=None):
    """Median wall time of ``reps`` runs of fn (each bracketed by device syncs; ``prep``
    runs before each, outside the clock).  Returns (median s, list of s)."""
    ts = []
    for _ in range(reps):
        if prep is not None:
            prep()
        sync()
        t0 = time.perf_counter()
        fn()
        sync()
        ts.append(time.perf_counter() - t0)
    return statistics.median(ts), ts


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
        key = f"{kern['variant']},{kern['tile_x']},{kern['tile_y']},{kern['zchunk']},{kern['layout']}"
        return table["kernels"][key][dom]["hbm_bytes"]
    except (OSError, KeyError, ValueError):
        return None


class Forward:
    """The 256^3 workload on the GPU: model, simulator with its tuned kernel, zero state."""

    def __init__(self, nt_max, kernel=None, layout="auto"):
        import torch

        import workloads as W
        from paper_2112_15071_amd import Simulator

        self.dev = torch.device("cuda:0")
        self.shot = W.c1(nt=nt_max)
        nx, ny, nz = self.shot.shape
        self.cells = nx * ny * nz
        self.model = [torch.as_tensor(a, dtype=torch.float32).to(self.dev)
                      for a in (self.shot.lam, self.shot.mu, self.shot.rho)]
        self.wav = torch.as_tensor(self.shot.wavelet, dtype=torch.float32).to(self.dev)
        self.zero = torch.zeros((9, nz, ny, nx), dtype=torch.float32, device=self.dev)
        self.sims = {}
        self.kernel = kernel
        self.layout = layout
        self.Simulator = Simulator

    def sim(self, K):
        """Simulator of K steps with the tuned (or given) kernel configuration."""
        if K not in self.sims:
            s = self.Simulator(*self.model, self.shot.h, self.shot.dt, K, dtype=self.model[0].dtype,
                               sponge=self.shot.sponge, device=self.dev, layout=self.layout)
            if not self.sims:
                if self.kernel:
                    variant, tx, ty, zc = self.kernel.split(",")
                    s.set_kernel(variant, int(ty), int(zc), int(tx))
                    log(f"[bench] kernel {s.kernel()} (given)")
                else:
                    tune = s.autotune(steps=20)
                    log(f"[bench] kernel {s.kernel()} (autotune {'cached' if tune['cached'] else 'run'})")
                self.kernel_cfg = s.kernel()
            else:
                k = self.kernel_cfg
                s.set_kernel(k["variant"], k["tile_y"], k["zchunk"], k["tile_x"])
            self.sims[K] = s
        return self.sims[K]

    def run(self, K, traces, profile=False):
        sim = self.sim(K)
        sh = self.shot
        sim.forward(sh.src_pos, sh.moment, sh.force, self.wav[:K], sh.rec_pos, keep_state=True, traces=traces)

    def timed(self, K, reps):
        import torch

        sim = self.sim(K)
        traces = torch.empty((self.shot.rec_pos.shape[0], 3, K), dtype=torch.float32, device=self.dev)
        self.run(K, traces)  # warm-up of this simulator
        return median_time(lambda: self.run(K, traces), reps, prep=lambda: sim.set_state(self.zero))

    def close(self):
        for s in self.sims.values():
            s.close()
        self.sims = {}


def bench_forward(fw, K, Wm, reps=5):
    """Headline: K steps, median of reps runs (after Wm warm-up steps), then the same K
    steps once more with per-kernel HIP events on the launch stream."""
    import torch

    from paper_2112_15071_amd import _abi

    log(f"[bench] 256^3 workload: steps {K}, warmup {Wm}")
    sim = fw.sim(K)
    if Wm > 0:
        warm = fw.sim(Wm)
        tr = torch.empty((fw.shot.rec_pos.shape[0], 3, Wm), dtype=torch.float32, device=fw.dev)
        warm.set_state(fw.zero)
        fw.run(Wm, tr)
        sync()
    el, ts = fw.timed(K, reps)
    gcs = fw.cells * K / el / 1e9
    log(f"[bench] forward {K} steps: median {el * 1e3:.3f} ms of {[round(t * 1e3, 3) for t in ts]} "
        f"-> {gcs:.2f} Gcell-steps/s")
    traces = torch.empty((fw.shot.rec_pos.shape[0], 3, K), dtype=torch.float32, device=fw.dev)
    sim.set_state(fw.zero)
    _abi.fd3d_profile(sim.ctx, True)
    fw.run(K, traces)
    ms, launches = _abi.fd3d_profile_read(sim.ctx)
    sync()
    _abi.fd3d_profile(sim.ctx, False)
    names = ("velocity", "record", "stress", "fused")
    per = {names[i]: ms[i] / launches[i] for i in range(4) if launches[i] > 0}
    if "fused" in per:
        dom = "fused"
    else:
        dom = "stress" if per["stress"] >= per["velocity"] else "velocity"
    kern = dict(sim.kernel(), layout=sim.layout())
    per_kernel = {}
    for name, t in per.items():
        if name in BYTES_PER_CELL:
            gbs = BYTES_PER_CELL[name] * fw.cells / (t * 1e-3) / 1e9
            per_kernel[name] = dict(avg_ms=round(t, 5), achieved_gbs=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4))
    step_ms = sum(per[n] for n in per if n in BYTES_PER_CELL)
    events_gbs = step_bytes(kern) * fw.cells / (step_ms * 1e-3) / 1e9
    wall_gbs = step_bytes(kern) * fw.cells * K / (el * 1e9)
    log(f"[bench] avg kernel ms {per}; dominant {dom} {per_kernel[dom]['achieved_gbs']:.0f} GB/s; "
        f"whole step {events_gbs:.0f} GB/s (events), {wall_gbs:.0f} GB/s (wall)")
    return dict(gcs=gcs, elapsed=el, times=ts, per=per, per_kernel=per_kernel, dom=dom, kernel=kern,
                bytes_launch=BYTES_PER_CELL[dom] * fw.cells, events_gbs=events_gbs, wall_gbs=wall_gbs,
                traffic=measured_traffic(kern, dom))


def bench_c1_full(fw, K=2000, reps=3):
    """The 256^3 workload over its full 2000 steps."""
    el, ts = fw.timed(K, reps)
    gcs = fw.cells * K / el / 1e9
    gbs = step_bytes(fw.kernel_cfg) * fw.cells * K / el / 1e9
    log(f"[bench] forward {K} steps: median {el:.4f} s of {[round(t, 4) for t in ts]} -> {gcs:.2f} Gcell-steps/s, "
        f"{gbs:.0f} GB/s")
    fw.sims.pop(K).close()
    return dict(gcs=round(gcs, 3), steps=K, seconds=round(el, 4), seconds_all=[round(t, 4) for t in ts],
                hbm_gbs_whole_step=round(gbs, 1), hbm_frac_whole_step=round(gbs / HBM_PEAK_GBS, 4))


def bench_c2(K=4000, reps=3):
    """The 512 x 512 x 256 free-surface workload (30-cell sponge on five faces): K of its
    4000 steps (all of them by default), median of reps runs from a zero state."""
    import torch

    import workloads as W
    from paper_2112_15071_amd import Simulator

    dev = torch.device("cuda:0")
    log(f"[bench] 512x512x256 free-surface workload: {K} of 4000 steps")
    shot = W.c2(nt=K)
    lam, mu, rho = (torch.as_tensor(a, dtype=torch.float32).to(dev) for a in (shot.lam, shot.mu, shot.rho))
    wav = torch.as_tensor(shot.wavelet, dtype=torch.float32).to(dev)
    sim = Simulator(lam, mu, rho, shot.h, shot.dt, K, sponge=shot.sponge, free_surface=True, device=dev)
    sim.autotune(steps=10)
    traces = torch.empty((shot.rec_pos.shape[0], 3, K), dtype=torch.float32, device=dev)
    nx, ny, nz = shot.shape
    zero = torch.zeros((9, nz, ny, nx), dtype=torch.float32, device=dev)
    run = lambda: sim.forward(shot.src_pos, shot.moment, shot.force, wav, shot.rec_pos, keep_state=True,
                              traces=traces)
    sim.set_state(zero)
    run()  # warm-up
    el, ts = median_time(run, reps, prep=lambda: sim.set_state(zero))
    kern = dict(sim.kernel(), layout=sim.layout())
    sim.close()
    gcs = shot.cells * K / el / 1e9
    gbs = step_bytes(kern) * shot.cells * K / el / 1e9
    log(f"[bench] c2: median {el:.3f} s of {[round(t, 3) for t in ts]} -> {gcs:.2f} Gcell-steps/s, {gbs:.0f} GB/s")
    return dict(gcs=round(gcs, 3), steps=K, of_steps=4000, seconds=round(el, 4), seconds_all=[round(t, 4) for t in ts],
                kernel=kern, hbm_gbs_whole_step=round(gbs, 1), hbm_frac_whole_step=round(gbs / HBM_PEAK_GBS, 4))


def stream_copy_ceiling(reps=20):
    """Device-to-device copy of 1 GiB with torch, timed with HIP events on the current
    stream: read + write bytes per second (a plain stream's rate)."""
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


def bench_batch(reps=3):
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

    def loop():  # plain per-shot loop (each shot with its own tuned kernel)
        for sim, d, tr in zip(sims, descs, traces):
            sim.forward(**d, traces=tr)

    loop()
    t_loop, ts_loop = median_time(loop, reps)
    graph = lambda: batch.forward(descs, use_graph=True, traces=traces)
    graph()  # capture + first replay
    t_graph, ts_graph = median_time(graph, reps)
    log(f"[bench] batch: loop median {t_loop:.3f} s {[round(t, 3) for t in ts_loop]}, graph median {t_graph:.3f} s "
        f"{[round(t, 3) for t in ts_graph]} (group budget {tune['group_mib']} MiB)")
    t_lock = t_graph
    if tune["group_mib"]:
        # the lockstep schedule with the same tile shapes, for comparison
        batch.set_schedule(0)
        graph()
        t_lock, _ = median_time(graph, 1)
        log(f"[bench] batch lockstep: graph {t_lock:.3f} s")
    batch.close()
    for s in sims:
        s.close()
    return dict(loop_gcs=round(cells_steps / t_loop / 1e9, 3), batched_gcs=round(cells_steps / t_graph / 1e9, 3),
                loop_s=round(t_loop, 3), batched_s=round(t_graph, 3), speedup=round(t_loop / t_graph, 3),
                loop_s_all=[round(t, 3) for t in ts_loop], batched_s_all=[round(t, 3) for t in ts_graph],
                lockstep_gcs=round(cells_steps / t_lock / 1e9, 3), group_mib=tune["group_mib"],
                tile=[tune["tile_x"], tune["tile_y"]], tile2=[tune["tile2_x"], tune["tile2_y"]],
                workgroups=tune["workgroups"], cell_steps=cells_steps)


def bench_coarse_medium(K=300, reps=3, coarse=(64, 64, 64), shape=(256, 256, 256)):
    """The two readings of a coarse medium (Sec. 2.2.1) on the 256^3 grid: the six-layer +
    perturbed generator on a 64^3 node grid over the same box (40.5 m node spacing), with
    the 256^3 workload's source, receivers, spacing and dt.  A: sampled once at the
    simulation nodes (fd3d_upsample, outside the clock), then the step kernels take node
    means (120 B per cell-step); B: the step kernels read the coarse arrays themselves,
    trilinear samples at every value's own position (108 B per cell-step: no model arrays
    streamed, the coarse ones stay cached).  K steps from a zero state, median of reps."""
    import torch

    import workloads as W
    from paper_2112_15071_amd import Simulator, upsample

    dev = torch.device("cuda:0")
    nx, ny, nz = shape
    mx, my, mz = coarse
    shot = W.c1(nt=K)
    hc = 10.0 * (nx - 1) / (mx - 1)
    model_c = [torch.as_tensor(a, dtype=torch.float32, device=dev) for a in W.layered_perturbed(coarse, hc, 1001)]
    model_n = [upsample(a, shape) for a in model_c]
    wav = torch.as_tensor(shot.wavelet[:K], dtype=torch.float32, device=dev)
    zero = torch.zeros((9, nz, ny, nx), dtype=torch.float32, device=dev)
    traces = torch.empty((len(shot.rec_pos), 3, K), dtype=torch.float32, device=dev)
    out = {}
    for name, model, grid in (("setup_upsample", model_n, None), ("in_kernel", model_c, shape)):
        sim = Simulator(*model, shot.h, shot.dt, K, sponge=shot.sponge, device=dev, grid=grid)
        sim.autotune(steps=10)
        run = lambda: sim.forward(shot.src_pos, shot.moment, shot.force, wav, shot.rec_pos, keep_state=True,
                                  traces=traces)
        sim.set_state(zero)
        run()
        el, ts = median_time(run, reps, prep=lambda: sim.set_state(zero))
        gcs = nx * ny * nz * K / el / 1e9
        b = 120 if grid is None else 108
        out[name] = dict(gcs=round(gcs, 3), ms_per_step=round(el / K * 1e3, 4), kernel=sim.kernel(),
                         bytes_per_cell_step=b, hbm_gbs=round(b * nx * ny * nz * K / el / 1e9, 1))
        log(f"[bench] coarse medium {name}: {gcs:.2f} Gcell-steps/s ({el / K * 1e3:.4f} ms/step), {sim.kernel()}")
        sim.close()
    out["speedup_in_kernel"] = round(out["in_kernel"]["gcs"] / out["setup_upsample"]["gcs"], 4)
    out["coarse_nodes"] = list(coarse)
    out["grid"] = list(shape)
    out["steps"] = K
    return out


def bench_layout_ab(K=300, reps=3):
    """The 256^3 workload with each field storage (fd3d_opts.layout): separate arrays and
    interleaved rows, each with its own tuned kernel; K steps from a zero state, median of
    reps.  The results are bitwise equal (tested); only the time differs."""
    import torch

    import workloads as W
    from paper_2112_15071_amd import Simulator

    dev = torch.device("cuda:0")
    shot = W.c1(nt=K)
    nx, ny, nz = shot.shape
    model = [torch.as_tensor(a, dtype=torch.float32, device=dev) for a in (shot.lam, shot.mu, shot.rho)]
    wav = torch.as_tensor(shot.wavelet[:K], dtype=torch.float32, device=dev)
    zero = torch.zeros((9, nz, ny, nx), dtype=torch.float32, device=dev)
    traces = torch.empty((len(shot.rec_pos), 3, K), dtype=torch.float32, device=dev)
    out = {}
    for lay in ("separate", "rows"):
        sim = Simulator(*model, shot.h, shot.dt, K, sponge=shot.sponge, device=dev, layout=lay)
        sim.autotune(steps=20)
        run = lambda: sim.forward(shot.src_pos, shot.moment, shot.force, wav, shot.rec_pos, keep_state=True,
                                  traces=traces)
        sim.set_state(zero)
        run()
        el, ts = median_time(run, reps, prep=lambda: sim.set_state(zero))
        gcs = nx * ny * nz * K / el / 1e9
        out[lay] = dict(gcs=round(gcs, 3), ms_per_step=round(el / K * 1e3, 4), kernel=sim.kernel(),
                        hbm_gbs=round(120 * nx * ny * nz * K / el / 1e9, 1))
        log(f"[bench] layout {lay}: {gcs:.2f} Gcell-steps/s ({el / K * 1e3:.4f} ms/step), {sim.kernel()}")
        sim.close()
    out["speedup_rows"] = round(out["rows"]["gcs"] / out["separate"]["gcs"], 4)
    out["steps"] = K
    return out


# Born (tangent-linear) forward, per cell and step, with the tile kernels: one velocity
# sweep and one stress sweep step the background (the forward's 120) and the perturbation
# together; the velocity sweep adds drho, the perturbation's stress read and its velocity
# read and written (13 values), the stress sweep dlam, dmu, the perturbation's velocity
# read and its stress read and written (17 values)
BORN_BYTES_PER_CELL_STEP = 120 + 4 * (1 + 6 + 2 * 3) + 4 * (2 + 3 + 2 * 6)


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
    el, ts = median_time(lambda: sim.born(*dm, **args), 3)
    cells = nx * ny * nz
    gbs = BORN_BYTES_PER_CELL_STEP * cells * K / el / 1e9
    log(f"[bench] born: {K} steps, median {el:.3f} s -> {cells * K / el / 1e9:.2f} Gcell-steps/s, {gbs:.0f} GB/s")
    kern = sim.kernel()
    sim.close()
    return dict(gcs=round(cells * K / el / 1e9, 3), ms_per_step=round(el / K * 1e3, 4), steps=K, kernel=kern,
                bytes_per_cell_step=BORN_BYTES_PER_CELL_STEP, hbm_gbs=round(gbs, 1),
                hbm_frac=round(gbs / HBM_PEAK_GBS, 4))


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
        run = lambda: sim.forward(src, W.explosion(1e15), (0.0, 0.0, 0.0), wav, rec, traces=traces)
        run()
        el, _ = median_time(run, 3)
        batch = BatchSimulator([sim])
        batch.set_schedule(1 << 50)  # one group: the shot's own kernel shape
        desc = [dict(src_pos=src, moment=W.explosion(1e15), wavelet=wav, rec_pos=rec)]
        graph = lambda: batch.forward(desc, use_graph=True, traces=[traces])
        graph()  # capture + first replay
        el_g, _ = median_time(graph, 3)
        batch.close()
        cells = nx * ny * nz
        best = min(el, el_g)
        st = sim.state()
        finite = bool(torch.isfinite(st).all()) and bool(torch.isfinite(traces).all()) and float(st.abs().max()) > 0.0
        del st
        p = PAPER_TABLE6[lev]
        row = dict(level=lev, grid=list(shape), cell_m=list(h), dt=dt, vacuum_planes=ks, state_finite=finite,
                   steps_timed=K,
                   gcs=round(cells * K / el / 1e9, 3), gcs_graph=round(cells * K / el_g / 1e9, 3),
                   ms_per_step=round(best / K * 1e3, 4), full_run_s=round(best / K * nt_full, 2),
                   paper_gpu_s=p[4], paper_cpu_s=p[3], kernel=sim.kernel())
        log(f"[bench] level {lev} {shape}: {row['gcs']} Gcell-steps/s ({row['gcs_graph']} from a graph), "
            f"{row['ms_per_step']} ms/step, {nt_full} steps in {row['full_run_s']} s (paper GLSL {p[4]} s), "
            f"state finite and nonzero: {finite}")
        out.append(row)
        sim.close()
        del lam, mu, rho
    return out


def bench_gradient(wave=None, nshots=8):
    import torch

    import workloads as W
    from paper_2112_15071_amd import Simulator
    from paper_2112_15071_amd.batch import BatchSimulator

    nt, k = 1500, 50
    log(f"[bench] FWI gradient: {nshots} shots, 256^3, {nt} steps, checkpoints every {k}")
    (tl, tm, tr_), start = W.c4_models()
    dev = torch.device("cuda:0")
    true = [torch.as_tensor(a, dtype=torch.float32, device=dev) for a in (tl, tm, tr_)]
    model = [torch.as_tensor(a, dtype=torch.float32, device=dev) for a in start]
    shots = W.c4_shots(*start)[:nshots]
    cells = int(model[0].numel())
    # observed data from the true model
    obs_sim = Simulator(*true, 10.0, 5e-4, nt, sponge=20, device=dev)
    obs_sim.autotune(steps=10)
    d_obs = [obs_sim.forward(**shot_desc(s)).clone() for s in shots]
    sync()
    obs_sim.close()
    del true
    # per-shot loop through one gradient workspace
    sim = Simulator(*model, 10.0, 5e-4, nt, sponge=20, device=dev)
    sim.autotune(steps=10)
    # the gradient's own kernel choice (its adjoint passes can rank tile shapes unlike the forward)
    gt = sim.autotune_gradient(shot_desc(shots[0]))
    log(f"[bench] gradient kernel {sim.kernel()} (tried {gt['tried']})")
    gws = sim.grad_workspace(k)
    g_loop = [torch.zeros_like(model[0]) for _ in range(3)]
    sync()
    per_shot = []
    J_loop = 0.0
    t0 = time.perf_counter()
    for s, o in zip(shots, d_obs):
        t1 = time.perf_counter()
        _, j = sim.gradient(gws, o, *g_loop, **shot_desc(s))
        sync()
        per_shot.append(time.perf_counter() - t1)
        J_loop = J_loop + j
    t_loop = time.perf_counter() - t0
    kern = sim.kernel()
    per_shot_bytes = gws.numel() + sim.workspace.numel()
    sim.close()
    del gws
    torch.cuda.empty_cache()
    log(f"[bench] gradient loop {t_loop:.2f} s, per shot median {statistics.median(per_shot):.3f} s")
    # batched waves sharing the model and the gradient arrays: as many shots per wave as
    # fit in 95 % of the free device memory (a shot: its gradient and forward workspaces)
    if wave is None:
        wave = max(1, int(0.95 * torch.cuda.mem_get_info()[0]) // per_shot_bytes)
        log(f"[bench] batched gradient wave: {wave} shots ({per_shot_bytes / 2**30:.1f} GiB each)")
    wave = min(wave, len(shots))
    sims = [Simulator(*model, 10.0, 5e-4, nt, sponge=20, device=dev) for _ in range(wave)]
    for x in sims:
        x.set_kernel(kern["variant"], kern["tile_y"], kern["zchunk"], kern["tile_x"])
    batch = BatchSimulator(sims)
    bt = batch.autotune_gradient([shot_desc(s) for s in shots[:wave]])
    log(f"[bench] batched gradient tile {bt['tile']}, z chunk {bt['zchunk']} (tried {bt['tried']})")
    gws_b = [x.grad_workspace(k) for x in sims]
    g_b = [torch.zeros_like(model[0]) for _ in range(3)]
    sync()
    per_wave = []
    J_b = 0.0
    t0 = time.perf_counter()
    for w0 in range(0, len(shots), wave):
        grp = shots[w0:w0 + wave]
        t1 = time.perf_counter()
        _, J = batch.gradient([shot_desc(s) for s in grp], d_obs[w0:w0 + wave], *g_b, ckpt_every=k, gws=gws_b)
        sync()
        per_wave.append((time.perf_counter() - t1) / len(grp))
        J_b = J_b + J.sum()
    t_b = time.perf_counter() - t0
    log(f"[bench] gradient batched {t_b:.2f} s, per shot by wave {[round(t, 3) for t in per_wave]}")
    diff = max(float((a - b).abs().max() / b.abs().max()) for a, b in zip(g_b, g_loop))
    batch.close()
    for x in sims:
        x.close()
    del gws_b
    torch.cuda.empty_cache()
    n = len(shots)
    bytes_shot = GRAD_BYTES_PER_CELL_STEP * cells * nt
    design_shot = GRAD_BYTES_DESIGN * cells * nt
    frac = lambda sps, b: round(sps * b / 1e9 / HBM_PEAK_GBS, 4)
    loop_sps, b_sps = n / t_loop, n / t_b
    return dict(loop_shots_per_s=round(loop_sps, 4), batched_shots_per_s=round(b_sps, 4),
                loop_s=round(t_loop, 2), batched_s=round(t_b, 2), speedup=round(t_loop / t_b, 3), wave=wave,
                loop_s_per_shot_median=round(statistics.median(per_shot), 4),
                loop_s_per_shot=[round(t, 4) for t in per_shot],
                batched_s_per_shot_by_wave=[round(t, 4) for t in per_wave],
                loop_kernel=kern, batch_tile=bt["tile"], batch_zchunk=bt["zchunk"],
                misfit=float(J_loop), max_rel_diff_batched_vs_loop=diff,
                bytes_per_cell_step_per_shot=GRAD_BYTES_PER_CELL_STEP,
                roofline={"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "batched_achieved": round(b_sps * bytes_shot / 1e9, 1),
                          "batched_frac": frac(b_sps, bytes_shot), "loop_frac": frac(loop_sps, bytes_shot),
                          "design_bytes_per_cell_step": GRAD_BYTES_DESIGN,
                          "batched_frac_at_design_bytes": frac(b_sps, design_shot),
                          "roofline_shots_per_s_at_design_bytes": round(HBM_PEAK_GBS * 1e9 / design_shot, 4),
                          "sigma_stored_bytes_per_cell_step": GRAD_BYTES_SIGMA_STORED,
                          "batched_frac_at_sigma_stored_bytes": frac(b_sps, GRAD_BYTES_SIGMA_STORED * cells * nt)})


def counters_run(kernels, K, grad=False):
    """Forward steps on the 256^3 workload with each kernel configuration in turn (with
    ``grad``, then a K-step checkpointed gradient with the first configuration), then
    three copies of 1 GiB with torch (a plain copy kernel of known size, which calibrates
    the HBM byte counters).  Meant to run under rocprofv3 --pmc."""
    import torch

    import workloads as W
    from paper_2112_15071_amd import Simulator

    dev = torch.device("cuda:0")
    shot = W.c1(nt=K)
    lam, mu, rho = (torch.as_tensor(a, dtype=torch.float32).to(dev) for a in (shot.lam, shot.mu, shot.rho))
    wav = torch.as_tensor(shot.wavelet, dtype=torch.float32).to(dev)
    def make(spec):
        variant, tx, ty, zc, *lay = spec.split(",")
        sim = Simulator(lam, mu, rho, shot.h, shot.dt, K, dtype=torch.float32, sponge=shot.sponge, device=dev,
                        layout=lay[0] if lay else "auto")
        sim.set_kernel(variant, int(ty), int(zc), int(tx))
        return sim

    for spec in kernels:
        sim = make(spec)
        log(f"[counters] {spec} ({sim.layout()}): {K} steps")
        sim.forward(shot.src_pos, shot.moment, shot.force, wav[:K], shot.rec_pos)
        sync()
        sim.close()
    if grad:
        # one checkpointed gradient of the first configuration: its recompute (the velocity
        # pass writing v^{n+1/2} into the segment slots, the stress pass) and the adjoint
        # passes
        sim = make(kernels[0])
        k = max(1, K // 2)
        gws = sim.grad_workspace(k)
        g = [torch.zeros_like(lam) for _ in range(3)]
        d_obs = torch.zeros((shot.rec_pos.shape[0], 3, K), dtype=torch.float32, device=dev)
        log(f"[counters] gradient {kernels[0]}: {K} steps, checkpoints every {k}")
        sim.gradient(gws, d_obs, *g, **shot_desc(shot))
        sync()
        sim.close()
    a = torch.ones(1 << 28, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    sync()
    log("[counters] 3 x 1 GiB copies done")


def cpu_baseline(shot, ns):
    """The FP64 oracle on the first ``ns`` steps of ``shot`` at full size (its own Ricker
    wavelet of ns samples with the shot's peak frequency, so the sample does not depend on
    how many steps the GPU leg ran), on every thread of this process, then on one thread
    over an eighth of the steps (the cost per step is constant)."""
    import oracle
    import workloads as W

    oracle.build(force=False)
    f0 = 12.0
    wav = W.ricker(f0, ns, shot.dt)
    cfg = oracle.Config(shot.shape, shot.h, shot.dt, ns, sponge=shot.sponge)
    src = oracle.Source(shot.src_pos, moment=shot.moment, force=shot.force)
    threads = oracle.get_threads()
    log(f"[bench] oracle baseline: {ns} steps at full size on {threads} threads")
    t0 = time.perf_counter()
    oracle.forward(cfg, shot.lam, shot.mu, shot.rho, src, wav, shot.rec_pos)
    dt = time.perf_counter() - t0
    cells = int(shot.cells)
    ns1 = max(1, ns // 8)
    oracle.set_threads(1)
    try:
        log(f"[bench] oracle baseline: {ns1} steps at full size on 1 thread")
        cfg1 = oracle.Config(shot.shape, shot.h, shot.dt, ns1, sponge=shot.sponge)
        t1 = time.perf_counter()
        oracle.forward(cfg1, shot.lam, shot.mu, shot.rho, src, wav[:ns1], shot.rec_pos)
        dt1 = time.perf_counter() - t1
    finally:
        oracle.set_threads(threads)
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), cpu)
    except OSError:
        pass
    nx, ny, nz = shot.shape
    return {"value": round(cells * ns / dt / 1e9, 5), "unit": "Gcell-steps/s", "cores": threads,
            "kind": "oracle", "cpu": cpu,
            "sample": f"FP64 oracle on the {nx}x{ny}x{nz} workload at full size, first {ns} steps ({dt:.1f} s)",
            "one_core": {"value": round(cells * ns1 / dt1 / 1e9, 5), "steps": ns1, "seconds": round(dt1, 2)}}


def paper_context():
    """The paper's Table 6 totals as Gcell-steps/s, with their hardware (context only)."""
    rows = []
    for lev, (nx, ny, nz), steps, cpu_s, gpu_s in PAPER_TABLE6:
        cs = nx * ny * nz * steps
        rows.append(dict(level=lev, grid=[nx, ny, nz], steps=steps, cpu_s=cpu_s, gpu_s=gpu_s,
                         gpu_gcs=round(cs / gpu_s / 1e9, 4), cpu_gcs=round(cs / cpu_s / 1e9, 4)))
    return {"source": "paper Table 6 (total time of one simulation per level of detail; grids and steps of Table 5)",
            "gpu": "GLSL 3.3 shaders on the Vega iGPU of an AMD Ryzen 7 4700U (HP ProBook 445 G7, 24 GB DDR4)",
            "cpu": "NumPy + OpenBLAS on the same Ryzen 7 4700U (about 30 % CPU utilisation)",
            "precision": "floating-point textures (taken as FP32)", "levels": rows}


def parse_args(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--cpu-steps", type=int, default=24, help="oracle steps for the CPU baseline sample (0: skip)")
    ap.add_argument("--no-c1-full", action="store_true", help="skip the 2000-step 256^3 run")
    ap.add_argument("--no-c2", action="store_true", help="skip the 512x512x256 free-surface section")
    ap.add_argument("--c2-steps", type=int, default=4000, help="timed steps of the 512x512x256 section (of 4000)")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--no-levels", action="store_true", help="skip the Table 5 level sweep")
    ap.add_argument("--no-born", action="store_true", help="skip the Born (tangent-linear) section")
    ap.add_argument("--no-coarse", action="store_true", help="skip the coarse-medium A/B section")
    ap.add_argument("--kernel", metavar="VARIANT,TX,TY,ZC", default=None,
                    help="forward kernel configuration (default: autotuned, cached per grid)")
    ap.add_argument("--grad-shots", type=int, default=8, help="shots of the gradient section (profiling runs: fewer)")
    ap.add_argument("--grad-wave", type=int, default=None,
                    help="shots per batched gradient wave (default: as many as fit in device memory)")
    ap.add_argument("--layout", choices=("auto", "separate", "rows"), default="auto",
                    help="field storage of the 256^3 forward sections (default: the library's choice)")
    ap.add_argument("--no-layout-ab", action="store_true", help="skip the separate-vs-rows A/B section")
    ap.add_argument("--counters", metavar="VARIANT,TX,TY,ZC[,LAYOUT]", action="append", default=[],
                    help="counter-collection run: --steps forward steps per kernel given (repeatable), then a "
                         "1 GiB device copy that calibrates FETCH_SIZE / WRITE_SIZE; prints no JSON")
    ap.add_argument("--counters-grad", action="store_true",
                    help="with --counters: also a --steps-step checkpointed gradient with the first configuration")
    return ap.parse_args(argv)


def run_sections(args, sections):
    """Run (name, fn) pairs in order; a section that raises records its error and the
    rest still run.  Returns ({name: result or None}, {name: error text})."""
    results, errors = {}, {}
    for name, fn in sections:
        try:
            results[name] = fn()
        except Exception as e:  # noqa: BLE001 - reported in the JSON line
            log(f"[bench] section {name} failed:\n{traceback.format_exc()}")
            results[name] = None
            errors[name] = f"{type(e).__name__}: {e}"
    return results, errors


def build_line(args, r, errors):
    f = r.get("forward")
    fw_shape = r.get("_shape", (256, 256, 256))
    nx, ny, nz = fw_shape
    out = {
        "metric": "FD Gcell-steps/s (forward, 256^3, FP32)",
        "value": round(f["gcs"], 3) if f else None,
        "unit": "Gcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f["elapsed"] / args.steps * 1e3, 4) if f else None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "256^3 six-layer + 5% Gaussian-correlated perturbation, h 10 m, dt 0.5 ms, random MT "
                        "source, 12 Hz Ricker, 256 receivers, 20-cell Cerjan sponge, O(2,4) velocity-stress",
            "grid": [nx, ny, nz],
            "cells": nx * ny * nz,
            "time_steps": args.steps,
            "timing": "median of 5 runs of the given steps, each from a zero state set before the clock",
            "kernel": f["kernel"] if f else None,
            "bytes_per_cell_step": step_bytes(f["kernel"]) if f else None,
            "hbm_gbs_whole_step": round(f["wall_gbs"], 1) if f else None,
            "hbm_frac_whole_step": round(f["wall_gbs"] / HBM_PEAK_GBS, 4) if f else None,
        },
        "roofline": None,
    }
    if f:
        out["ms_per_step_runs"] = [round(t / args.steps * 1e3, 4) for t in f["times"]]
        out["roofline"] = {
            "bound": "hbm",
            "kernel": f["dom"],
            "achieved": f["per_kernel"][f["dom"]]["achieved_gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": f["per_kernel"][f["dom"]]["frac"],
            "traffic": f["traffic"],
            "bytes_per_launch": f["bytes_launch"],
            "per_kernel": f["per_kernel"],
            "whole_step": {"bytes_per_cell": step_bytes(f["kernel"]),
                           "achieved_events": round(f["events_gbs"], 1),
                           "frac_events": round(f["events_gbs"] / HBM_PEAK_GBS, 4),
                           "achieved_wall": round(f["wall_gbs"], 1),
                           "frac_wall": round(f["wall_gbs"] / HBM_PEAK_GBS, 4)},
        }
    for key in ("c1_full", "stream_copy_gbs", "c2_forward", "batched_forward", "gradient", "levels", "born",
                "coarse_medium", "layout_ab"):
        out[key] = r.get(key)
    out["paper_table6"] = paper_context()
    out["cpu_baseline"] = r.get("cpu_baseline")
    out["errors"] = errors or None
    return out


def main(argv=None):
    args = parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU path is not built.",
              file=sys.stderr)
        return 2
    if args.counters:
        counters_run(args.counters, args.steps, args.counters_grad)
        return 0
    state = {}

    def fwd():
        state["fw"] = Forward(max(args.steps, args.warmup, 2000 if not args.no_c1_full else 1), args.kernel,
                              args.layout)
        return bench_forward(state["fw"], args.steps, args.warmup)

    def c1_full():
        return bench_c1_full(state["fw"]) if "fw" in state and not args.no_c1_full else None

    def release():
        if "fw" in state:
            state["fw"].close()
            state["shot"] = state.pop("fw").shot
            import torch

            torch.cuda.empty_cache()

    def cpu():
        if args.cpu_steps <= 0:
            return None
        shot = state.get("shot")
        if shot is None:
            import workloads as W

            shot = W.c1(nt=1)
        return cpu_baseline(shot, args.cpu_steps)

    sections = [
        ("forward", fwd),
        ("c1_full", c1_full),
        ("_release", release),
        ("stream_copy_gbs", stream_copy_ceiling),
        ("c2_forward", (lambda: None) if args.no_c2 else (lambda: bench_c2(args.c2_steps))),
        ("batched_forward", (lambda: None) if args.no_batch else bench_batch),
        ("gradient", (lambda: None) if args.no_grad else (lambda: bench_gradient(wave=args.grad_wave, nshots=args.grad_shots))),
        ("levels", (lambda: None) if args.no_levels else bench_levels),
        ("born", (lambda: None) if args.no_born else bench_born),
        ("coarse_medium", (lambda: None) if args.no_coarse else bench_coarse_medium),
        ("layout_ab", (lambda: None) if args.no_layout_ab else bench_layout_ab),
        ("cpu_baseline", cpu),
    ]
    results, errors = run_sections(args, sections)
    results.pop("_release", None)
    out = build_line(args, results, errors)
    print(json.dumps(out), flush=True)
    return 1 if errors else 0


if __name__ == "__main__":
    sys.exit(main())
