"""Benchmark: forward elastic FD throughput (Gcell-steps/s) on one MI355X.

Workload: the 256^3 six-layer + 5 % Gaussian-perturbed model (h 10 m, dt 0.5 ms),
random moment-tensor source with a 12 Hz Ricker wavelet, 256 receivers, 20-cell
sponge, FP32.  A "step" is one time step of the whole forward path: velocity pass
(force source, damping), receiver sampling, stress pass (moment source, damping).

    python bench.py [--steps 2000] [--warmup 100] [--gpus 1]

Prints ONE JSON line.  Per-kernel durations come from HIP events recorded on the
stream the kernels run on; the CPU baseline is the FP64 oracle on a bounded sample
of the same workload (first few steps at full size) on this host's cores.
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
# algorithmic (compulsory) bytes per cell per launch, FP32: every field read once and
# every updated field written once
BYTES_PER_CELL = {
    "velocity": 4 * (6 + 3 + 1 + 3),   # read 6 stress, 3 velocity, rho; write 3 velocity
    "stress": 4 * (3 + 6 + 2 + 6),     # read 3 velocity, 6 stress, lambda, mu; write 6 stress
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--cpu-steps", type=int, default=4, help="oracle steps for the CPU baseline sample (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU path is not built.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_2112_15071_amd import Simulator, _abi

    dev = torch.device("cuda:0")
    K, Wm = args.steps, args.warmup
    log(f"[bench] generating the 256^3 workload (steps {K}, warmup {Wm})")
    shot = W.c1(nt=max(K, Wm))
    nx, ny, nz = shot.shape
    cells = nx * ny * nz
    lam, mu, rho = (torch.as_tensor(a, dtype=torch.float32).to(dev) for a in (shot.lam, shot.mu, shot.rho))
    wav = torch.as_tensor(shot.wavelet, dtype=torch.float32).to(dev)
    kw = dict(dtype=torch.float32, sponge=shot.sponge, device=dev)

    if Wm > 0:
        warm = Simulator(lam, mu, rho, shot.h, shot.dt, Wm, **kw)
        warm.forward(shot.src_pos, shot.moment, shot.force, wav[:Wm], shot.rec_pos)
        torch.cuda.synchronize()
        warm.close()
        del warm

    sim = Simulator(lam, mu, rho, shot.h, shot.dt, K, **kw)
    traces = torch.empty((shot.rec_pos.shape[0], 3, K), dtype=torch.float32, device=dev)
    log(f"[bench] timed forward: {K} steps on {nx}x{ny}x{nz}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.forward(shot.src_pos, shot.moment, shot.force, wav[:K], shot.rec_pos, traces=traces)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    gcs = cells * K / elapsed / 1e9
    log(f"[bench] {elapsed:.3f} s -> {gcs:.2f} Gcell-steps/s")

    # same run again with per-kernel HIP events on the launch stream
    _abi.fd3d_profile(sim.ctx, True)
    torch.cuda.synchronize()
    p0 = time.perf_counter()
    sim.forward(shot.src_pos, shot.moment, shot.force, wav[:K], shot.rec_pos, traces=traces)
    ms, launches = _abi.fd3d_profile_read(sim.ctx)
    torch.cuda.synchronize()
    p1 = time.perf_counter()
    _abi.fd3d_profile(sim.ctx, False)
    names = ("velocity", "record", "stress")
    per = {names[i]: (ms[i] / max(launches[i], 1)) for i in range(3)}
    log(f"[bench] profiled run {p1 - p0:.3f} s; avg kernel ms: " + ", ".join(f"{k} {v:.4f}" for k, v in per.items()))
    dom = "stress" if ms[2] >= ms[0] else "velocity"
    bytes_launch = BYTES_PER_CELL[dom] * cells
    achieved = bytes_launch / (per[dom] * 1e-3) / 1e9
    both = (BYTES_PER_CELL["velocity"] + BYTES_PER_CELL["stress"]) * cells * K / (elapsed * 1e9)
    log(f"[bench] dominant {dom}: {achieved:.0f} GB/s; whole step {both:.0f} GB/s")
    sim.close()

    cpu = None
    if args.cpu_steps > 0:
        import oracle

        oracle.build(force=False)
        ns = args.cpu_steps
        cfg = oracle.Config(shot.shape, shot.h, shot.dt, ns, sponge=shot.sponge)
        src = oracle.Source(shot.src_pos, moment=shot.moment, force=shot.force)
        log(f"[bench] oracle baseline: {ns} steps at full size on {oracle.get_threads()} threads")
        c0 = time.perf_counter()
        oracle.forward(cfg, shot.lam, shot.mu, shot.rho, src, shot.wavelet[:ns], shot.rec_pos)
        c1 = time.perf_counter()
        cpu = {"value": cells * ns / (c1 - c0) / 1e9, "unit": "Gcell-steps/s", "cores": oracle.get_threads(),
               "kind": "oracle", "sample": f"FP64 oracle, 256^3 workload, first {ns} of 2000 steps ({c1 - c0:.1f} s)"}
        log(f"[bench] oracle {cpu['value']:.4f} Gcell-steps/s")

    out = {
        "metric": "FD Gcell-steps/s (forward, 256^3, FP32)",
        "value": round(gcs, 3),
        "unit": "Gcell-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": round(elapsed / K * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "256^3 six-layer + 5% Gaussian-correlated perturbation, h 10 m, dt 0.5 ms, random MT "
                        "source, 12 Hz Ricker, 256 receivers, 20-cell Cerjan sponge, O(2,4) velocity-stress",
            "grid": [nx, ny, nz],
            "cells": cells,
            "time_steps": K,
            "hbm_gbs_whole_step": round(both, 1),
            "bytes_per_cell_step": BYTES_PER_CELL["velocity"] + BYTES_PER_CELL["stress"],
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
            "avg_kernel_ms": {k: round(v, 5) for k, v in per.items()},
            "bytes_per_launch": bytes_launch,
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
