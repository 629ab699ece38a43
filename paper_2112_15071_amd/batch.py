"""Many shots stepped together: one persistent launch per pass over every shot's tiles,
optionally replayed from one hipGraph holding the whole step sequence.

    sims = [Simulator(lam_s, mu_s, rho_s, dx, dt, nt) for each shot]
    batch = BatchSimulator(sims)
    traces = batch.forward([dict(src_pos=..., moment=..., wavelet=..., rec_pos=...), ...])
"""
from __future__ import annotations

from typing import Dict, List, Sequence

import numpy as np
import torch

from . import _abi
from .simulator import Simulator, _stream, make_source


class BatchSimulator:
    def __init__(self, sims: Sequence[Simulator]):
        if not sims:
            raise ValueError("empty batch")
        self.sims = list(sims)
        ctxs = [s.ctx for s in self.sims]
        nbytes = _abi.fd3d_batch_workspace_bytes(ctxs)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.sims[0].device)
        self._b = _abi.fd3d_batch_create(ctxs, self.workspace.data_ptr(), nbytes)
        self._keep = None

    @property
    def handle(self) -> int:
        return self._b

    def set_kernel(self, tile_x: int, tile_y: int, workgroups: int = 0, tile2=None) -> None:
        """Tile shape of the batched launches; tile2 = (tile_x, tile_y) of a second shape
        with the same workgroup size for the shots it covers with fewer idle columns."""
        t2 = tile2 or (0, 0)
        _abi.fd3d_batch_set_tiles(self._b, tile_x, tile_y, t2[0], t2[1], workgroups)

    def set_schedule(self, group_bytes: int = 0) -> None:
        """Order of the batched forward: 0 = lockstep (every launch covers every shot);
        otherwise cache-blocked groups of shots whose fields and models add up to at most
        group_bytes, each group stepped through all its steps before the next."""
        _abi.fd3d_batch_set_schedule(self._b, group_bytes)

    def autotune(self, steps: int = 10, cache: bool = True) -> dict:
        """Autotune every distinct grid shape of the batch for single-shot runs (each
        context also keeps its own z chunk, which the batch uses), then time the batched
        launch itself for every tile shape and grid mode in lockstep, then the
        cache-blocked schedule, and keep the fastest."""
        seen = {}
        for sim in self.sims:
            key = (sim.shape, sim.dtype)
            if key not in seen:
                seen[key] = sim.autotune(steps, cache)
            else:
                e = seen[key]
                sim.set_kernel(e["variant"], e["tile_y"], e["zchunk"], e["tile_x"])
        best = _abi.fd3d_batch_autotune(self._b, steps, _stream())
        best["per_shape"] = {f"{k[0]}": v for k, v in seen.items()}
        return best

    # (tile_x, tile_y, zchunk) configurations the batched-gradient tuner tries; zchunk 0:
    # each shot's whole depth (with several shots per launch, whole-depth sweeps can fill
    # the chip where one shot's cannot)
    GRADIENT_CANDIDATES = ((256, 4, 64), (256, 4, 128), (256, 4, 0), (128, 8, 64), (128, 4, 64), (128, 4, 128),
                           (64, 16, 64), (64, 8, 32))

    @staticmethod
    def _set_zchunk(sims, zc: int) -> None:
        for sim in sims:
            k = sim.kernel()
            sim.set_kernel(k["variant"], k["tile_y"], zc if zc > 0 else sim.shape[2], k["tile_x"])

    def autotune_gradient(self, shots: List[Dict], steps: int = 40, ckpt_every: int = 20, candidates=None) -> dict:
        """Pick the tile shape and z chunk of the batched gradient: times the batched
        gradient over ``steps`` steps (checkpoints every ``ckpt_every``, zero observed data,
        each shot's wavelet cut to ``steps``) on scratch contexts over the same models for
        every candidate (tile_x, tile_y, zchunk), then sets the fastest tile shape here and
        its z chunk on every simulator of the batch."""
        import time

        from .simulator import _shot_args

        steps = min(int(steps), min(sim.nt for sim in self.sims))
        ck = min(ckpt_every, steps)
        scratch = [sim.like(steps) for sim in self.sims]
        sb = BatchSimulator(scratch)
        args = [_shot_args(sh, steps) for sh in shots]
        d_obs = [torch.zeros((Simulator._rec(a.get("rec_pos"))[1], 3, steps), dtype=sim.dtype, device=sim.device)
                 for a, sim in zip(args, scratch)]
        gws = [sim.grad_workspace(ck) for sim in scratch]
        g = [[torch.zeros_like(sim.lam) for sim in scratch] for _ in range(3)]  # per shot: grids may differ
        times = {}
        for c in candidates or self.GRADIENT_CANDIDATES:
            tx, ty, zc = c
            try:
                sb.set_kernel(tx, ty)
                BatchSimulator._set_zchunk(scratch, zc)
            except _abi.FD3DError:
                continue  # a shape not built for this dtype, or too deep a window
            sb.gradient(args, d_obs, *g, ckpt_every=ck, gws=gws)
            torch.cuda.current_stream().synchronize()
            t0 = time.perf_counter()
            sb.gradient(args, d_obs, *g, ckpt_every=ck, gws=gws)
            torch.cuda.current_stream().synchronize()
            times[c] = (time.perf_counter() - t0) * 1e3 / steps
        sb.close()
        for sim in scratch:
            sim.close()
        if not times:
            raise RuntimeError("no batched-gradient configuration runs for this batch")
        best = min(times, key=times.get)
        self.set_kernel(best[0], best[1])
        BatchSimulator._set_zchunk(self.sims, best[2])
        return dict(tile=[best[0], best[1]], zchunk=self.sims[0].kernel()["zchunk"], ms_per_step=times[best],
                    tried={f"{x}x{y},{z if z else 'nz'}": round(v, 4) for (x, y, z), v in times.items()})

    def forward(self, shots: List[Dict], use_graph: bool = True, keep_state: bool = False,
                traces: List[torch.Tensor] = None) -> List[torch.Tensor]:
        if len(shots) != len(self.sims):
            raise ValueError("one shot description per simulator")
        srcs, nrec, rptr, tptr, keep = [], [], [], [], []
        out = []
        for k, (sim, sh) in enumerate(zip(self.sims, shots)):
            w = sim._wavelet(sh.get("wavelet"))
            srcs.append(make_source(sh["src_pos"], sh.get("moment", (0.0,) * 6), sh.get("force", (0.0,) * 3), w)
                        if sh.get("src_pos") is not None else _abi.fd3d_source())
            rp, nr = Simulator._rec(sh.get("rec_pos"))
            tr = traces[k] if traces is not None else torch.empty((nr, 3, sim.nt), dtype=sim.dtype, device=sim.device)
            nrec.append(nr)
            rptr.append(rp.ctypes.data if nr else 0)
            tptr.append(tr.data_ptr() if nr else 0)
            keep.append((rp, w))
            out.append(tr)
        flags = _abi.FD3D_KEEP_STATE if keep_state else 0
        _abi.fd3d_batch_forward(self._b, srcs, nrec, rptr, tptr, flags, use_graph, _stream())
        self._keep = keep
        return out

    def gradient(self, shots: List[Dict], d_obs: List[torch.Tensor], g_lam, g_mu, g_rho, ckpt_every: int = 50,
                 gws: List[torch.Tensor] = None, keep_state: bool = False):
        """Batched L2-misfit gradient.  g_* are one tensor (shared by all shots) or a list
        of per-shot tensors, accumulated.  Returns (traces list, misfit tensor [nshot])."""
        S = len(self.sims)
        if len(shots) != S or len(d_obs) != S:
            raise ValueError("one shot description and one d_obs per simulator")
        as_list = lambda g: list(g) if isinstance(g, (list, tuple)) else [g] * S
        gl, gm, gr = as_list(g_lam), as_list(g_mu), as_list(g_rho)
        if gws is None:
            gws = [sim.grad_workspace(ckpt_every) for sim in self.sims]
        bbytes = _abi.fd3d_batch_grad_workspace_bytes(self._b, ckpt_every)
        if getattr(self, "_bws", None) is None or self._bws.numel() < bbytes:
            self._bws = torch.empty(bbytes, dtype=torch.uint8, device=self.sims[0].device)
        srcs, nrec, rptr, keep, traces, obs = [], [], [], [], [], []
        for sim, sh, ob, g1, g2, g3 in zip(self.sims, shots, d_obs, gl, gm, gr):
            w = sim._wavelet(sh.get("wavelet"))
            srcs.append(make_source(sh["src_pos"], sh.get("moment", (0.0,) * 6), sh.get("force", (0.0,) * 3), w)
                        if sh.get("src_pos") is not None else _abi.fd3d_source())
            rp, nr = Simulator._rec(sh.get("rec_pos"))
            o = ob.to(device=sim.device, dtype=sim.dtype).contiguous()
            if tuple(o.shape) != (nr, 3, sim.nt):
                raise ValueError("d_obs must be [nrec, 3, nt]")
            for g in (g1, g2, g3):
                if g.dtype != sim.dtype or not g.is_contiguous() or tuple(g.shape) != tuple(sim.lam.shape):
                    raise ValueError("gradient buffers must be contiguous [nz, ny, nx] tensors of the context dtype")
            nrec.append(nr)
            rptr.append(rp.ctypes.data)
            keep.append((rp, w, o))
            obs.append(o)
            traces.append(torch.empty((nr, 3, sim.nt), dtype=sim.dtype, device=sim.device))
        misfit = torch.zeros(S, dtype=self.sims[0].dtype, device=self.sims[0].device)
        flags = _abi.FD3D_KEEP_STATE if keep_state else 0
        _abi.fd3d_batch_gradient(self._b, srcs, nrec, rptr, [o.data_ptr() for o in obs],
                                 [t.data_ptr() for t in traces], [misfit[s:s + 1].data_ptr() for s in range(S)],
                                 [g.data_ptr() for g in gl], [g.data_ptr() for g in gm], [g.data_ptr() for g in gr],
                                 [g.data_ptr() for g in gws], [g.numel() for g in gws], ckpt_every, flags,
                                 self._bws.data_ptr(), self._bws.numel(), _stream())
        self._keep = (keep, gws)
        return traces, misfit

    def close(self) -> None:
        if getattr(self, "_b", 0):
            torch.cuda.current_stream().synchronize()
            _abi.fd3d_batch_destroy(self._b)
            self._b = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
