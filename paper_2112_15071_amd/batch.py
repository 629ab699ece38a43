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

    def set_kernel(self, tile_x: int, tile_y: int, workgroups: int = 0) -> None:
        _abi.fd3d_batch_set_kernel(self._b, tile_x, tile_y, workgroups)

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
