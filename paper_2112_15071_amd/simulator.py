"""Torch-facing wrapper of the fd3d C ABI: device memory and streams come from torch,
every step of the method runs in the HIP library.

    sim = Simulator(lam, mu, rho, dx=10.0, dt=1e-3, nt=500, sponge=20)
    traces = sim.forward(src_pos=(32, 32, 32), moment=(1e15, 1e15, 1e15, 0, 0, 0),
                         wavelet=w, rec_pos=rec)            # [nrec, 3, nt] on the GPU
    state = sim.state()                                     # [9, nz, ny, nx]
"""
from __future__ import annotations

from typing import Optional, Sequence

import json
import os

import numpy as np
import torch

from . import _abi

FIELDS = ("vx", "vy", "vz", "sxx", "syy", "szz", "sxy", "sxz", "syz")


def _dtype_code(dtype: torch.dtype) -> int:
    if dtype == torch.float32:
        return _abi.FD3D_F32
    if dtype == torch.float64:
        return _abi.FD3D_F64
    raise ValueError("dtype must be torch.float32 or torch.float64")


def _stream() -> int:
    return int(torch.cuda.current_stream().cuda_stream)


def make_opts(dtype: torch.dtype, sponge=0, sponge_alpha: float = 0.0, free_surface: bool = False,
              check_finite: bool = False, max_receivers: int = 4096, dy: float = 0.0,
              dz: float = 0.0, vacuum_top: int = 0, vacuum_map: int = 0, coarse=None,
              layout: str = "auto") -> _abi.fd3d_opts:
    o = _abi.fd3d_opts()
    o.dtype = _dtype_code(dtype)
    sp = [int(sponge)] * 6 if np.isscalar(sponge) else [int(v) for v in sponge]
    if len(sp) != 6:
        raise ValueError("sponge is one width or six (x-, x+, y-, y+, z-, z+)")
    for f in range(6):
        o.sponge[f] = sp[f]
    o.sponge_alpha = float(sponge_alpha)
    o.free_surface = int(bool(free_surface))
    o.check_finite = int(bool(check_finite))
    o.max_receivers = int(max_receivers)
    o.dy, o.dz = float(dy), float(dz)
    o.vacuum_top = int(vacuum_top)
    o.vacuum_map = int(vacuum_map) or None
    if coarse is not None:
        for a in range(3):
            o.coarse[a] = int(coarse[a])
    if layout not in LAYOUTS:
        raise ValueError(f"layout must be one of {sorted(LAYOUTS)}")
    o.layout = LAYOUTS[layout]
    return o


# field storage in the workspace (fd3d_opts.layout): "rows" interleaves the nine fields' rows
# ([nz][ny][9][nx]), "separate" keeps one array per field, "auto" lets the library choose
LAYOUTS = {"auto": _abi.FD3D_LAYOUT_AUTO, "separate": _abi.FD3D_LAYOUT_SEPARATE, "rows": _abi.FD3D_LAYOUT_ROWS}


def make_source(pos, moment=(0.0,) * 6, force=(0.0,) * 3, wavelet: Optional[torch.Tensor] = None) -> _abi.fd3d_source:
    s = _abi.fd3d_source()
    for a in range(3):
        s.pos[a] = float(pos[a])
        s.force[a] = float(force[a])
    for q in range(6):
        s.moment[q] = float(moment[q])
    s.wavelet = int(wavelet.data_ptr()) if wavelet is not None else None
    return s


def upsample(coarse: torch.Tensor, shape) -> torch.Tensor:
    """A medium array given on a coarse node grid ([mz, my, mx] device tensor) sampled
    trilinearly at the nodes of the simulation grid ``shape`` = (nx, ny, nz), both grids
    spanning the same box (fd3d_upsample)."""
    c = coarse.contiguous()
    if c.dim() != 3 or not c.is_cuda:
        raise ValueError("coarse must be a 3-D device tensor [mz, my, mx]")
    nx, ny, nz = (int(v) for v in shape)
    out = torch.empty((nz, ny, nx), dtype=c.dtype, device=c.device)
    mz, my, mx = c.shape
    _abi.fd3d_upsample(c.data_ptr(), (mx, my, mz), out.data_ptr(), (nx, ny, nz), _dtype_code(c.dtype), _stream())
    return out


def forward_static(lam, mu, rho, dx: float, dt: float, nt: int, src_pos=None, moment=(0.0,) * 6, force=(0.0,) * 3,
                   wavelet=None, rec_pos=None, dtype: torch.dtype = torch.float32, sponge=20,
                   sponge_alpha: float = 0.0, free_surface: bool = False, traces: Optional[torch.Tensor] = None,
                   state: Optional[torch.Tensor] = None, max_receivers: int = 4096):
    """One forward run whose workspace is the library's static device scratch
    (fd3d_forward_static): for small grids in code that must not allocate device memory.
    Inputs are device tensors of ``dtype``; ``traces`` [nrec, 3, nt] and ``state``
    [9, nz, ny, nx] (optional) are written.  dx is one spacing or (dx, dy, dz).  Returns
    (traces, state).  Synchronises the current stream."""
    nz, ny, nx = lam.shape
    sp = tuple(float(v) for v in np.broadcast_to(np.asarray(dx, dtype=np.float64), (3,)))
    opts = make_opts(dtype, sponge, sponge_alpha, free_surface, False, max_receivers, sp[1], sp[2])
    for a in (lam, mu, rho, wavelet, traces, state):
        if a is not None and (not a.is_cuda or a.dtype != dtype or not a.is_contiguous()):
            raise ValueError("inputs and outputs must be contiguous device tensors of the given dtype")
    if wavelet is not None and wavelet.numel() != nt:
        raise ValueError(f"wavelet needs nt = {nt} samples")
    src = make_source(src_pos, moment, force, wavelet) if src_pos is not None else None
    rp, nrec = Simulator._rec(rec_pos)
    if nrec and (traces is None or tuple(traces.shape) != (nrec, 3, nt)):
        raise ValueError(f"traces must be [nrec, 3, nt] = {(nrec, 3, nt)}")
    if state is not None and tuple(state.shape) != (9, nz, ny, nx):
        raise ValueError("state must be [9, nz, ny, nx]")
    _abi.fd3d_forward_static((nx, ny, nz), lam.data_ptr(), mu.data_ptr(), rho.data_ptr(), sp[0], dt, nt, opts, src,
                             nrec, rp.ctypes.data if nrec else None, traces.data_ptr() if nrec else None,
                             [state[f].data_ptr() for f in range(9)] if state is not None else None, _stream())
    return traces, state


def _shot_args(shot: dict, steps: int) -> dict:
    """Source and receiver arguments of a shot description, its wavelet cut to ``steps``."""
    args = {k: shot[k] for k in ("src_pos", "moment", "force", "rec_pos") if shot.get(k) is not None}
    if shot.get("wavelet") is not None:
        args["wavelet"] = torch.as_tensor(shot["wavelet"])[:steps]
    return args


class Simulator:
    """One grid and model on one GPU; forward runs of ``nt`` steps."""

    def __init__(self, lam, mu, rho, dx: float, dt: float, nt: int, dtype: torch.dtype = torch.float32,
                 sponge=20, sponge_alpha: float = 0.0, free_surface: bool = False, check_finite: bool = False,
                 max_receivers: int = 4096, device="cuda", vacuum_top: int = 0, vacuum_map=None, grid=None,
                 layout: str = "auto"):
        """``grid`` = (nx, ny, nz) of the simulation when it differs from the medium arrays'
        shape: lam, mu, rho are then a coarse medium over the same box, read by trilinear
        samples at every value's own position inside the step kernels (fd3d_opts.coarse;
        forward only, tile kernels).  ``layout``: the fields' storage ("auto", "separate",
        "rows"; fd3d_opts.layout), which changes speed, never results."""
        self.device = torch.device(device)
        self.dtype = dtype
        self.lam, self.mu, self.rho = (torch.as_tensor(a).to(device=self.device, dtype=dtype).contiguous()
                                       for a in (lam, mu, rho))
        if self.lam.dim() != 3 or self.mu.shape != self.lam.shape or self.rho.shape != self.lam.shape:
            raise ValueError("lam, mu, rho must share one [nz, ny, nx] shape")
        nz, ny, nx = self.lam.shape
        self.coarse = None
        if grid is not None and tuple(int(v) for v in grid) != (nx, ny, nz):
            self.coarse = (nx, ny, nz)
            nx, ny, nz = (int(v) for v in grid)
        self.shape = (nx, ny, nz)
        # one spacing, or (dx, dy, dz) for cells of different size per axis
        self.spacing = tuple(float(v) for v in (np.broadcast_to(np.asarray(dx, dtype=np.float64), (3,))))
        self.dx, self.dt, self.nt = self.spacing[0], float(dt), int(nt)
        # vacuum surface: one first-solid plane, or one per column ([ny, nx] integers)
        self.vacuum_map = None
        if vacuum_map is not None:
            self.vacuum_map = torch.as_tensor(vacuum_map).to(device=self.device, dtype=torch.int32).contiguous()
            if tuple(self.vacuum_map.shape) != (ny, nx):
                raise ValueError("vacuum_map must be [ny, nx]")
            vacuum_top = vacuum_top or int(self.vacuum_map.max())
        self.opts = make_opts(dtype, sponge, sponge_alpha, free_surface, check_finite, max_receivers,
                              self.spacing[1], self.spacing[2], vacuum_top,
                              self.vacuum_map.data_ptr() if self.vacuum_map is not None else 0, self.coarse,
                              layout)
        nbytes = _abi.fd3d_workspace_bytes(nx, ny, nz, self.opts)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._ctx = _abi.fd3d_create(nx, ny, nz, self.lam.data_ptr(), self.mu.data_ptr(), self.rho.data_ptr(),
                                     self.dx, self.dt, self.nt, self.opts, self.workspace.data_ptr(), nbytes, _stream())
        self._rec_keep = None

    # -- helpers -------------------------------------------------------------
    def _wavelet(self, wavelet) -> Optional[torch.Tensor]:
        if wavelet is None:
            return None
        w = torch.as_tensor(wavelet).to(device=self.device, dtype=self.dtype).contiguous()
        if w.numel() != self.nt:
            raise ValueError(f"wavelet needs nt = {self.nt} samples")
        return w

    @staticmethod
    def _rec(rec_pos):
        if rec_pos is None:
            return np.zeros((0, 3)), 0
        r = np.ascontiguousarray(np.asarray(rec_pos, dtype=np.float64).reshape(-1, 3))
        return r, r.shape[0]

    @property
    def ctx(self) -> int:
        return self._ctx

    _VARIANTS = {"cell": 0, "tile": 1, "fused": 2}

    def set_kernel(self, variant: str = "tile", tile_y: int = 8, zchunk: int = 32, tile_x: int = 64) -> None:
        """Select the step-loop kernels: "cell" (one thread per cell), "tile" (LDS halo
        planes + register z sweep over tile_x x tile_y columns, zchunk planes) or "fused"
        (velocity and stress of a step in one sweep, tile_x = 64)."""
        k = _abi.fd3d_kernel()
        k.variant = self._VARIANTS[variant]
        k.tile_x, k.tile_y, k.zchunk = int(tile_x), int(tile_y), int(zchunk)
        _abi.fd3d_set_kernel(self._ctx, k)

    def layout(self) -> str:
        """The field storage the library chose: "separate" or "rows"."""
        return {v: n for n, v in LAYOUTS.items()}[_abi.fd3d_get_layout(self._ctx)]

    def kernel(self) -> dict:
        k = _abi.fd3d_get_kernel(self._ctx)
        name = {v: n for n, v in self._VARIANTS.items()}[k.variant]
        return {"variant": name, "tile_x": k.tile_x, "tile_y": k.tile_y, "zchunk": k.zchunk}

    def autotune(self, steps: int = 20, cache: bool = True) -> dict:
        """Pick the fastest kernel variant, tile shape and z chunk for this grid (fd3d_autotune), with a
        JSON cache keyed by grid shape, dtype, free surface and device (CU count, memory size)
        ($FD3D_AUTOTUNE_CACHE, default ~/.cache/fd3d/autotune.json).  Zeroes the state."""
        nx, ny, nz = self.shape
        props = torch.cuda.get_device_properties(self.device)
        dev = f"{props.multi_processor_count}cu-{props.total_memory >> 30}gib"
        cm = "" if self.coarse is None else "/cm{}x{}x{}".format(*self.coarse)
        key = f"{nx}x{ny}x{nz}/{str(self.dtype)}/fs{int(self.opts.free_surface)}{cm}/{self.layout()}/{dev}"
        path = os.environ.get("FD3D_AUTOTUNE_CACHE", os.path.expanduser("~/.cache/fd3d/autotune.json"))
        table = {}
        if cache and os.path.exists(path):
            try:
                with open(path) as f:
                    table = json.load(f)
            except (OSError, ValueError):
                table = {}
        if cache and key in table and "variant" in table[key]:
            e = table[key]
            self.set_kernel(e["variant"], e["tile_y"], e["zchunk"], e["tile_x"])
            return dict(e, cached=True)
        _, ms = _abi.fd3d_autotune(self._ctx, steps, _stream())
        e = dict(self.kernel(), ms_per_step=ms)
        if cache:
            table[key] = e
            try:
                os.makedirs(os.path.dirname(path), exist_ok=True)
                tmp = path + f".{os.getpid()}.tmp"
                with open(tmp, "w") as f:
                    json.dump(table, f, indent=1, sort_keys=True)
                os.replace(tmp, path)
            except OSError:
                pass
        return dict(e, cached=False)

    # kernel configurations the gradient tuner tries (variant, tile_x, tile_y, zchunk)
    GRADIENT_CANDIDATES = (("tile", 256, 4, 64), ("tile", 256, 4, 128), ("tile", 256, 4, 0), ("tile", 128, 4, 64),
                           ("tile", 128, 4, 128), ("tile", 128, 8, 64), ("tile", 64, 16, 64), ("tile", 64, 8, 32))

    def like(self, nt: int) -> "Simulator":
        """A new context over the same model arrays, spacing and options, with nt steps and
        this context's kernel configuration."""
        o = self.opts
        sim = Simulator(self.lam, self.mu, self.rho, self.spacing, self.dt, nt, dtype=self.dtype,
                        sponge=[o.sponge[f] for f in range(6)], sponge_alpha=o.sponge_alpha,
                        free_surface=bool(o.free_surface), check_finite=bool(o.check_finite),
                        max_receivers=o.max_receivers, device=self.device, vacuum_top=o.vacuum_top,
                        vacuum_map=self.vacuum_map, grid=self.shape, layout=self.layout())
        k = self.kernel()
        sim.set_kernel(k["variant"], k["tile_y"], k["zchunk"], k["tile_x"])
        return sim

    def autotune_gradient(self, shot: dict, steps: int = 40, ckpt_every: int = 20, candidates=None) -> dict:
        """Pick the kernel configuration for gradients of this grid: times fd3d_gradient over
        ``steps`` steps (checkpoints every ``ckpt_every``, zero observed data, ``shot``'s
        source and receivers with its wavelet cut to ``steps``) on a scratch context over the
        same model for every candidate (variant, tile_x, tile_y, zchunk; zchunk 0: the whole
        depth), and sets the fastest here.  The forward tuner (``autotune``) times the forward passes only; the adjoint
        passes move more fields per cell and can rank tile shapes differently."""
        import time

        cands = candidates or self.GRADIENT_CANDIDATES
        steps = min(int(steps), self.nt)
        scratch = self.like(steps)
        gws = scratch.grad_workspace(min(ckpt_every, steps))
        args = _shot_args(shot, steps)
        nrec = Simulator._rec(args.get("rec_pos"))[1]
        d_obs = torch.zeros((nrec, 3, steps), dtype=self.dtype, device=self.device)
        g = [torch.zeros_like(self.lam) for _ in range(3)]
        times = {}
        for c in cands:
            variant, tx, ty, zc = c
            try:
                scratch.set_kernel(variant, ty, zc if zc > 0 else self.shape[2], tx)
            except _abi.FD3DError:
                continue  # not built for this dtype or too deep a window for this grid
            scratch.gradient(gws, d_obs, *g, **args)
            torch.cuda.current_stream().synchronize()
            t0 = time.perf_counter()
            scratch.gradient(gws, d_obs, *g, **args)
            torch.cuda.current_stream().synchronize()
            times[c] = (time.perf_counter() - t0) * 1e3 / steps
        scratch.close()
        if not times:
            raise RuntimeError("no gradient kernel candidate runs on this grid")
        best = min(times, key=times.get)
        self.set_kernel(best[0], best[2], best[3] if best[3] > 0 else self.shape[2], best[1])
        return dict(self.kernel(), ms_per_step=times[best],
                    tried={f"{v},{x},{y},{z if z else 'nz'}": round(t, 4) for (v, x, y, z), t in times.items()})

    def info(self):
        """(vp_max, vs_min, rho_min, dt_max) read back at creation."""
        return _abi.fd3d_model_info(self._ctx)

    # -- public API ----------------------------------------------------------
    def forward(self, src_pos=None, moment=(0.0,) * 6, force=(0.0,) * 3, wavelet=None, rec_pos=None,
                keep_state: bool = False, traces: Optional[torch.Tensor] = None) -> torch.Tensor:
        w = self._wavelet(wavelet)
        src = make_source(src_pos, moment, force, w) if src_pos is not None else None
        rp, nrec = self._rec(rec_pos)
        if traces is None:
            traces = torch.empty((nrec, 3, self.nt), dtype=self.dtype, device=self.device)
        flags = _abi.FD3D_KEEP_STATE if keep_state else 0
        _abi.fd3d_forward(self._ctx, src, nrec, rp.ctypes.data if nrec else None,
                          traces.data_ptr() if nrec else None, flags, _stream())
        self._rec_keep = (rp, w)  # host/device inputs stay referenced until the next call
        return traces

    # -- tangent-linear (Born) ----------------------------------------------------
    def born(self, dlam, dmu, drho, src_pos=None, moment=(0.0,) * 6, force=(0.0,) * 3, wavelet=None, rec_pos=None):
        """Tangent-linear forward (fd3d_born): returns (traces, dtraces), the background traces
        and their derivative along the model perturbation (dlam, dmu, drho) (node arrays of
        the model's shape).  The perturbation state lives in a second context over the same
        model, created on first use with this one's options and kernel."""
        if getattr(self, "_born_sim", None) is None:
            o = self.opts
            sp = [o.sponge[f] for f in range(6)]
            self._born_sim = Simulator(self.lam, self.mu, self.rho, self.spacing, self.dt, self.nt, dtype=self.dtype,
                                       sponge=sp, sponge_alpha=o.sponge_alpha, free_surface=bool(o.free_surface),
                                       max_receivers=o.max_receivers, device=self.device, layout=self.layout())
        d = self._born_sim
        k = self.kernel()
        d.set_kernel(k["variant"], k["tile_y"], k["zchunk"], k["tile_x"])
        dm = [torch.as_tensor(a).to(device=self.device, dtype=self.dtype).contiguous() for a in (dlam, dmu, drho)]
        for a in dm:
            if a.shape != self.lam.shape:
                raise ValueError("dlam, dmu, drho must have the model's shape")
        w = self._wavelet(wavelet)
        src = make_source(src_pos, moment, force, w) if src_pos is not None else None
        rp, nrec = self._rec(rec_pos)
        traces = torch.empty((nrec, 3, self.nt), dtype=self.dtype, device=self.device)
        dtraces = torch.empty_like(traces)
        _abi.fd3d_born(self._ctx, d._ctx, src, *(a.data_ptr() for a in dm), nrec, rp.ctypes.data if nrec else None,
                       traces.data_ptr() if nrec else None, dtraces.data_ptr() if nrec else None, _stream())
        self._rec_keep = (rp, w, dm)
        return traces, dtraces

    # -- gradient --------------------------------------------------------------
    def grad_workspace(self, ckpt_every: int) -> torch.Tensor:
        """Device buffer for checkpoints, adjoint state and gradient accumulators."""
        nbytes = _abi.fd3d_grad_workspace_bytes(self._ctx, int(ckpt_every))
        gws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        gws.ckpt_every = int(ckpt_every)
        return gws

    def forward_ckpt(self, gws: torch.Tensor, src_pos=None, moment=(0.0,) * 6, force=(0.0,) * 3, wavelet=None,
                     rec_pos=None, keep_state: bool = False, traces: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Forward run that also stores checkpoints in ``gws`` for a later adjoint."""
        w = self._wavelet(wavelet)
        src = make_source(src_pos, moment, force, w) if src_pos is not None else None
        rp, nrec = self._rec(rec_pos)
        if traces is None:
            traces = torch.empty((nrec, 3, self.nt), dtype=self.dtype, device=self.device)
        flags = _abi.FD3D_KEEP_STATE if keep_state else 0
        _abi.fd3d_forward_ckpt(self._ctx, src, nrec, rp.ctypes.data if nrec else None,
                               traces.data_ptr() if nrec else None, flags, gws.data_ptr(), gws.numel(),
                               gws.ckpt_every, _stream())
        self._rec_keep = (rp, w)
        return traces

    def adjoint(self, gws: torch.Tensor, residual: torch.Tensor, g_lam: torch.Tensor, g_mu: torch.Tensor,
                g_rho: torch.Tensor, src_pos=None, moment=(0.0,) * 6, force=(0.0,) * 3, wavelet=None,
                rec_pos=None) -> None:
        """Reverse sweep; accumulates dJ/dlambda, dJ/dmu, dJ/drho (node arrays) into g_*."""
        w = self._wavelet(wavelet)
        src = make_source(src_pos, moment, force, w) if src_pos is not None else None
        rp, nrec = self._rec(rec_pos)
        res = residual.to(device=self.device, dtype=self.dtype).contiguous()
        if tuple(res.shape) != (nrec, 3, self.nt):
            raise ValueError(f"residual must be [nrec, 3, nt] = {(nrec, 3, self.nt)}")
        for g in (g_lam, g_mu, g_rho):
            if g.dtype != self.dtype or not g.is_contiguous() or tuple(g.shape) != tuple(self.lam.shape):
                raise ValueError("gradient buffers must be contiguous [nz, ny, nx] tensors of the context dtype")
        _abi.fd3d_adjoint(self._ctx, src, nrec, rp.ctypes.data if nrec else None, res.data_ptr(),
                          g_lam.data_ptr(), g_mu.data_ptr(), g_rho.data_ptr(), gws.data_ptr(), gws.numel(),
                          _stream())
        self._rec_keep = (rp, w, res)

    def gradient(self, gws: torch.Tensor, d_obs: torch.Tensor, g_lam: torch.Tensor, g_mu: torch.Tensor,
                 g_rho: torch.Tensor, src_pos=None, moment=(0.0,) * 6, force=(0.0,) * 3, wavelet=None,
                 rec_pos=None):
        """One shot of J = 1/2 |d - d_obs|^2: returns (traces, J as a 1-element tensor);
        the gradient is accumulated into g_*."""
        w = self._wavelet(wavelet)
        src = make_source(src_pos, moment, force, w) if src_pos is not None else None
        rp, nrec = self._rec(rec_pos)
        obs = d_obs.to(device=self.device, dtype=self.dtype).contiguous()
        if tuple(obs.shape) != (nrec, 3, self.nt):
            raise ValueError(f"d_obs must be [nrec, 3, nt] = {(nrec, 3, self.nt)}")
        for g in (g_lam, g_mu, g_rho):
            if g.dtype != self.dtype or not g.is_contiguous() or tuple(g.shape) != tuple(self.lam.shape):
                raise ValueError("gradient buffers must be contiguous [nz, ny, nx] tensors of the context dtype")
        traces = torch.empty((nrec, 3, self.nt), dtype=self.dtype, device=self.device)
        J = torch.empty(1, dtype=self.dtype, device=self.device)
        _abi.fd3d_gradient(self._ctx, src, nrec, rp.ctypes.data, obs.data_ptr(), traces.data_ptr(), J.data_ptr(),
                           g_lam.data_ptr(), g_mu.data_ptr(), g_rho.data_ptr(), gws.data_ptr(), gws.numel(),
                           gws.ckpt_every, _stream())
        self._rec_keep = (rp, w, obs)
        return traces, J

    def adjoint_state(self, gws: torch.Tensor) -> torch.Tensor:
        """Adjoint of the initial state (v^{-1/2}, sigma^0) after ``adjoint``."""
        nx, ny, nz = self.shape
        out = torch.empty((9, nz, ny, nx), dtype=self.dtype, device=self.device)
        _abi.fd3d_get_adjoint_state(self._ctx, gws.data_ptr(), [out[f].data_ptr() for f in range(9)], _stream())
        return out

    def state(self) -> torch.Tensor:
        nx, ny, nz = self.shape
        out = torch.empty((9, nz, ny, nx), dtype=self.dtype, device=self.device)
        _abi.fd3d_get_state(self._ctx, [out[f].data_ptr() for f in range(9)], _stream())
        return out

    def set_state(self, st) -> None:
        nx, ny, nz = self.shape
        st = torch.as_tensor(st).to(device=self.device, dtype=self.dtype).contiguous()
        if tuple(st.shape) != (9, nz, ny, nx):
            raise ValueError("state must be [9, nz, ny, nx]")
        self._state_keep = st
        _abi.fd3d_set_state(self._ctx, [st[f].data_ptr() for f in range(9)], _stream())

    def close(self) -> None:
        if getattr(self, "_born_sim", None) is not None:
            self._born_sim.close()
            self._born_sim = None
        if getattr(self, "_ctx", 0):
            torch.cuda.current_stream().synchronize()
            _abi.fd3d_destroy(self._ctx)
            self._ctx = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
