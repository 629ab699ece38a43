"""ctypes binding of the fd3d C ABI (include/fd3d.h): argument marshalling only.

Every function keeps its C name.  Pointers are passed as integers (device
addresses from torch tensors, host addresses from numpy arrays).  A non-zero
return code raises FD3DError with the library's message.  There is no fallback:
if libfd3d.so is missing, importing this module fails.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfd3d.so")

FD3D_OK = 0
FD3D_EINVAL = -1
FD3D_ECFL = -2
FD3D_EMODEL = -3
FD3D_ERANGE = -4
FD3D_EWS = -5
FD3D_EHIP = -6
FD3D_ENONFINITE = -7
FD3D_ESTATE = -8
FD3D_F32 = 0
FD3D_F64 = 1
FD3D_KEEP_STATE = 1
FD3D_KERNEL_CELL = 0
FD3D_KERNEL_TILE = 1
FD3D_KERNEL_FUSED = 2
FD3D_STATIC_SCRATCH_BYTES = 64 << 20
FD3D_LAYOUT_AUTO = 0
FD3D_LAYOUT_SEPARATE = 1
FD3D_LAYOUT_ROWS = 2

ERRNAMES = {
    FD3D_EINVAL: "FD3D_EINVAL", FD3D_ECFL: "FD3D_ECFL", FD3D_EMODEL: "FD3D_EMODEL", FD3D_ERANGE: "FD3D_ERANGE",
    FD3D_EWS: "FD3D_EWS", FD3D_EHIP: "FD3D_EHIP", FD3D_ENONFINITE: "FD3D_ENONFINITE", FD3D_ESTATE: "FD3D_ESTATE",
}


class FD3DError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class fd3d_opts(ctypes.Structure):
    _fields_ = [
        ("dtype", ctypes.c_int),
        ("sponge", ctypes.c_int * 6),
        ("sponge_alpha", ctypes.c_double),
        ("free_surface", ctypes.c_int),
        ("check_finite", ctypes.c_int),
        ("max_receivers", ctypes.c_int),
        ("dy", ctypes.c_double),
        ("dz", ctypes.c_double),
        ("vacuum_top", ctypes.c_int),
        ("vacuum_map", ctypes.c_void_p),
        ("coarse", ctypes.c_int * 3),
        ("layout", ctypes.c_int),
    ]


class fd3d_kernel(ctypes.Structure):
    _fields_ = [
        ("variant", ctypes.c_int),
        ("tile_x", ctypes.c_int),
        ("tile_y", ctypes.c_int),
        ("zchunk", ctypes.c_int),
    ]


class fd3d_source(ctypes.Structure):
    _fields_ = [
        ("pos", ctypes.c_double * 3),
        ("moment", ctypes.c_double * 6),
        ("force", ctypes.c_double * 3),
        ("wavelet", ctypes.c_void_p),
    ]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")

_lib = ctypes.CDLL(LIB_PATH)

_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
_sz = ctypes.c_size_t
_dp = ctypes.POINTER(ctypes.c_double)

_SIGS = {
    "fd3d_version": ([], ctypes.c_char_p),
    "fd3d_last_error": ([], ctypes.c_char_p),
    "fd3d_workspace_bytes": ([_i, _i, _i, ctypes.POINTER(fd3d_opts), ctypes.POINTER(_sz)], _i),
    "fd3d_create": ([ctypes.POINTER(_vp), _i, _i, _i, _vp, _vp, _vp, _d, _d, _i, ctypes.POINTER(fd3d_opts), _vp, _sz, _vp], _i),
    "fd3d_forward": ([_vp, ctypes.POINTER(fd3d_source), _i, _dp, _vp, _i, _vp], _i),
    "fd3d_get_state": ([_vp, ctypes.POINTER(_vp), _vp], _i),
    "fd3d_set_state": ([_vp, ctypes.POINTER(_vp), _vp], _i),
    "fd3d_model_info": ([_vp, _dp], _i),
    "fd3d_get_layout": ([_vp, ctypes.POINTER(_i)], _i),
    "fd3d_grad_workspace_bytes": ([_vp, _i, ctypes.POINTER(_sz)], _i),
    "fd3d_forward_ckpt": ([_vp, ctypes.POINTER(fd3d_source), _i, _dp, _vp, _i, _vp, _sz, _i, _vp], _i),
    "fd3d_adjoint": ([_vp, ctypes.POINTER(fd3d_source), _i, _dp, _vp, _vp, _vp, _vp, _vp, _sz, _vp], _i),
    "fd3d_gradient": ([_vp, ctypes.POINTER(fd3d_source), _i, _dp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _i, _vp], _i),
    "fd3d_born": ([_vp, _vp, ctypes.POINTER(fd3d_source), _vp, _vp, _vp, _i, _dp, _vp, _vp, _vp], _i),
    "fd3d_get_adjoint_state": ([_vp, _vp, ctypes.POINTER(_vp), _vp], _i),
    "fd3d_batch_workspace_bytes": ([_i, ctypes.POINTER(_vp), ctypes.POINTER(_sz)], _i),
    "fd3d_batch_create": ([ctypes.POINTER(_vp), _i, ctypes.POINTER(_vp), _vp, _sz], _i),
    "fd3d_batch_set_kernel": ([_vp, _i, _i, _i], _i),
    "fd3d_batch_set_tiles": ([_vp, _i, _i, _i, _i, _i], _i),
    "fd3d_batch_set_schedule": ([_vp, _sz], _i),
    "fd3d_batch_autotune": ([_vp, _i, ctypes.POINTER(_i), ctypes.POINTER(ctypes.c_double), _vp], _i),
    "fd3d_batch_forward": ([_vp, ctypes.POINTER(fd3d_source), ctypes.POINTER(_i), ctypes.POINTER(_dp),
                            ctypes.POINTER(_vp), _i, _i, _vp], _i),
    "fd3d_batch_grad_workspace_bytes": ([_vp, _i, ctypes.POINTER(_sz)], _i),
    "fd3d_batch_gradient": ([_vp, ctypes.POINTER(fd3d_source), ctypes.POINTER(_i), ctypes.POINTER(_dp),
                             ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                             ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_sz), _i, _i,
                             _vp, _sz, _vp], _i),
    "fd3d_batch_destroy": ([_vp], None),
    "fd3d_autotune": ([_vp, _i, ctypes.POINTER(fd3d_kernel), _dp, _vp], _i),
    "fd3d_set_kernel": ([_vp, ctypes.POINTER(fd3d_kernel)], _i),
    "fd3d_get_kernel": ([_vp, ctypes.POINTER(fd3d_kernel)], _i),
    "fd3d_profile": ([_vp, _i], _i),
    "fd3d_profile_read": ([_vp, _dp, ctypes.POINTER(_i)], _i),
    "fd3d_upsample": ([_vp, _i, _i, _i, _vp, _i, _i, _i, _i, _vp], _i),
    "fd3d_forward_static": ([_i, _i, _i, _vp, _vp, _vp, _d, _d, _i, ctypes.POINTER(fd3d_opts),
                             ctypes.POINTER(fd3d_source), _i, _dp, _vp, ctypes.POINTER(_vp), _vp], _i),
    "fd3d_destroy": ([_vp], None),
}

for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res


def exported_symbols():
    """Names this binding resolves in the library."""
    return list(_SIGS)


def _check(rc: int):
    if rc != FD3D_OK:
        raise FD3DError(rc, _lib.fd3d_last_error().decode())


def fd3d_version() -> str:
    return _lib.fd3d_version().decode()


def fd3d_last_error() -> str:
    return _lib.fd3d_last_error().decode()


def fd3d_workspace_bytes(nx: int, ny: int, nz: int, opts: fd3d_opts | None) -> int:
    out = _sz(0)
    _check(_lib.fd3d_workspace_bytes(nx, ny, nz, ctypes.byref(opts) if opts is not None else None, ctypes.byref(out)))
    return int(out.value)


def fd3d_create(nx, ny, nz, lam, mu, rho, dx, dt, nt, opts, workspace, ws_bytes, stream) -> int:
    ctx = _vp(0)
    _check(_lib.fd3d_create(ctypes.byref(ctx), nx, ny, nz, lam, mu, rho, float(dx), float(dt), int(nt),
                            ctypes.byref(opts) if opts is not None else None, workspace, ws_bytes, stream))
    return int(ctx.value)


def fd3d_forward(ctx, src: fd3d_source | None, nrec: int, rec_pos_ptr, traces, flags: int, stream) -> None:
    _check(_lib.fd3d_forward(ctx, ctypes.byref(src) if src is not None else None, nrec,
                             ctypes.cast(rec_pos_ptr, _dp) if rec_pos_ptr else None, traces, flags, stream))


def _ptr9(fields):
    arr = (_vp * 9)(*[int(p) for p in fields])
    return arr


def fd3d_get_state(ctx, fields, stream) -> None:
    _check(_lib.fd3d_get_state(ctx, _ptr9(fields), stream))


def fd3d_set_state(ctx, fields, stream) -> None:
    _check(_lib.fd3d_set_state(ctx, _ptr9(fields), stream))


def fd3d_model_info(ctx):
    out = (ctypes.c_double * 4)()
    _check(_lib.fd3d_model_info(ctx, out))
    return list(out)


def fd3d_get_layout(ctx) -> int:
    out = ctypes.c_int(0)
    _check(_lib.fd3d_get_layout(ctx, ctypes.byref(out)))
    return out.value


def _src(src):
    return ctypes.byref(src) if src is not None else None


def _dpp(p):
    return ctypes.cast(p, _dp) if p else None


def fd3d_grad_workspace_bytes(ctx, ckpt_every: int) -> int:
    out = _sz(0)
    _check(_lib.fd3d_grad_workspace_bytes(ctx, int(ckpt_every), ctypes.byref(out)))
    return int(out.value)


def fd3d_forward_ckpt(ctx, src, nrec, rec_pos_ptr, traces, flags, gws, gws_bytes, ckpt_every, stream) -> None:
    _check(_lib.fd3d_forward_ckpt(ctx, _src(src), nrec, _dpp(rec_pos_ptr), traces, flags, gws, gws_bytes,
                                  int(ckpt_every), stream))


def fd3d_adjoint(ctx, src, nrec, rec_pos_ptr, residual, g_lam, g_mu, g_rho, gws, gws_bytes, stream) -> None:
    _check(_lib.fd3d_adjoint(ctx, _src(src), nrec, _dpp(rec_pos_ptr), residual, g_lam, g_mu, g_rho, gws, gws_bytes,
                             stream))


def fd3d_gradient(ctx, src, nrec, rec_pos_ptr, d_obs, traces, misfit, g_lam, g_mu, g_rho, gws, gws_bytes,
                  ckpt_every, stream) -> None:
    _check(_lib.fd3d_gradient(ctx, _src(src), nrec, _dpp(rec_pos_ptr), d_obs, traces, misfit, g_lam, g_mu, g_rho,
                              gws, gws_bytes, int(ckpt_every), stream))


def fd3d_born(ctx, dctx, src, dlam, dmu, drho, nrec, rec_pos_ptr, traces, dtraces, stream) -> None:
    _check(_lib.fd3d_born(ctx, dctx, _src(src), dlam, dmu, drho, nrec, _dpp(rec_pos_ptr), traces, dtraces, stream))


def fd3d_get_adjoint_state(ctx, gws, fields, stream) -> None:
    _check(_lib.fd3d_get_adjoint_state(ctx, gws, _ptr9(fields), stream))


def fd3d_batch_workspace_bytes(ctxs) -> int:
    arr = (_vp * len(ctxs))(*ctxs)
    out = _sz(0)
    _check(_lib.fd3d_batch_workspace_bytes(len(ctxs), arr, ctypes.byref(out)))
    return int(out.value)


def fd3d_batch_create(ctxs, workspace, ws_bytes) -> int:
    arr = (_vp * len(ctxs))(*ctxs)
    b = _vp(0)
    _check(_lib.fd3d_batch_create(ctypes.byref(b), len(ctxs), arr, workspace, ws_bytes))
    return int(b.value)


def fd3d_batch_set_kernel(batch, tile_x: int, tile_y: int, workgroups: int = 0) -> None:
    _check(_lib.fd3d_batch_set_kernel(batch, int(tile_x), int(tile_y), int(workgroups)))


def fd3d_batch_set_tiles(batch, tile_x: int, tile_y: int, tile2_x: int = 0, tile2_y: int = 0,
                         workgroups: int = 0) -> None:
    _check(_lib.fd3d_batch_set_tiles(batch, int(tile_x), int(tile_y), int(tile2_x), int(tile2_y), int(workgroups)))


def fd3d_batch_set_schedule(batch, group_bytes: int) -> None:
    _check(_lib.fd3d_batch_set_schedule(batch, int(group_bytes)))


def fd3d_batch_autotune(batch, steps: int, stream):
    best = (_i * 6)()
    ms = ctypes.c_double(0.0)
    _check(_lib.fd3d_batch_autotune(batch, int(steps), best, ctypes.byref(ms), stream))
    return dict(tile_x=best[0], tile_y=best[1], tile2_x=best[2], tile2_y=best[3], workgroups=best[4],
                group_mib=best[5], ms_per_step=ms.value)


def fd3d_batch_forward(batch, srcs, nrec, rec_ptrs, traces, flags, use_graph, stream) -> None:
    """srcs: list of fd3d_source (or None); nrec: list of int; rec_ptrs: host addresses of
    double[nrec][3]; traces: device addresses of T[nrec][3][nt]."""
    n = len(nrec)
    sarr = (fd3d_source * n)(*srcs) if srcs is not None else None
    narr = (_i * n)(*nrec)
    rarr = (_dp * n)(*[ctypes.cast(p, _dp) if p else None for p in rec_ptrs])
    tarr = (_vp * n)(*traces)
    _check(_lib.fd3d_batch_forward(batch, sarr, narr, rarr, tarr, int(flags), int(bool(use_graph)), stream))


def fd3d_batch_grad_workspace_bytes(batch, ckpt_every: int) -> int:
    out = _sz(0)
    _check(_lib.fd3d_batch_grad_workspace_bytes(batch, int(ckpt_every), ctypes.byref(out)))
    return int(out.value)


def fd3d_batch_gradient(batch, srcs, nrec, rec_ptrs, d_obs, traces, misfit, g_lam, g_mu, g_rho, gws, gws_bytes,
                        ckpt_every, flags, bws, bws_bytes, stream) -> None:
    n = len(nrec)
    vp = lambda xs: (_vp * n)(*xs)
    _check(_lib.fd3d_batch_gradient(batch, (fd3d_source * n)(*srcs), (_i * n)(*nrec),
                                    (_dp * n)(*[ctypes.cast(p, _dp) for p in rec_ptrs]), vp(d_obs), vp(traces),
                                    vp(misfit), vp(g_lam), vp(g_mu), vp(g_rho), vp(gws), (_sz * n)(*gws_bytes),
                                    int(ckpt_every), int(flags), bws, bws_bytes, stream))


def fd3d_batch_destroy(batch) -> None:
    _lib.fd3d_batch_destroy(batch)


def fd3d_autotune(ctx, steps: int, stream):
    k = fd3d_kernel()
    ms = ctypes.c_double(0.0)
    _check(_lib.fd3d_autotune(ctx, int(steps), ctypes.byref(k), ctypes.byref(ms), stream))
    return k, float(ms.value)


def fd3d_set_kernel(ctx, k: fd3d_kernel) -> None:
    _check(_lib.fd3d_set_kernel(ctx, ctypes.byref(k)))


def fd3d_get_kernel(ctx) -> fd3d_kernel:
    k = fd3d_kernel()
    _check(_lib.fd3d_get_kernel(ctx, ctypes.byref(k)))
    return k


def fd3d_profile(ctx, enable: bool) -> None:
    _check(_lib.fd3d_profile(ctx, int(bool(enable))))


def fd3d_profile_read(ctx):
    """Summed ms and launch counts per pass (velocity, record, stress, fused step) of the
    last call."""
    ms = (ctypes.c_double * 4)()
    n = (ctypes.c_int * 4)()
    _check(_lib.fd3d_profile_read(ctx, ms, n))
    return list(ms), list(n)


def fd3d_destroy(ctx) -> None:
    _lib.fd3d_destroy(ctx)


def fd3d_upsample(coarse_ptr, mshape, fine_ptr, nshape, dtype_code: int, stream) -> None:
    """mshape, nshape: (x, y, z) sizes of the coarse and the simulation grid."""
    _check(_lib.fd3d_upsample(coarse_ptr, int(mshape[0]), int(mshape[1]), int(mshape[2]), fine_ptr,
                              int(nshape[0]), int(nshape[1]), int(nshape[2]), int(dtype_code), stream))


def fd3d_forward_static(shape, lam, mu, rho, dx: float, dt: float, nt: int, opts: fd3d_opts | None,
                        src: fd3d_source | None, nrec: int, rec_pos_ptr, traces, final_state, stream) -> None:
    """shape: (nx, ny, nz); final_state: 9 device pointers or None."""
    fs = _ptr9(final_state) if final_state is not None else None
    _check(_lib.fd3d_forward_static(int(shape[0]), int(shape[1]), int(shape[2]), lam, mu, rho, float(dx), float(dt),
                                    int(nt), ctypes.byref(opts) if opts is not None else None,
                                    ctypes.byref(src) if src is not None else None, int(nrec),
                                    ctypes.cast(rec_pos_ptr, _dp) if rec_pos_ptr else None, traces, fs, stream))
