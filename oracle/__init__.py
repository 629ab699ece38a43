"""FP64 CPU oracle of the staggered-grid elastic velocity-stress scheme.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code with
the HIP library (``paper_2112_15071_amd``) and never imports it.

The arithmetic lives in ``fd3d_oracle.c`` (plain loops, OpenMP over z); this module
only marshals numpy arrays.  Arrays are float64, C-contiguous, shaped
``[nz, ny, nx]`` (x fastest).  The state is ``[9, nz, ny, nx]`` in the order
vx, vy, vz, sxx, syy, szz, sxy, sxz, syz.

Paper passages (arXiv 2112.15071): Sec. 2.1 Eq.(1)-(3) (equations), Sec. 2.1.1
(staggering), Eq.(4) (stencil), Sec. 2.2 (in-place update), Sec. 2.2.1 (effective
parameters), Sec. 2.4 (receivers), Sec. 2.5 (damping, free surface).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fd3d_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FIELDS = ("vx", "vy", "vz", "sxx", "syy", "szz", "sxy", "sxz", "syz")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int * 3),
        ("h", ctypes.c_double * 3),
        ("dt", ctypes.c_double),
        ("nt", ctypes.c_int),
        ("periodic", ctypes.c_int * 3),
        ("free_surface", ctypes.c_int),
        ("vacuum_top", ctypes.c_int),
        ("vacuum_map", ctypes.POINTER(ctypes.c_int)),
        ("sponge", ctypes.c_int * 6),
        ("alpha", ctypes.c_double),
        ("coarse", ctypes.c_int * 3),
    ]


class _Src(ctypes.Structure):
    _fields_ = [
        ("pos", ctypes.c_double * 3),
        ("moment", ctypes.c_double * 6),
        ("force", ctypes.c_double * 3),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_forward.argtypes = [
            ctypes.POINTER(_Cfg), dp, dp, dp, ctypes.POINTER(_Src), dp, ctypes.c_int, dp, dp, dp, ctypes.c_int,
        ]
        lib.oracle_forward.restype = ctypes.c_int
        lib.oracle_gradient.argtypes = [
            ctypes.POINTER(_Cfg), dp, dp, dp, ctypes.POINTER(_Src), dp, ctypes.c_int, dp, dp, dp, dp, dp, dp, dp,
        ]
        lib.oracle_gradient.restype = ctypes.c_int
        lib.oracle_born.argtypes = [
            ctypes.POINTER(_Cfg), dp, dp, dp, dp, dp, dp, ctypes.POINTER(_Src), dp, ctypes.c_int, dp, dp, dp,
        ]
        lib.oracle_born.restype = ctypes.c_int
        lib.oracle_profiles.argtypes = [ctypes.POINTER(_Cfg), dp]
        lib.oracle_medium.argtypes = [ctypes.POINTER(_Cfg), dp, dp, dp, dp]
        lib.oracle_medium.restype = ctypes.c_int
        lib.oracle_deriv1d.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, dp, dp]
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_get_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class Config:
    """Grid and scheme options.  ``shape`` is (nx, ny, nz); ``h`` is one spacing for all
    axes or (dx, dy, dz)."""

    shape: Sequence[int]
    h: object
    dt: float
    nt: int
    sponge: Sequence[int] = (0, 0, 0, 0, 0, 0)  # x-, x+, y-, y+, z- (top), z+
    alpha: float = 0.0  # <= 0: 0.3 / width per face
    free_surface: bool = False
    periodic: Sequence[bool] = (False, False, False)
    vacuum_top: int = 0  # > 0: vacuum formulation, first solid node plane
    vacuum_map: Optional[np.ndarray] = None  # [ny, nx] first solid plane per column (topography)
    # (mx, my, mz): the medium arrays are a coarse node grid over the same box, sampled
    # trilinearly at every value's own position (Sec. 2.2.1); None: node arrays
    coarse: Optional[Sequence[int]] = None

    def _c(self) -> _Cfg:
        c = _Cfg()
        for a in range(3):
            c.n[a] = int(self.shape[a])
            c.periodic[a] = int(bool(self.periodic[a]))
        hs = tuple(self.h) if np.ndim(self.h) else (self.h,) * 3
        for a in range(3):
            c.h[a] = float(hs[a])
        c.dt = float(self.dt)
        c.nt = int(self.nt)
        c.free_surface = int(bool(self.free_surface))
        c.vacuum_top = int(self.vacuum_top)
        if self.vacuum_map is not None:
            nx, ny = int(self.shape[0]), int(self.shape[1])
            m = np.ascontiguousarray(np.asarray(self.vacuum_map, dtype=np.int32))
            if m.shape != (ny, nx):
                raise ValueError("vacuum_map must be [ny, nx]")
            self._map_keep = m  # referenced by the struct for the call
            c.vacuum_map = m.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        sp = list(self.sponge)
        if len(sp) == 1:
            sp = sp * 6
        for f in range(6):
            c.sponge[f] = int(sp[f])
        c.alpha = float(self.alpha)
        if self.coarse is not None:
            for a in range(3):
                c.coarse[a] = int(self.coarse[a])
        return c

    @property
    def medium_zyx(self):
        """Shape of the medium arrays: the coarse grid's, or the simulation grid's."""
        if self.coarse is None:
            return self.zyx
        mx, my, mz = (int(v) for v in self.coarse)
        return (mz, my, mx)

    @property
    def zyx(self):
        nx, ny, nz = (int(v) for v in self.shape)
        return (nz, ny, nx)


@dataclass
class Source:
    """Point source at ``pos`` (grid units, x y z)."""

    pos: Sequence[float]
    moment: Sequence[float] = (0.0,) * 6  # Mxx Myy Mzz Mxy Mxz Myz
    force: Sequence[float] = (0.0,) * 3

    def _c(self) -> _Src:
        s = _Src()
        for a in range(3):
            s.pos[a] = float(self.pos[a])
            s.force[a] = float(self.force[a])
        for q in range(6):
            s.moment[q] = float(self.moment[q])
        return s


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None and a.shape != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {a.shape}")
    return a


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(_load().oracle_get_threads())


def forward(cfg: Config, lam, mu, rho, src: Optional[Source] = None, wavelet=None, rec_pos=None,
            state=None):
    """Run ``cfg.nt`` steps.  Returns (traces [nrec,3,nt], state [9,nz,ny,nx]).

    ``state`` (optional) is the initial (v^{-1/2}, sigma^0); zero when omitted.
    """
    lib = _load()
    zyx = cfg.zyx
    lam, mu, rho = (_f64(a, cfg.medium_zyx) for a in (lam, mu, rho))
    wav = None if wavelet is None else _f64(wavelet, (cfg.nt,))
    rp = np.zeros((0, 3)) if rec_pos is None else _f64(rec_pos)
    rp = rp.reshape(-1, 3)
    nrec = rp.shape[0]
    traces = np.zeros((nrec, 3, cfg.nt))
    st = np.zeros((9,) + zyx) if state is None else _f64(state, (9,) + zyx).copy()
    c = cfg._c()
    s = src._c() if src is not None else None
    rc = lib.oracle_forward(ctypes.byref(c), _ptr(lam), _ptr(mu), _ptr(rho),
                            ctypes.byref(s) if s is not None else None, _ptr(wav), nrec, _ptr(rp),
                            _ptr(traces), _ptr(st), int(state is not None))
    if rc:
        raise ValueError(f"oracle_forward failed ({rc})")
    return traces, st


def gradient(cfg: Config, lam, mu, rho, src: Optional[Source], wavelet, rec_pos, residual, state0=None):
    """Exact discrete adjoint (store-all).  Returns (g_lam, g_mu, g_rho, adj_state).

    ``residual`` is dJ/dd [nrec,3,nt]; ``adj_state`` is the adjoint of the initial
    state [9,nz,ny,nx].  Small grids only (every step is stored).
    """
    lib = _load()
    zyx = cfg.zyx
    lam, mu, rho = (_f64(a, zyx) for a in (lam, mu, rho))
    wav = None if wavelet is None else _f64(wavelet, (cfg.nt,))
    rp = _f64(rec_pos).reshape(-1, 3)
    nrec = rp.shape[0]
    res = _f64(residual, (nrec, 3, cfg.nt))
    s0 = None if state0 is None else _f64(state0, (9,) + zyx)
    gl, gm, gr = (np.zeros(zyx) for _ in range(3))
    adj = np.zeros((9,) + zyx)
    c = cfg._c()
    s = src._c() if src is not None else None
    rc = lib.oracle_gradient(ctypes.byref(c), _ptr(lam), _ptr(mu), _ptr(rho),
                             ctypes.byref(s) if s is not None else None, _ptr(wav), nrec, _ptr(rp),
                             _ptr(res), _ptr(s0), _ptr(gl), _ptr(gm), _ptr(gr), _ptr(adj))
    if rc:
        raise ValueError(f"oracle_gradient failed ({rc})")
    return gl, gm, gr, adj


def born(cfg: Config, lam, mu, rho, dlam, dmu, drho, src: Optional[Source], wavelet, rec_pos):
    """Tangent-linear (Born) forward: (traces, dtraces) [nrec,3,nt], the background traces
    and their derivative along the model perturbation (dlam, dmu, drho).  No free surface."""
    lib = _load()
    zyx = cfg.zyx
    arrs = [_f64(a, zyx) for a in (lam, mu, rho, dlam, dmu, drho)]
    wav = None if wavelet is None else _f64(wavelet, (cfg.nt,))
    rp = _f64(rec_pos).reshape(-1, 3)
    nrec = rp.shape[0]
    tr = np.zeros((nrec, 3, cfg.nt))
    dtr = np.zeros((nrec, 3, cfg.nt))
    c = cfg._c()
    s = src._c() if src is not None else None
    rc = lib.oracle_born(ctypes.byref(c), *(_ptr(a) for a in arrs), ctypes.byref(s) if s is not None else None,
                         _ptr(wav), nrec, _ptr(rp), _ptr(tr), _ptr(dtr))
    if rc:
        raise ValueError(f"oracle_born failed ({rc})")
    return tr, dtr


def profiles(cfg: Config):
    """Damping profiles {(axis, half): array} as the oracle builds them."""
    lib = _load()
    n = [int(v) for v in cfg.shape]
    out = np.zeros(2 * sum(n))
    lib.oracle_profiles(ctypes.byref(cfg._c()), _ptr(out))
    res, off = {}, 0
    for ax in range(3):
        for half in range(2):
            res[(ax, half)] = out[off:off + n[ax]].copy()
            off += n[ax]
    return res


def deriv1d(f, h: float, plus: bool) -> np.ndarray:
    """Eq.(4) on a 1D line: plus -> integer to half points; else half to integer."""
    lib = _load()
    f = _f64(f)
    out = np.zeros_like(f)
    lib.oracle_deriv1d(f.size, float(h), int(bool(plus)), _ptr(f), _ptr(out))
    return out


def misfit(traces, d_obs) -> float:
    """J = 1/2 sum (d - d_obs)^2 (no dt weighting)."""
    r = np.asarray(traces) - np.asarray(d_obs)
    return 0.5 * float(np.sum(r * r))


MEDIUM = ("rho_vx", "rho_vy", "rho_vz", "lam", "mu", "mu_xy", "mu_xz", "mu_yz")


def medium(cfg: Config, lam, mu, rho) -> np.ndarray:
    """The medium values the scheme uses (Sec. 2.2.1), [8, nz, ny, nx] in the order of
    MEDIUM: rho at the three velocity samples, lambda and mu at the nodes, mu at the three
    shear samples (zero at pinned samples); node means of node arrays, or trilinear samples
    of a coarse grid when ``cfg.coarse`` is set."""
    lib = _load()
    lam, mu, rho = (_f64(a, cfg.medium_zyx) for a in (lam, mu, rho))
    out = np.zeros((8,) + cfg.zyx)
    if lib.oracle_medium(ctypes.byref(cfg._c()), _ptr(lam), _ptr(mu), _ptr(rho), _ptr(out)):
        raise ValueError("oracle_medium failed")
    return out


def upsample(coarse, shape) -> np.ndarray:
    """Medium parameters given on a coarse node grid, sampled trilinearly at the nodes of
    the simulation grid (Sec. 2.2.1: the medium textures may be smaller than the
    simulation grid; every read is a trilinear sample).  ``coarse`` is [mz, my, mx],
    ``shape`` the simulation grid (nx, ny, nz); both grids span the same box, corner node
    to corner node, so fine node i sits at coarse coordinate i (m - 1) / (n - 1).
    Written out per axis as the textbook formula, no library interpolator."""
    c = _f64(coarse)
    mz, my, mx = c.shape
    nx, ny, nz = (int(v) for v in shape)

    def axis(n, m):
        """Lower coarse index and weight of the upper one for each fine node."""
        q = np.arange(n) * ((m - 1) / (n - 1)) if n > 1 else np.zeros(1)
        lo = np.minimum(np.floor(q).astype(np.int64), max(m - 2, 0))
        return lo, q - lo

    (ix, wx), (iy, wy), (iz, wz) = axis(nx, mx), axis(ny, my), axis(nz, mz)
    ix1, iy1, iz1 = np.minimum(ix + 1, mx - 1), np.minimum(iy + 1, my - 1), np.minimum(iz + 1, mz - 1)
    out = np.zeros((nz, ny, nx))
    for k in range(nz):
        for dz, fz in ((iz[k], 1.0 - wz[k]), (iz1[k], wz[k])):
            for dy, fy in ((iy, 1.0 - wy), (iy1, wy)):
                for dx, fx in ((ix, 1.0 - wx), (ix1, wx)):
                    out[k] += fz * fy[:, None] * fx[None, :] * c[dz][np.ix_(dy, dx)]
    return out
