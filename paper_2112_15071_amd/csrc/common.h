// Shared device-side definitions of the fd3d HIP library (gfx950).
//
// Field order, staggering (Sec. 2.1.1), the Eq.(4) weights and the kernel
// parameter blocks used by every pass.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fd3d {

enum Field { VX = 0, VY, VZ, SXX, SYY, SZZ, SXY, SXZ, SYZ, NFIELD };

// Half-offset flags (x, y, z) of each component, Sec. 2.1.1.
__host__ __device__ constexpr int stag(int c, int axis)
{
    return (c == VX) ? (axis == 0)
         : (c == VY) ? (axis == 1)
         : (c == VZ) ? (axis == 2)
         : (c == SXY) ? (axis != 2)
         : (c == SXZ) ? (axis != 1)
         : (c == SYZ) ? (axis != 0)
         : 0;
}

// Eq.(4): weights of f(x+1/2)-f(x-1/2) and f(x+3/2)-f(x-3/2).
template <typename T> __host__ __device__ constexpr T c1() { return T(9.0 / 8.0); }
template <typename T> __host__ __device__ constexpr T c2() { return T(-1.0 / 24.0); }

// Staggered derivative from the two differences of Eq.(4), times the reciprocal spacing
// of the derivative's axis.
template <typename T>
__device__ __forceinline__ T dstag(T near_hi, T near_lo, T far_hi, T far_lo, T rd)
{
    return (c1<T>() * (near_hi - near_lo) + c2<T>() * (far_hi - far_lo)) * rd;
}

// Everything a pass needs about one grid.  Arrays are x-fastest, unpadded.
template <typename T> struct Grid {
    int nx, ny, nz;
    long sy, sz;           // strides of y and z (nx, nx*ny)
    T dt, rdx, rdy, rdz;   // time step and 1/dx, 1/dy, 1/dz
    const T *lam, *mu, *rho;
    T *f[NFIELD];
    const T *g[3][2];      // damping profile per axis at integer [0] / half [1] positions
    T *save[NFIELD];       // gradient recompute: where the velocity pass writes v^{n+1/2}
                           // (save[VX..VZ]; the others unused)
    int ks;                // vacuum surface: first solid node plane (0: no vacuum)
    const int *ksmap;      // optional first solid plane per node column [ny][nx] (topography)
    int cm[3];             // coarse medium: lam, mu, rho hold (mx, my, mz) nodes (cm[0] = 0: node arrays)
    T cs[3];               // (m - 1) / (n - 1) per axis: coarse coordinate per grid unit
};

// Coarse medium (Sec. 2.2.1: the medium textures may be smaller than the simulation grid,
// every read a trilinear sample).  The coarse node grid spans the same box as the
// simulation grid, so coordinate x (grid units, integer or half-integer) sits at coarse
// coordinate X = x (m - 1) / (n - 1); a medium value is the trilinear interpolation of the
// eight coarse nodes around the value's own position.  Per axis: the lower coarse node and
// the weight of the upper one (m >= 2; positions past the last node extrapolate from the
// last cell, which only pinned samples reach).
template <typename T> struct CoarseAxis {
    int lo;
    T f;
};

template <typename T> __device__ __forceinline__ CoarseAxis<T> coarse_axis(T x, T scale, int m)
{
    const T X = x * scale;
    const int b = (int)X;  // X >= 0
    const int lo = b < m - 2 ? b : m - 2;
    return {lo, X - (T)lo};
}

// Bilinear sample of coarse plane kc at the column (ax, ay) of a coarse array with mx
// nodes per row and mxy per plane.
template <typename T>
__device__ __forceinline__ T coarse_bil(const T *a, int mx, int mxy, const CoarseAxis<T> &ax,
                                        const CoarseAxis<T> &ay, int kc)
{
    const T *p = a + (long)kc * mxy + (long)ay.lo * mx + ax.lo;
    const T lo = (T(1) - ax.f) * p[0] + ax.f * p[1];
    const T hi = (T(1) - ax.f) * p[mx] + ax.f * p[mx + 1];
    return (T(1) - ay.f) * lo + ay.f * hi;
}

template <typename T> __device__ __forceinline__ T lerp_w(T a, T b, T f) { return (T(1) - f) * a + f * b; }

// Reciprocal of a sampled density (FP32: the hardware reciprocal, as buoy).
__device__ __forceinline__ float rcp_rho(float r) { return __builtin_amdgcn_rcpf(r); }
__device__ __forceinline__ double rcp_rho(double r) { return 1.0 / r; }

// First solid planes seen by the samples of column (i, j): at the node, and between
// columns i, i+1 (x half positions) and rows j, j+1 (y half positions), where a sample
// takes the deepest plane of the columns beside it.
struct SurfacePlanes {
    int n, x, y;
};
template <typename T>
__device__ __forceinline__ SurfacePlanes surface_planes(const Grid<T> &G, int i, int j)
{
    if (!G.ksmap || i >= G.nx || j >= G.ny) return {G.ks, G.ks, G.ks};
    const int a = G.ksmap[i + G.nx * j];
    const int b = G.ksmap[(i + 1 < G.nx ? i + 1 : i) + G.nx * j];
    const int c = G.ksmap[i + G.nx * (j + 1 < G.ny ? j + 1 : j)];
    return {a, a > b ? a : b, a > c ? a : c};
}

// Vacuum surface (Sec. 2.5): z derivatives whose result lies within one cell of the first
// solid plane ks take the second-order difference -- results at integer planes
// ks - 1 .. ks + 1 and at half planes ks - 1/2, ks + 1/2 (k = ks - 1, ks).
__host__ __device__ __forceinline__ bool o2_int(int ks, int k) { return ks > 0 && (unsigned)(k - ks + 1) <= 2u; }
__host__ __device__ __forceinline__ bool o2_half(int ks, int k) { return ks > 0 && (unsigned)(k - ks + 1) <= 1u; }

// z derivative of Eq.(4) from the queue q (q[1], q[2] the near pair), or its second-order
// form next to a vacuum surface.
template <typename T>
__device__ __forceinline__ T dz_or_o2(bool o2, T near_hi, T near_lo, T far_hi, T far_lo, T rdz)
{
    return o2 ? (near_hi - near_lo) * rdz : dstag(near_hi, near_lo, far_hi, far_lo, rdz);
}

// A point source as kernel argument: per component, the base of its 2x2x2 tap box
// on that component's subgrid, and in device memory the eight coefficients per
// component (x fastest, then y, z), read only where a tap lies.
// Velocity components: dt w F / dx^3 (times b and s[n] in the kernel).
// Stress components:  -dt w M / dx^3 (times s[n] in the kernel).
template <typename T> struct Inject {
    int on;
    int i0[NFIELD], j0[NFIELD], k0[NFIELD];
    const T *coef;  // [NFIELD][8]
    const T *wavelet;
};

// One receiver component: eight storage indices (-1: none) and trilinear weights.
template <typename T> struct RecTap {
    int idx[8];
    T w[8];
};

// Largest number of shots in one batched launch (per-workgroup LDS table of shot bases).
constexpr int kMaxShots = 256;

// Per-workgroup copy of the shots' first work items; the shot of item w is then found
// in LDS and made wave-uniform, so the shot's descriptor is read through scalar loads.
__device__ __forceinline__ void load_bases(int *s_base, const int *base, int stride_ints, int nshot)
{
    for (int s = threadIdx.x; s < nshot; s += blockDim.x) s_base[s] = base[(long)s * stride_ints];
    __syncthreads();
}

__device__ __forceinline__ int shot_of(const int *s_base, int nshot, int w)
{
    int s = 0;
    while (s + 1 < nshot && s_base[s + 1] <= w) ++s;
    return __builtin_amdgcn_readfirstlane(s);
}

// Effective buoyancy between two density samples, 1 / ((a + b) / 2) (Sec. 2.2.1).  FP32
// uses the hardware reciprocal (within 1 ulp); FP64 the correctly rounded division.
__device__ __forceinline__ float buoy(float a, float b) { return __builtin_amdgcn_rcpf((a + b) * 0.5f); }
__device__ __forceinline__ double buoy(double a, double b) { return 1.0 / ((a + b) * 0.5); }

// True when some tap of source component c lies in the box [i0, i1) x [j0, j1) x [k0, k1).
template <typename T>
__device__ __forceinline__ bool taps_in(const Inject<T> &s, int c, int i0, int i1, int j0, int j1, int k0, int k1)
{
    return s.i0[c] + 1 >= i0 && s.i0[c] < i1 && s.j0[c] + 1 >= j0 && s.j0[c] < j1 && s.k0[c] + 1 >= k0 &&
           s.k0[c] < k1;
}

// Coefficient of tap t (-1: none) of source component c.
template <typename T> __device__ __forceinline__ T coef_of(const Inject<T> &s, int c, int t)
{
    return t >= 0 ? s.coef[c * 8 + t] : T(0);
}

// Tap number of (i,j,k) in a source box, or -1.
template <typename T>
__device__ __forceinline__ int tap_of(const Inject<T> &s, int c, int i, int j, int k)
{
    unsigned a = (unsigned)(i - s.i0[c]), b = (unsigned)(j - s.j0[c]), d = (unsigned)(k - s.k0[c]);
    return (a < 2u && b < 2u && d < 2u) ? (int)(a + 2u * b + 4u * d) : -1;
}

} // namespace fd3d
