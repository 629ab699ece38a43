// Discrete adjoint of one step (velocity pass, receiver sampling, stress pass) and the
// chain rule to the node arrays lambda, mu, rho.  One thread per cell.
//
// Adjoint arrays (same layout as the state): A_v (3 components), A_s (6).  Each pass
// applies its damping factor lazily, so that no pass rewrites an array that a
// neighbouring thread still reads:
//   start of step n:  adjoint(sigma^{n+1}) = A_s,  adjoint(v^{n+1/2}) so far = G_v A_v
//   adj_stress:  T = G_s A_s;  A_v <- G_v A_v - dt D_S(C T);  gradients of C from E v^{n+1/2}
//   residual:    A_v += W^T r^n
//   adj_vel:     U = G_v A_v;  A_s <- G_s A_s - dt E(b U);  gradient of b
// leaving adjoint(sigma^n) = A_s and adjoint(v^{n-1/2}) = G_v A_v.  D_S is the
// divergence stencil of the velocity pass and E the strain-rate stencil of the stress
// pass; under the zero-halo rules D_S = -E^T, so these are the transposed passes.
//
// The gradient of b needs, at each velocity sample, U times the step's increment over b,
// dt D_S sigma^n + c s (c the force source's coefficient), which the velocity pass
// multiplied by b, added to v^{n-1/2} and damped: v^{n+1/2} = G_v (v^{n-1/2} + b (...)).
// With U = G_v A_v that product is A_v (v^{n+1/2} - G_v v^{n-1/2}) rho_eff, formed from
// the two stored velocities, so the segment recompute stores v^{n+1/2} only (not sigma^n).
//
// The tiled adjoint (velocity-type and stress-type tile bodies) keeps, in place of A_v,
// Y = b G_v A_v, the field its adjoint stress pass reads: its velocity pass forms A_v from
// the Y of the step after (G_v A_v = Y rho_eff), its share of the gradient of b and the
// new Y in one sweep, and its residual injection adds the injected share to Y and g_b at
// the taps.  Its gradient of b is the same sum taken by parts over the steps: with
// A_v^n = G_v A_v^{n+1} + r^n - dt D_S X^n (r^n the injected residual),
//   sum_n A_v^n (v^{n+1/2} - G_v v^{n-1/2}) rho_eff
//     = sum_n v^{n+1/2} rho_eff (r^n - dt D_S X^n) - v^{-1/2} rho_eff G_v A_v^0,
// which needs v^{n+1/2} alone; the last term (the initial velocity, zero unless the
// forward started from a given state) is added once at the end of the sweep.
#pragma once

#include "common.h"

namespace fd3d {

// Adjoint of one grid: adjoint state, gradient accumulators at staggered points and the
// stored forward fields of the step being reversed.
template <typename T> struct AdjGrid {
    T *a[NFIELD];      // A_v, A_s
    T *gl, *gm;        // lambda, mu at nodes (normal-stress part)
    T *gs[3];          // mu_xy, mu_xz, mu_yz at the shear-stress points
    T *gb[3];          // buoyancy at vx, vy, vz points
    const T *vst[3];   // stored v^{n+1/2}
    const T *vprev[3]; // stored v^{n-1/2}
};

template <typename T>
__device__ __forceinline__ T rdc(const T *f, int c, int i, int j, int k, const Grid<T> &G)
{
    const int lx = G.nx - 1 - stag(c, 0), ly = G.ny - 1 - stag(c, 1), lz = G.nz - 1 - stag(c, 2);
    const bool ok = (unsigned)i <= (unsigned)lx && (unsigned)j <= (unsigned)ly && (unsigned)k <= (unsigned)lz;
    return ok ? f[i + G.sy * j + G.sz * k] : T(0);
}

template <typename T> __device__ __forceinline__ T damp(const Grid<T> &G, int c, int i, int j, int k)
{
    return G.g[0][stag(c, 0)][i] * G.g[1][stag(c, 1)][j] * G.g[2][stag(c, 2)][k];
}

template <typename T> __device__ __forceinline__ bool in_grid(const Grid<T> &G, int i, int j, int k)
{
    return (unsigned)i < (unsigned)G.nx && (unsigned)j < (unsigned)G.ny && (unsigned)k < (unsigned)G.nz;
}

// C applied to T = G_s A_s at a stress sample (zero outside the active range).
template <typename T>
__device__ __forceinline__ T xval(const Grid<T> &G, const AdjGrid<T> &A, int c, int i, int j, int k)
{
    const int lx = G.nx - 1 - stag(c, 0), ly = G.ny - 1 - stag(c, 1), lz = G.nz - 1 - stag(c, 2);
    if (!((unsigned)i <= (unsigned)lx && (unsigned)j <= (unsigned)ly && (unsigned)k <= (unsigned)lz)) return T(0);
    const long p = i + G.sy * j + G.sz * k;
    if (c <= SZZ) {
        const T g = damp(G, SXX, i, j, k);
        const T txx = g * A.a[SXX][p], tyy = g * A.a[SYY][p], tzz = g * A.a[SZZ][p];
        const T tc = c == SXX ? txx : (c == SYY ? tyy : tzz);
        return G.lam[p] * ((txx + tyy) + tzz) + T(2) * G.mu[p] * tc;
    }
    long u = 0, w = 0;
    if (c == SXY) { u = 1; w = G.sy; }
    if (c == SXZ) { u = 1; w = G.sz; }
    if (c == SYZ) { u = G.sy; w = G.sz; }
    const T me = ((G.mu[p] + G.mu[p + u]) + (G.mu[p + w] + G.mu[p + u + w])) / T(4);
    return me * (damp(G, c, i, j, k) * A.a[c][p]);
}

// (a10) adjoint of the stress pass, at the samples of node (i,j,k).
template <typename T>
__device__ __forceinline__ void adj_stress_body(const Grid<T> &G, const AdjGrid<T> &A, int i, int j, int k)
{
    const long p = i + G.sy * j + G.sz * k;
    const T rdx = G.rdx, rdy = G.rdy, rdz = G.rdz, dt = G.dt;

    // A_v <- G_v A_v - dt D_S(C T)
    if (i <= G.nx - 2) {
        const T d = dstag(xval(G, A, SXX, i + 1, j, k), xval(G, A, SXX, i, j, k), xval(G, A, SXX, i + 2, j, k), xval(G, A, SXX, i - 1, j, k), rdx)
                  + dstag(xval(G, A, SXY, i, j, k), xval(G, A, SXY, i, j - 1, k), xval(G, A, SXY, i, j + 1, k), xval(G, A, SXY, i, j - 2, k), rdy)
                  + dstag(xval(G, A, SXZ, i, j, k), xval(G, A, SXZ, i, j, k - 1), xval(G, A, SXZ, i, j, k + 1), xval(G, A, SXZ, i, j, k - 2), rdz);
        A.a[VX][p] = damp(G, VX, i, j, k) * A.a[VX][p] - dt * d;
    }
    if (j <= G.ny - 2) {
        const T d = dstag(xval(G, A, SXY, i, j, k), xval(G, A, SXY, i - 1, j, k), xval(G, A, SXY, i + 1, j, k), xval(G, A, SXY, i - 2, j, k), rdx)
                  + dstag(xval(G, A, SYY, i, j + 1, k), xval(G, A, SYY, i, j, k), xval(G, A, SYY, i, j + 2, k), xval(G, A, SYY, i, j - 1, k), rdy)
                  + dstag(xval(G, A, SYZ, i, j, k), xval(G, A, SYZ, i, j, k - 1), xval(G, A, SYZ, i, j, k + 1), xval(G, A, SYZ, i, j, k - 2), rdz);
        A.a[VY][p] = damp(G, VY, i, j, k) * A.a[VY][p] - dt * d;
    }
    if (k <= G.nz - 2) {
        const T d = dstag(xval(G, A, SXZ, i, j, k), xval(G, A, SXZ, i - 1, j, k), xval(G, A, SXZ, i + 1, j, k), xval(G, A, SXZ, i - 2, j, k), rdx)
                  + dstag(xval(G, A, SYZ, i, j, k), xval(G, A, SYZ, i, j - 1, k), xval(G, A, SYZ, i, j + 1, k), xval(G, A, SYZ, i, j - 2, k), rdy)
                  + dstag(xval(G, A, SZZ, i, j, k + 1), xval(G, A, SZZ, i, j, k), xval(G, A, SZZ, i, j, k + 2), xval(G, A, SZZ, i, j, k - 1), rdz);
        A.a[VZ][p] = damp(G, VZ, i, j, k) * A.a[VZ][p] - dt * d;
    }

    // gradients of C: strain rates of the stored v^{n+1/2} against T
    const T *vx = A.vst[0], *vy = A.vst[1], *vz = A.vst[2];
    const T exx = dstag(rdc(vx, VX, i, j, k, G), rdc(vx, VX, i - 1, j, k, G), rdc(vx, VX, i + 1, j, k, G), rdc(vx, VX, i - 2, j, k, G), rdx);
    const T eyy = dstag(rdc(vy, VY, i, j, k, G), rdc(vy, VY, i, j - 1, k, G), rdc(vy, VY, i, j + 1, k, G), rdc(vy, VY, i, j - 2, k, G), rdy);
    const T ezz = dstag(rdc(vz, VZ, i, j, k, G), rdc(vz, VZ, i, j, k - 1, G), rdc(vz, VZ, i, j, k + 1, G), rdc(vz, VZ, i, j, k - 2, G), rdz);
    const T gn = damp(G, SXX, i, j, k);
    const T txx = gn * A.a[SXX][p], tyy = gn * A.a[SYY][p], tzz = gn * A.a[SZZ][p];
    A.gl[p] += dt * ((exx + eyy) + ezz) * ((txx + tyy) + tzz);
    A.gm[p] += dt * T(2) * ((exx * txx + eyy * tyy) + ezz * tzz);
    if (i <= G.nx - 2 && j <= G.ny - 2) {
        const T e = dstag(rdc(vx, VX, i, j + 1, k, G), rdc(vx, VX, i, j, k, G), rdc(vx, VX, i, j + 2, k, G), rdc(vx, VX, i, j - 1, k, G), rdy)
                  + dstag(rdc(vy, VY, i + 1, j, k, G), rdc(vy, VY, i, j, k, G), rdc(vy, VY, i + 2, j, k, G), rdc(vy, VY, i - 1, j, k, G), rdx);
        A.gs[0][p] += dt * e * (damp(G, SXY, i, j, k) * A.a[SXY][p]);
    }
    if (i <= G.nx - 2 && k <= G.nz - 2) {
        const T e = dstag(rdc(vx, VX, i, j, k + 1, G), rdc(vx, VX, i, j, k, G), rdc(vx, VX, i, j, k + 2, G), rdc(vx, VX, i, j, k - 1, G), rdz)
                  + dstag(rdc(vz, VZ, i + 1, j, k, G), rdc(vz, VZ, i, j, k, G), rdc(vz, VZ, i + 2, j, k, G), rdc(vz, VZ, i - 1, j, k, G), rdx);
        A.gs[1][p] += dt * e * (damp(G, SXZ, i, j, k) * A.a[SXZ][p]);
    }
    if (j <= G.ny - 2 && k <= G.nz - 2) {
        const T e = dstag(rdc(vy, VY, i, j, k + 1, G), rdc(vy, VY, i, j, k, G), rdc(vy, VY, i, j, k + 2, G), rdc(vy, VY, i, j, k - 1, G), rdz)
                  + dstag(rdc(vz, VZ, i, j + 1, k, G), rdc(vz, VZ, i, j, k, G), rdc(vz, VZ, i, j + 2, k, G), rdc(vz, VZ, i, j - 1, k, G), rdy);
        A.gs[2][p] += dt * e * (damp(G, SYZ, i, j, k) * A.a[SYZ][p]);
    }
}

// b U at a velocity sample: G_v A_v / rho_eff (zero outside the active range).
template <typename T>
__device__ __forceinline__ T yval(const Grid<T> &G, const AdjGrid<T> &A, int c, int i, int j, int k)
{
    const int lx = G.nx - 1 - stag(c, 0), ly = G.ny - 1 - stag(c, 1), lz = G.nz - 1 - stag(c, 2);
    if (!((unsigned)i <= (unsigned)lx && (unsigned)j <= (unsigned)ly && (unsigned)k <= (unsigned)lz)) return T(0);
    const long p = i + G.sy * j + G.sz * k;
    const long e = c == VX ? 1 : (c == VY ? G.sy : G.sz);
    return (damp(G, c, i, j, k) * A.a[c][p]) * buoy(G.rho[p], G.rho[p + e]);
}

// Contribution of step n to the gradient of b at velocity sample c of node (i,j,k):
// A_v (v^{n+1/2} - G_v v^{n-1/2}) rho_eff (see the top of this file).
template <typename T>
__device__ __forceinline__ T gb_term(const Grid<T> &G, const AdjGrid<T> &A, int c, int i, int j, int k, long p)
{
    const long e = c == VX ? 1 : (c == VY ? G.sy : G.sz);
    const T g = damp(G, c, i, j, k);
    const T inc = A.vst[c - VX][p] - g * A.vprev[c - VX][p];
    return A.a[c][p] * (inc * ((G.rho[p] + G.rho[p + e]) * T(0.5)));
}

// (a12) adjoint of the velocity pass, at the samples of node (i,j,k).
template <typename T>
__device__ __forceinline__ void adj_vel_body(const Grid<T> &G, const AdjGrid<T> &A, int i, int j, int k)
{
    const long p = i + G.sy * j + G.sz * k;
    const T rdx = G.rdx, rdy = G.rdy, rdz = G.rdz, dt = G.dt;

    // A_s <- G_s A_s - dt E(b U)
    {
        const T gn = damp(G, SXX, i, j, k);
        const T exx = dstag(yval(G, A, VX, i, j, k), yval(G, A, VX, i - 1, j, k), yval(G, A, VX, i + 1, j, k), yval(G, A, VX, i - 2, j, k), rdx);
        const T eyy = dstag(yval(G, A, VY, i, j, k), yval(G, A, VY, i, j - 1, k), yval(G, A, VY, i, j + 1, k), yval(G, A, VY, i, j - 2, k), rdy);
        const T ezz = dstag(yval(G, A, VZ, i, j, k), yval(G, A, VZ, i, j, k - 1), yval(G, A, VZ, i, j, k + 1), yval(G, A, VZ, i, j, k - 2), rdz);
        A.a[SXX][p] = gn * A.a[SXX][p] - dt * exx;
        A.a[SYY][p] = gn * A.a[SYY][p] - dt * eyy;
        A.a[SZZ][p] = gn * A.a[SZZ][p] - dt * ezz;
    }
    if (i <= G.nx - 2 && j <= G.ny - 2) {
        const T e = dstag(yval(G, A, VX, i, j + 1, k), yval(G, A, VX, i, j, k), yval(G, A, VX, i, j + 2, k), yval(G, A, VX, i, j - 1, k), rdy)
                  + dstag(yval(G, A, VY, i + 1, j, k), yval(G, A, VY, i, j, k), yval(G, A, VY, i + 2, j, k), yval(G, A, VY, i - 1, j, k), rdx);
        A.a[SXY][p] = damp(G, SXY, i, j, k) * A.a[SXY][p] - dt * e;
    }
    if (i <= G.nx - 2 && k <= G.nz - 2) {
        const T e = dstag(yval(G, A, VX, i, j, k + 1), yval(G, A, VX, i, j, k), yval(G, A, VX, i, j, k + 2), yval(G, A, VX, i, j, k - 1), rdz)
                  + dstag(yval(G, A, VZ, i + 1, j, k), yval(G, A, VZ, i, j, k), yval(G, A, VZ, i + 2, j, k), yval(G, A, VZ, i - 1, j, k), rdx);
        A.a[SXZ][p] = damp(G, SXZ, i, j, k) * A.a[SXZ][p] - dt * e;
    }
    if (j <= G.ny - 2 && k <= G.nz - 2) {
        const T e = dstag(yval(G, A, VY, i, j, k + 1), yval(G, A, VY, i, j, k), yval(G, A, VY, i, j, k + 2), yval(G, A, VY, i, j, k - 1), rdz)
                  + dstag(yval(G, A, VZ, i, j + 1, k), yval(G, A, VZ, i, j, k), yval(G, A, VZ, i, j + 2, k), yval(G, A, VZ, i, j - 1, k), rdy);
        A.a[SYZ][p] = damp(G, SYZ, i, j, k) * A.a[SYZ][p] - dt * e;
    }

    // gradient of b at the velocity samples: U times the step's increment over b
    if (i <= G.nx - 2) A.gb[0][p] += gb_term(G, A, VX, i, j, k, p);
    if (j <= G.ny - 2) A.gb[1][p] += gb_term(G, A, VY, i, j, k, p);
    if (k <= G.nz - 2) A.gb[2][p] += gb_term(G, A, VZ, i, j, k, p);
}

// Single-grid launches of the two adjoint passes (64 x 4 threads per block, one z plane).
template <typename T> __global__ void __launch_bounds__(256) adj_stress_cell(Grid<T> G, AdjGrid<T> A)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= G.nx || j >= G.ny) return;
    adj_stress_body(G, A, i, j, (int)blockIdx.z);
}

template <typename T> __global__ void __launch_bounds__(256) adj_vel_cell(Grid<T> G, AdjGrid<T> A)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    if (i >= G.nx || j >= G.ny) return;
    adj_vel_body(G, A, i, j, (int)blockIdx.z);
}

// (a11) adjoint of the sampling for the receivers of one colour (no two of them share a
// tap): A_v[tap] += w r[r][c][n].
template <typename T>
__device__ __forceinline__ void inject_one(T *__restrict__ ax, T *__restrict__ ay, T *__restrict__ az,
                                           const RecTap<T> *__restrict__ taps, int r, int c,
                                           const T *__restrict__ res, int nt, int n)
{
    T *f = c == 0 ? ax : (c == 1 ? ay : az);
    const RecTap<T> &t = taps[r * 3 + c];
    const T v = res[((long)r * 3 + c) * nt + n];
#pragma unroll
    for (int m = 0; m < 8; ++m)
        if (t.idx[m] >= 0) f[t.idx[m]] += t.w[m] * v;
}

template <typename T>
__global__ void __launch_bounds__(256) inject_residual(T *__restrict__ ax, T *__restrict__ ay, T *__restrict__ az,
                                                       const RecTap<T> *__restrict__ taps, const int *__restrict__ list,
                                                       int count, const T *__restrict__ res, int nt, int n)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= 3 * count) return;
    inject_one(ax, ay, az, taps, list[q / 3], q % 3, res, nt, n);
}

// (a11) for the tiled adjoint, whose velocity pass has already formed Y and its share of
// the gradient of b: the injected d = w r at a tap adds G_v d b to Y and
// d v^{n+1/2} rho_eff to g_b there.  Field pointers and strides of one grid (a tap's
// storage index gives its node).
template <typename T> struct TapAdjoint {
    T *y[3], *gb[3];
    const T *vst[3];  // stored v^{n+1/2}
    const T *rho;
    const T *g[3][2];  // damping profiles (as Grid::g)
    long sy, sz;
};

// Tap m of component c of receiver r (one thread per tap: the eight taps of a receiver
// component are distinct samples).  Storage indices are below 2^31, so the node is found
// with 32-bit divisions.
template <typename T>
__device__ __forceinline__ void inject_tap_tiled(const TapAdjoint<T> &A, const RecTap<T> *__restrict__ taps, int r,
                                                 int c, int m, const T *__restrict__ res, int nt, int n)
{
    const RecTap<T> &t = taps[r * 3 + c];
    const int q = t.idx[m];
    if (q < 0) return;
    const T d = t.w[m] * res[((long)r * 3 + c) * nt + n];
    const unsigned sy = (unsigned)A.sy, sz = (unsigned)A.sz;
    const unsigned k = (unsigned)q / sz, rem = (unsigned)q - k * sz;
    const unsigned j = rem / sy, i = rem - j * sy;
    const T g = A.g[0][c == 0][i] * A.g[1][c == 1][j] * A.g[2][c == 2][k];
    const long e = c == 0 ? 1 : (c == 1 ? A.sy : A.sz);
    const T ra = A.rho[q], rb = A.rho[q + e];
    A.y[c][q] += (g * d) * buoy(ra, rb);
    A.gb[c][q] += (A.vst[c][q] * ((ra + rb) * T(0.5))) * d;
}

template <typename T>
__global__ void __launch_bounds__(256) inject_residual_tiled(TapAdjoint<T> A, const RecTap<T> *__restrict__ taps,
                                                             const int *__restrict__ list, int count,
                                                             const T *__restrict__ res, int nt, int n)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= 24 * count) return;
    const int rc = q >> 3;
    inject_tap_tiled(A, taps, list[rc / 3], rc % 3, q & 7, res, nt, n);
}

// (a13) chain rule from the staggered-point gradients to the node arrays (gathers, no
// atomics): g_lam += gl; g_mu += gm + 1/4 sum of the shear gradients whose mean uses the
// node; g_rho += sum over the adjacent velocity samples of -b^2/2 g_b.
template <typename T>
__global__ void __launch_bounds__(256) grad_finalize(Grid<T> G, AdjGrid<T> A, T *__restrict__ g_lam,
                                                     T *__restrict__ g_mu, T *__restrict__ g_rho)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= G.nx || j >= G.ny) return;
    const long p = i + G.sy * j + G.sz * k;
    const long po = i + (long)G.nx * (j + (long)G.ny * k);  // the node arrays' own index
    g_lam[po] += A.gl[p];
    T sh = T(0);
    for (int di = -1; di <= 0; ++di)
        for (int dj = -1; dj <= 0; ++dj) sh += rdc(A.gs[0], SXY, i + di, j + dj, k, G);
    for (int di = -1; di <= 0; ++di)
        for (int dk = -1; dk <= 0; ++dk) sh += rdc(A.gs[1], SXZ, i + di, j, k + dk, G);
    for (int dj = -1; dj <= 0; ++dj)
        for (int dk = -1; dk <= 0; ++dk) sh += rdc(A.gs[2], SYZ, i, j + dj, k + dk, G);
    g_mu[po] += A.gm[p] + sh / T(4);
    T gr = T(0);
    for (int c = 0; c < 3; ++c) {
        const long e = c == 0 ? 1 : (c == 1 ? G.sy : G.sz);
        for (int d = -1; d <= 0; ++d) {
            const int ii = i + (c == 0 ? d : 0), jj = j + (c == 1 ? d : 0), kk = k + (c == 2 ? d : 0);
            const T g = rdc(A.gb[c], VX + c, ii, jj, kk, G);
            if (g != T(0)) {
                const long q = ii + G.sy * jj + G.sz * kk;
                const T b = buoy(G.rho[q], G.rho[q + e]);
                gr += -g * (b * b) / T(2);
            }
        }
    }
    g_rho[po] += gr;
}

// Adjoint of the initial velocity, G_v A_v, into out (a node array, x fastest and
// unpadded): from A_v (the one-thread-per-cell adjoint), or from Y (the tiled adjoint),
// below.
template <typename T>
__global__ void __launch_bounds__(256) scale_velocity(Grid<T> G, const T *__restrict__ a, int c, T *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= G.nx || j >= G.ny) return;
    out[i + (long)G.nx * (j + (long)G.ny * k)] = damp(G, c, i, j, k) * a[i + G.sy * j + G.sz * k];
}

// The last term of the tiled adjoint's gradient of b: g_b -= v^{-1/2} rho_eff (Y rho_eff),
// with v^{-1/2} the initial velocity (v0) and Y that of the first step.
template <typename T>
__global__ void __launch_bounds__(256) gb_initial_velocity(Grid<T> G, const T *__restrict__ v0x,
                                                           const T *__restrict__ v0y, const T *__restrict__ v0z,
                                                           const T *__restrict__ yx, const T *__restrict__ yy,
                                                           const T *__restrict__ yz, T *gbx, T *gby, T *gbz)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= G.nx || j >= G.ny) return;
    const long p = i + G.sy * j + G.sz * k;
    const T *v0[3] = {v0x, v0y, v0z}, *y[3] = {yx, yy, yz};
    T *gb[3] = {gbx, gby, gbz};
    const bool act[3] = {i <= G.nx - 2, j <= G.ny - 2, k <= G.nz - 2};
    const long e[3] = {1, G.sy, G.sz};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (!act[c]) continue;
        const T re = (G.rho[p] + G.rho[p + e[c]]) * T(0.5);
        gb[c][p] -= (v0[c][p] * re) * (y[c][p] * re);
    }
}

// G_v A_v = Y rho_eff at the active samples of component c (zero elsewhere).
template <typename T>
__global__ void __launch_bounds__(256) velocity_from_y(Grid<T> G, const T *__restrict__ y, int c, T *__restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= G.nx || j >= G.ny) return;
    const bool act = c == VX ? i <= G.nx - 2 : (c == VY ? j <= G.ny - 2 : k <= G.nz - 2);
    T v = T(0);
    if (act) {
        const long p = i + G.sy * j + G.sz * k, e = c == VX ? 1 : (c == VY ? G.sy : G.sz);
        v = y[p] * ((G.rho[p] + G.rho[p + e]) * T(0.5));
    }
    out[i + (long)G.nx * (j + (long)G.ny * k)] = v;
}

// ---------------------------------------------------------------------------------
// Residual injection for many shots per launch.  Colour c's receivers of every shot form
// one flat work list (shot-major, three components per receiver); shots never share
// adjoint arrays, so one launch per colour is free of races.
constexpr int kMaxBatchColors = 4;

template <typename T> struct ShotInject {
    TapAdjoint<T> t;  // the shot's Y, g_b, stored velocities of the step's segment slot, model
    const RecTap<T> *taps;
    const int *colors;
    const T *res;
    int coff[kMaxBatchColors + 1];  // colour c: colors[coff[c] .. coff[c+1])
    int rbase[kMaxBatchColors];     // first work item of this shot in colour c's flat list
};

// total: work items of the colour (three per receiver); one thread per tap of an item.
template <typename T>
__global__ void __launch_bounds__(256) inject_residual_multi(const ShotInject<T> *__restrict__ d, int nshot, int color,
                                                             int total, int nt, int n)
{
    __shared__ int s_base[kMaxShots];
    for (int t = threadIdx.x; t < nshot; t += blockDim.x) s_base[t] = d[t].rbase[color];
    __syncthreads();
    const int qt = blockIdx.x * blockDim.x + threadIdx.x;
    if (qt >= 8 * total) return;
    const int q = qt >> 3;
    int s = 0;
    while (s + 1 < nshot && s_base[s + 1] <= q) ++s;
    const ShotInject<T> &sh = d[s];
    const int l = q - sh.rbase[color];
    const int r = sh.colors[sh.coff[color] + l / 3];
    inject_tap_tiled(sh.t, sh.taps, r, l % 3, qt & 7, sh.res, nt, n);
}

// Copies of many equally long arrays (checkpoint save / restore of every shot).
template <typename T> struct CopyDesc {
    const T *src;
    T *dst;
    long n;
};

template <typename T> __global__ void __launch_bounds__(256) copy_multi(const CopyDesc<T> *__restrict__ d)
{
    const CopyDesc<T> &c = d[blockIdx.y];
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < c.n; q += (long)gridDim.x * blockDim.x)
        c.dst[q] = c.src[q];
}

// Residual r = d - d_obs of one shot's traces and per-block partial sums of r^2 / 2
// (deterministic two-stage reduction: misfit_final adds the partials in order).
template <typename T>
__global__ void __launch_bounds__(256) residual_misfit(const T *__restrict__ d, const T *__restrict__ obs,
                                                       T *__restrict__ r, long n, double *__restrict__ part)
{
    __shared__ double sh[256];
    double acc = 0.0;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
        const T v = d[q] - obs[q];
        r[q] = v;
        acc += (double)v * (double)v;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

template <typename T>
__global__ void __launch_bounds__(64) misfit_final(const double *__restrict__ part, int nb, T *__restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[b];
    out[0] = (T)(0.5 * s);
}

} // namespace fd3d
