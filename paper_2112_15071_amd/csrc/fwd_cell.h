// One-thread-per-cell forward passes (velocity, stress) and receiver sampling.
//
// Every neighbour is read straight from global memory with a bounds test; this
// is the simplest complete form of the passes and serves small grids, the FP64
// mode and the free-surface top planes.
#pragma once

#include "common.h"

namespace fd3d {

// Sample of component C at (i,j,k); zero outside the component's active range.
template <int C, typename T>
__device__ __forceinline__ T rd(const Grid<T> &G, int i, int j, int k)
{
    const int lx = G.nx - 1 - stag(C, 0), ly = G.ny - 1 - stag(C, 1), lz = G.nz - 1 - stag(C, 2);
    const bool ok = (unsigned)i <= (unsigned)lx && (unsigned)j <= (unsigned)ly && (unsigned)k <= (unsigned)lz;
    return ok ? G.f[C][i + G.sy * j + G.sz * k] : T(0);
}

// Stress read for the velocity pass; with the free surface, values above k = 0 are
// odd images: szz(-m) = -szz(m), and sxz/syz at z = -(m+1/2) mirror z = m+1/2.
template <int C, bool FS, typename T>
__device__ __forceinline__ T rds(const Grid<T> &G, int i, int j, int k)
{
    if (FS && k < 0) {
        if (C == SZZ) return -rd<SZZ>(G, i, j, -k);
        if (C == SXZ || C == SYZ) return -rd<C>(G, i, j, -1 - k);
        return T(0);
    }
    return rd<C>(G, i, j, k);
}

// (V) of one step: v <- G (v + dt b div(sigma) + b c s), Eq.(1) with Eq.(4).
template <typename T, bool FS>
__global__ void __launch_bounds__(256) vel_cell(Grid<T> G, Inject<T> src, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= G.nx || j >= G.ny) return;
    const long p = i + G.sy * j + G.sz * k;
    const T s = src.on ? src.wavelet[n] : T(0);
    const SurfacePlanes sp = surface_planes(G, i, j);
    const T rdx = G.rdx, rdy = G.rdy, rdz = G.rdz;

    if (i <= G.nx - 2) {
        T d = dstag(rds<SXX, FS>(G, i + 1, j, k), rds<SXX, FS>(G, i, j, k), rds<SXX, FS>(G, i + 2, j, k), rds<SXX, FS>(G, i - 1, j, k), rdx)
            + dstag(rds<SXY, FS>(G, i, j, k), rds<SXY, FS>(G, i, j - 1, k), rds<SXY, FS>(G, i, j + 1, k), rds<SXY, FS>(G, i, j - 2, k), rdy)
            + dz_or_o2(o2_int(sp.x, k), rds<SXZ, FS>(G, i, j, k), rds<SXZ, FS>(G, i, j, k - 1), rds<SXZ, FS>(G, i, j, k + 1), rds<SXZ, FS>(G, i, j, k - 2), rdz);
        const T b = buoy(G.rho[p], G.rho[p + 1]);
        T v = G.f[VX][p] + G.dt * b * d;
        const int t = tap_of(src, VX, i, j, k);
        if (t >= 0) v += b * src.coef[VX * 8 + t] * s;
        v = v * (G.g[0][1][i] * G.g[1][0][j] * G.g[2][0][k]);
        G.f[VX][p] = v;
        if (G.save[VX]) G.save[VX][p] = v;
    }
    if (j <= G.ny - 2) {
        T d = dstag(rds<SXY, FS>(G, i, j, k), rds<SXY, FS>(G, i - 1, j, k), rds<SXY, FS>(G, i + 1, j, k), rds<SXY, FS>(G, i - 2, j, k), rdx)
            + dstag(rds<SYY, FS>(G, i, j + 1, k), rds<SYY, FS>(G, i, j, k), rds<SYY, FS>(G, i, j + 2, k), rds<SYY, FS>(G, i, j - 1, k), rdy)
            + dz_or_o2(o2_int(sp.y, k), rds<SYZ, FS>(G, i, j, k), rds<SYZ, FS>(G, i, j, k - 1), rds<SYZ, FS>(G, i, j, k + 1), rds<SYZ, FS>(G, i, j, k - 2), rdz);
        const T b = buoy(G.rho[p], G.rho[p + G.sy]);
        T v = G.f[VY][p] + G.dt * b * d;
        const int t = tap_of(src, VY, i, j, k);
        if (t >= 0) v += b * src.coef[VY * 8 + t] * s;
        v = v * (G.g[0][0][i] * G.g[1][1][j] * G.g[2][0][k]);
        G.f[VY][p] = v;
        if (G.save[VY]) G.save[VY][p] = v;
    }
    if (k <= G.nz - 2) {
        T d = dstag(rds<SXZ, FS>(G, i, j, k), rds<SXZ, FS>(G, i - 1, j, k), rds<SXZ, FS>(G, i + 1, j, k), rds<SXZ, FS>(G, i - 2, j, k), rdx)
            + dstag(rds<SYZ, FS>(G, i, j, k), rds<SYZ, FS>(G, i, j - 1, k), rds<SYZ, FS>(G, i, j + 1, k), rds<SYZ, FS>(G, i, j - 2, k), rdy)
            + dz_or_o2(o2_half(sp.n, k), rds<SZZ, FS>(G, i, j, k + 1), rds<SZZ, FS>(G, i, j, k), rds<SZZ, FS>(G, i, j, k + 2), rds<SZZ, FS>(G, i, j, k - 1), rdz);
        const T b = buoy(G.rho[p], G.rho[p + G.sz]);
        T v = G.f[VZ][p] + G.dt * b * d;
        const int t = tap_of(src, VZ, i, j, k);
        if (t >= 0) v += b * src.coef[VZ * 8 + t] * s;
        v = v * (G.g[0][0][i] * G.g[1][0][j] * G.g[2][1][k]);
        G.f[VZ][p] = v;
        if (G.save[VZ]) G.save[VZ][p] = v;
    }
}

// (S) of one step: sigma <- G (sigma + dt C:eps(v) + c s), Eq.(2) with Eq.(4); with
// the free surface: szz = 0 at k = 0, dz vz from szz = 0 at k = 0, second-order dz
// where the fourth-order stencil would reach above the surface.
template <typename T, bool FS>
__global__ void __launch_bounds__(256) stress_cell(Grid<T> G, Inject<T> src, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z;
    if (i >= G.nx || j >= G.ny) return;
    const long p = i + G.sy * j + G.sz * k;
    const T s = src.on ? src.wavelet[n] : T(0);
    const SurfacePlanes sp = surface_planes(G, i, j);
    const T rdx = G.rdx, rdy = G.rdy, rdz = G.rdz, dt = G.dt;

    const T exx = dstag(rd<VX>(G, i, j, k), rd<VX>(G, i - 1, j, k), rd<VX>(G, i + 1, j, k), rd<VX>(G, i - 2, j, k), rdx);
    const T eyy = dstag(rd<VY>(G, i, j, k), rd<VY>(G, i, j - 1, k), rd<VY>(G, i, j + 1, k), rd<VY>(G, i, j - 2, k), rdy);
    const T l = G.lam[p], m = G.mu[p];
    T ezz;
    if (FS && k == 0) ezz = -l / (l + T(2) * m) * (exx + eyy);
    else if (FS && k == 1) ezz = (rd<VZ>(G, i, j, 1) - rd<VZ>(G, i, j, 0)) * rdz;
    else ezz = dz_or_o2(o2_int(sp.n, k), rd<VZ>(G, i, j, k), rd<VZ>(G, i, j, k - 1), rd<VZ>(G, i, j, k + 1), rd<VZ>(G, i, j, k - 2), rdz);
    const T tr = exx + eyy + ezz;
    const T gn = G.g[0][0][i] * G.g[1][0][j] * G.g[2][0][k];
    {
        T sxx = G.f[SXX][p] + dt * (l * tr + T(2) * m * exx);
        T syy = G.f[SYY][p] + dt * (l * tr + T(2) * m * eyy);
        T szz = G.f[SZZ][p] + dt * (l * tr + T(2) * m * ezz);
        int t = tap_of(src, SXX, i, j, k);
        if (t >= 0) {
            sxx += src.coef[SXX * 8 + t] * s;
            syy += src.coef[SYY * 8 + t] * s;
            szz += src.coef[SZZ * 8 + t] * s;
        }
        G.f[SXX][p] = sxx * gn;
        G.f[SYY][p] = syy * gn;
        G.f[SZZ][p] = (FS && k == 0) ? T(0) : szz * gn;
    }
    if (i <= G.nx - 2 && j <= G.ny - 2) {
        const T e = dstag(rd<VX>(G, i, j + 1, k), rd<VX>(G, i, j, k), rd<VX>(G, i, j + 2, k), rd<VX>(G, i, j - 1, k), rdy)
                  + dstag(rd<VY>(G, i + 1, j, k), rd<VY>(G, i, j, k), rd<VY>(G, i + 2, j, k), rd<VY>(G, i - 1, j, k), rdx);
        const T mxy = ((G.mu[p] + G.mu[p + 1]) + (G.mu[p + G.sy] + G.mu[p + 1 + G.sy])) / T(4);
        T v = G.f[SXY][p] + dt * mxy * e;
        const int t = tap_of(src, SXY, i, j, k);
        if (t >= 0) v += src.coef[SXY * 8 + t] * s;
        G.f[SXY][p] = v * (G.g[0][1][i] * G.g[1][1][j] * G.g[2][0][k]);
    }
    if (i <= G.nx - 2 && k <= G.nz - 2) {
        const T dzvx = (FS && k == 0) ? (rd<VX>(G, i, j, 1) - rd<VX>(G, i, j, 0)) * rdz
                     : dz_or_o2(o2_half(sp.x, k), rd<VX>(G, i, j, k + 1), rd<VX>(G, i, j, k), rd<VX>(G, i, j, k + 2), rd<VX>(G, i, j, k - 1), rdz);
        const T e = dzvx + dstag(rd<VZ>(G, i + 1, j, k), rd<VZ>(G, i, j, k), rd<VZ>(G, i + 2, j, k), rd<VZ>(G, i - 1, j, k), rdx);
        const T mxz = ((G.mu[p] + G.mu[p + 1]) + (G.mu[p + G.sz] + G.mu[p + 1 + G.sz])) / T(4);
        T v = G.f[SXZ][p] + dt * mxz * e;
        const int t = tap_of(src, SXZ, i, j, k);
        if (t >= 0) v += src.coef[SXZ * 8 + t] * s;
        G.f[SXZ][p] = v * (G.g[0][1][i] * G.g[1][0][j] * G.g[2][1][k]);
    }
    if (j <= G.ny - 2 && k <= G.nz - 2) {
        const T dzvy = (FS && k == 0) ? (rd<VY>(G, i, j, 1) - rd<VY>(G, i, j, 0)) * rdz
                     : dz_or_o2(o2_half(sp.y, k), rd<VY>(G, i, j, k + 1), rd<VY>(G, i, j, k), rd<VY>(G, i, j, k + 2), rd<VY>(G, i, j, k - 1), rdz);
        const T e = dzvy + dstag(rd<VZ>(G, i, j + 1, k), rd<VZ>(G, i, j, k), rd<VZ>(G, i, j + 2, k), rd<VZ>(G, i, j - 1, k), rdy);
        const T myz = ((G.mu[p] + G.mu[p + G.sy]) + (G.mu[p + G.sz] + G.mu[p + G.sy + G.sz])) / T(4);
        T v = G.f[SYZ][p] + dt * myz * e;
        const int t = tap_of(src, SYZ, i, j, k);
        if (t >= 0) v += src.coef[SYZ * 8 + t] * s;
        G.f[SYZ][p] = v * (G.g[0][0][i] * G.g[1][1][j] * G.g[2][1][k]);
    }
}

// (R) of one step as a job that a launch can carry: work item q < nq (= 3 nrec) writes
// traces[q][n] = sum_m w_m v_c[idx_m], c = q % 3 (trilinear, Sec. 2.4).
template <typename T> struct RecJob {
    const T *v[3];
    const RecTap<T> *taps;
    T *traces;
    int nq, nt;
};

template <typename T> __device__ __forceinline__ void sample_receiver(const RecJob<T> &r, int q, int n)
{
    const int c = q % 3;
    const T *f = c == 0 ? r.v[0] : (c == 1 ? r.v[1] : r.v[2]);
    const RecTap<T> &t = r.taps[q];
    T s = T(0);
#pragma unroll
    for (int m = 0; m < 8; ++m)
        if (t.idx[m] >= 0) s += t.w[m] * f[t.idx[m]];
    r.traces[(long)q * r.nt + n] = s;
}

// Workgroups needed to carry a job with NT threads each.
template <typename T> inline int rec_blocks(const RecJob<T> &r, int nt) { return (r.nq + nt - 1) / nt; }

template <typename T> __global__ void __launch_bounds__(256) record(RecJob<T> r, int n)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < r.nq) sample_receiver(r, q, n);
}

// Receiver sampling of many shots: shot s owns work items [base, base + 3 nrec) of a
// flat list.
template <typename T> struct ShotRec {
    const T *v[3];
    const RecTap<T> *taps;
    T *traces;
    int nrec, base;
};

template <typename T> __device__ __forceinline__ void sample_shot_receiver(const ShotRec<T> &d, int l, int nt, int n)
{
    const int c = l % 3;
    const T *f = d.v[c];
    const RecTap<T> &t = d.taps[l];
    T acc = T(0);
#pragma unroll
    for (int m = 0; m < 8; ++m)
        if (t.idx[m] >= 0) acc += t.w[m] * f[t.idx[m]];
    d.traces[(long)l * nt + n] = acc;
}

// Shot of work item q: the last s with base[s] <= q (bases ascending, base[0] = 0).
__device__ __forceinline__ int rec_shot(const int *s_base, int nshot, int q)
{
    int s = 0;
    while (s + 1 < nshot && s_base[s + 1] <= q) ++s;
    return s;
}

// Receiver sampling of a batch carried by a persistent launch of wgs workgroups: the
// workgroups past the first wgs take the total work items of the flat list.
template <typename T> struct RecMulti {
    const ShotRec<T> *shots;
    int nshot, total, nt, wgs;
};

template <typename T> inline int rec_blocks(const RecMulti<T> &r, int nt) { return (r.total + nt - 1) / nt; }

// Body of one such workgroup (block-uniform; s_base: LDS scratch of kMaxShots ints).
template <typename T> __device__ __forceinline__ void sample_batch_receivers(const RecMulti<T> &r, int *s_base, int n)
{
    for (int t = threadIdx.x; t < r.nshot; t += blockDim.x) s_base[t] = r.shots[t].base;
    __syncthreads();
    const int q = ((int)blockIdx.x - r.wgs) * (int)blockDim.x + (int)threadIdx.x;
    if (q >= r.total) return;
    const int s = rec_shot(s_base, r.nshot, q);
    sample_shot_receiver(r.shots[s], q - r.shots[s].base, r.nt, n);
}

} // namespace fd3d
