// Small utility kernels: fills, copies with pinned-slot masking, model statistics
// (deterministic two-stage reduction) and the non-finite check.
#pragma once

#include "common.h"

namespace fd3d {

constexpr int kReduceBlocks = 512;
constexpr int kReduceThreads = 256;
constexpr int kStats = 6;  // vp_max, vs_min(mu>0), rho_min, mu_min, m2_min, bad

template <typename T>
__global__ void __launch_bounds__(256) fill_zero(T *__restrict__ p, long n)
{
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x)
        p[q] = T(0);
}

// dst = src for the active samples of a component with half offsets (sx, sy, sz), 0 at its
// pinned slots (all offsets 0: a plain copy).  Each side has its own row and plane strides
// (a node array: nx, nx ny; a field of the interleaved-rows layout: 9 nx, 9 nx ny).
template <typename T>
__global__ void __launch_bounds__(256) copy_masked(T *__restrict__ dst, long dsy, long dsz, const T *__restrict__ src,
                                                   long ssy, long ssz, int nx, int ny, int nz, int sx, int sy, int sz)
{
    const long n = (long)nx * ny * nz;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
        const int i = (int)(q % nx);
        const int j = (int)((q / nx) % ny);
        const int k = (int)(q / ((long)nx * ny));
        const bool ok = i <= nx - 1 - sx && j <= ny - 1 - sy && k <= nz - 1 - sz;
        dst[i + dsy * j + dsz * k] = ok ? src[i + ssy * j + ssz * k] : T(0);
    }
}

// Medium given on a coarse node grid c[mz][my][mx], sampled trilinearly at every node of
// the simulation grid f[nz][ny][nx] (Sec. 2.2.1); both grids span the same box, so node i
// sits at coarse coordinate i (m - 1) / (n - 1).  Weights and sums in double.
__device__ __forceinline__ void coarse_axis(int i, int n, int m, int &lo, int &hi, double &t)
{
    const double q = n > 1 ? i * ((double)(m - 1) / (double)(n - 1)) : 0.0;
    lo = (int)floor(q);
    lo = lo < m - 2 ? lo : (m - 2 > 0 ? m - 2 : 0);
    hi = lo + 1 < m - 1 ? lo + 1 : m - 1;
    t = q - lo;
}

template <typename T>
__global__ void __launch_bounds__(256) upsample_trilinear(const T *__restrict__ c, int mx, int my, int mz,
                                                          T *__restrict__ f, int nx, int ny, int nz)
{
    const long n = (long)nx * ny * nz;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
        const int i = (int)(q % nx);
        const int j = (int)((q / nx) % ny);
        const int k = (int)(q / ((long)nx * ny));
        int x0, x1, y0, y1, z0, z1;
        double tx, ty, tz;
        coarse_axis(i, nx, mx, x0, x1, tx);
        coarse_axis(j, ny, my, y0, y1, ty);
        coarse_axis(k, nz, mz, z0, z1, tz);
        const int zs[2] = {z0, z1}, ys[2] = {y0, y1}, xs[2] = {x0, x1};
        const double wz[2] = {1.0 - tz, tz}, wy[2] = {1.0 - ty, ty}, wx[2] = {1.0 - tx, tx};
        double v = 0.0;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int d = 0; d < 2; ++d)
                    v += wz[a] * wy[b] * wx[d] * (double)c[xs[d] + (long)mx * (ys[b] + (long)my * zs[a])];
        f[q] = (T)v;
    }
}

__device__ __forceinline__ double dmin(double a, double b) { return a < b ? a : b; }
__device__ __forceinline__ double dmax(double a, double b) { return a > b ? a : b; }

// Per-block partial statistics of the model, written to part[block][kStats].
template <typename T>
__global__ void __launch_bounds__(kReduceThreads) model_stats(const T *__restrict__ lam, const T *__restrict__ mu,
                                                              const T *__restrict__ rho, long n, double *__restrict__ part)
{
    __shared__ double sh[kStats][kReduceThreads];
    double vpmax = 0.0, vsmin = 1e300, rmin = 1e300, mmin = 1e300, m2min = 1e300, bad = 0.0;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
        const double l = (double)lam[q], m = (double)mu[q], r = (double)rho[q];
        if (!isfinite(l) || !isfinite(m) || !isfinite(r)) { bad = 1.0; continue; }
        rmin = dmin(rmin, r);
        mmin = dmin(mmin, m);
        m2min = dmin(m2min, l + 2.0 * m);
        if (r > 0.0 && l + 2.0 * m > 0.0) vpmax = dmax(vpmax, sqrt((l + 2.0 * m) / r));
        if (r > 0.0 && m > 0.0) vsmin = dmin(vsmin, sqrt(m / r));
    }
    const int t = threadIdx.x;
    sh[0][t] = vpmax; sh[1][t] = vsmin; sh[2][t] = rmin; sh[3][t] = mmin; sh[4][t] = m2min; sh[5][t] = bad;
    __syncthreads();
    for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
        if (t < w) {
            sh[0][t] = dmax(sh[0][t], sh[0][t + w]);
            for (int s = 1; s < 5; ++s) sh[s][t] = dmin(sh[s][t], sh[s][t + w]);
            sh[5][t] = dmax(sh[5][t], sh[5][t + w]);
        }
        __syncthreads();
    }
    if (t < kStats) part[blockIdx.x * kStats + t] = sh[t][0];
}

static __global__ void __launch_bounds__(kReduceThreads) stats_final(const double *__restrict__ part, int nblocks,
                                                              double *__restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double r[kStats] = {0.0, 1e300, 1e300, 1e300, 1e300, 0.0};
    for (int b = 0; b < nblocks; ++b) {
        r[0] = dmax(r[0], part[b * kStats + 0]);
        for (int s = 1; s < 5; ++s) r[s] = dmin(r[s], part[b * kStats + s]);
        r[5] = dmax(r[5], part[b * kStats + 5]);
    }
    for (int s = 0; s < kStats; ++s) out[s] = r[s];
}

// flag[0] = 1 if any of the nine fields holds a non-finite value (written only then).
template <typename T>
__global__ void __launch_bounds__(256) finite_check(Grid<T> G, int *__restrict__ flag)
{
    const long n = (long)G.nx * G.ny * G.nz;
    bool bad = false;
    for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
        const int i = (int)(q % G.nx);
        const int j = (int)((q / G.nx) % G.ny);
        const int k = (int)(q / ((long)G.nx * G.ny));
        const long p = i + G.sy * j + G.sz * k;
        for (int c = 0; c < NFIELD; ++c) bad |= !isfinite(G.f[c][p]);
    }
    if (bad) flag[0] = 1;
}

} // namespace fd3d
