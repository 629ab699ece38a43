// Fused time step: the velocity update and the stress update of one step in a single
// z sweep, on a double-buffered state (read the old state, write the new one).
//
// The two-pass step reads the stress twice and the velocity twice per step (once in
// each pass); the fused step reads the old state once and writes the new one once:
// 12 fields in (6 stress, 3 velocity, rho, lambda, mu), 9 out, 84 B per cell in FP32
// against 120 B for the two passes.  The price is recomputation: the stress stencils of
// a tile need the new velocity on a 2-cell ring around it, and that ring belongs to the
// neighbouring tiles, so every workgroup recomputes the new velocity on its tile plus
// the ring from the old state (which no workgroup overwrites: it lives in the other
// buffer).
//
// Per z plane p a workgroup
//   1. stages the old stress plane p and rho over the tile plus a 4-cell ring in LDS
//      (one thread per velocity column loads its own samples, a few load the outer ring),
//   2. computes the new velocity at plane p on the tile plus the 2-cell ring, one thread
//      per column, z derivatives from per-thread register queues of the old stress,
//   3. computes the new stress at plane p - 2 on the tile from the new velocity of planes
//      p - 4 .. p: x/y stencils from a ring of three LDS planes, z stencils from
//      per-thread register queues.
// All loads of plane p + 1 are issued before the compute of plane p, and one barrier per
// plane orders the LDS traffic.  A z chunk [k0, k1) computes the velocity on planes
// k0 - 2 .. k1 + 1 and stores the velocity and stress of its own planes only.
//
// Every sample is computed with the expressions of the two-pass kernels (same operand
// order), so the two variants agree bit for bit.  Samples outside the grid and pinned
// staggered samples of the new velocity are zero; the new state is written at every
// grid sample of the chunk (pinned slots included, as zero), so the output buffer needs
// no initialisation.
#pragma once

#include "fwd_tile.h"

namespace fd3d {

template <int TX, int TY> struct Fused {
    static constexpr int EX = TX + 4, EY = TY + 4;  // velocity box: columns [-2, TX+2) x [-2, TY+2)
    static constexpr int NE = EX * EY;              // velocity threads
    static constexpr int NT = (NE + 63) / 64 * 64;  // workgroup size
    static constexpr int BX = TX + 8, BY = TY + 8;  // old-state box: [-4, TX+4) x [-4, TY+4)
    static constexpr int NB = BX * BY;
    static constexpr int MX = TX + 1;  // mu box: [0, TX] x [0, TY]
    static constexpr int NM = MX * (TY + 1);
    __device__ static int e_index(int x, int y) { return (y + 2) * EX + x + 2; }
    __device__ static int b_index(int x, int y) { return (y + 4) * BX + x + 4; }
};

// Column (x, y) of velocity thread t, relative to the tile corner: the tile row by row,
// the two rows below it, the two rows above it, then the four side columns (full box
// height, so they hold the corners).  Threads past the box get an idle sentinel.
template <int TX, int TY> __device__ __forceinline__ bool fused_column(int t, int &x, int &y)
{
    constexpr int O = TX * TY, R = 2 * TX, EY = Fused<TX, TY>::EY;
    if (t < O) {
        x = t % TX;
        y = t / TX;
    } else if (t < O + R) {
        x = (t - O) % TX;
        y = -2 + (t - O) / TX;
    } else if (t < O + 2 * R) {
        x = (t - O - R) % TX;
        y = TY + (t - O - R) / TX;
    } else if (t < Fused<TX, TY>::NE) {
        const int u = t - O - 2 * R, c = u / EY;
        y = -2 + u % EY;
        x = c < 2 ? c - 2 : TX + c - 2;
    } else {
        x = y = 0;
        return false;
    }
    return true;
}

// Cell r of the ring [XA, XB) x [YA, YB) minus the velocity box: left columns and right
// columns (full height), then bottom rows and top rows (velocity-box width).
template <int TX, int TY, int XA, int XB, int YA, int YB> __device__ __forceinline__ bool ring_cell(int r, int &x, int &y)
{
    constexpr int H = YB - YA, NL = -2 - XA, NR = XB - (TX + 2), NBOT = -2 - YA, NTOP = YB - (TY + 2), EX = TX + 4;
    if (r < NL * H) {
        x = XA + r / H;
        y = YA + r % H;
        return true;
    }
    r -= NL * H;
    if (r < NR * H) {
        x = TX + 2 + r / H;
        y = YA + r % H;
        return true;
    }
    r -= NR * H;
    if (r < NBOT * EX) {
        y = YA + r / EX;
        x = -2 + r % EX;
        return true;
    }
    r -= NBOT * EX;
    if (r < NTOP * EX) {
        y = TY + 2 + r / EX;
        x = -2 + r % EX;
        return true;
    }
    return false;
}

// The ring cell this thread loads for one old-state plane (thread t takes cell
// (t - OFF) mod NT; OFF spreads the rings of the six planes over the workgroup).
template <typename T, int TX, int TY, int XA, int XB, int YA, int YB, int OFF>
__device__ __forceinline__ Slot ring_slot(int t, int i0, int j0, int nx, int ny, int sy)
{
    using F = Fused<TX, TY>;
    Slot s{F::NB, kOOB};
    int x, y;
    const int r = (t + F::NT - OFF % F::NT) % F::NT;
    if (ring_cell<TX, TY, XA, XB, YA, YB>(r, x, y)) {
        s.lds = F::b_index(x, y);
        const int gi = i0 + x, gj = j0 + y;
        if (gi >= 0 && gi < nx && gj >= 0 && gj < ny) s.off = (unsigned)(gi + sy * gj) * (unsigned)sizeof(T);
    }
    return s;
}

// The mu ring cell of this thread: right column x = TX, top row y = TY, the corner.
template <typename T, int TX, int TY, int OFF>
__device__ __forceinline__ Slot mu_slot(int t, int i0, int j0, int nx, int ny, int sy)
{
    using F = Fused<TX, TY>;
    Slot s{F::NM, kOOB};
    const int r = (t + F::NT - OFF % F::NT) % F::NT;
    int x = -1, y = -1;
    if (r < TY) {
        x = TX;
        y = r;
    } else if (r < TY + TX) {
        x = r - TY;
        y = TY;
    } else if (r == TY + TX) {
        x = TX;
        y = TY;
    }
    if (x >= 0) {
        s.lds = y * F::MX + x;
        const int gi = i0 + x, gj = j0 + y;
        if (gi < nx && gj < ny) s.off = (unsigned)(gi + sy * gj) * (unsigned)sizeof(T);
    }
    return s;
}

// Arguments of the fused step, kept compact so that the sweep holds few scalar
// registers: each state copy is one base pointer with a fixed field stride, the
// source's tap boxes are given by per-axis origins on the integer and half subgrids, and
// its coefficients are copied into LDS at kernel start.
template <typename T> struct FusedArgs {
    const T *in;    // current state: field q at in + q * fs
    T *out;         // next state, same layout
    long fs;        // elements between consecutive fields
    int nx, ny, nz, sy;
    long sz;
    T dt, rdx, rdy, rdz;
    const T *lam, *mu, *rho;
    const T *gx[2], *gy[2], *gz[2];  // damping profiles at integer [0] / half [1] positions
    const T *wavelet;                // source time function; NULL: no source
    int n;                           // time step
    int origin[3][2];                // source tap-box origin per axis, integer / half subgrid
    int mask;                        // bit q: component q carries source coefficients
    T coef[NFIELD][8];               // source coefficients (x fastest, then y, z)
};

template <typename T, int TX, int TY, bool FS>
__device__ __forceinline__ void fused_body(const FusedArgs<T> &A, int i0, int j0, int k0, int k1)
{
    using F = Fused<TX, TY>;
    static_assert(TX == 64, "one wave per tile row");
    constexpr int BX = F::BX, EX = F::EX, MX = F::MX;
    __shared__ T s_old[2][6][F::NB + 1];  // old sxx, syy, sxy, sxz, syz, rho of one plane
    __shared__ T s_v[3][3][F::NE + 1];    // new vx, vy, vz of three planes
    __shared__ T s_mu[3][F::NM + 1];      // mu of three planes
    __shared__ T s_coef[NFIELD * 8];

    const int nx = A.nx, ny = A.ny, nz = A.nz;
    const int sy = A.sy;
    const long sz = A.sz, fs = A.fs;
    const int t = threadIdx.x;
#pragma unroll
    for (int m = 0; m < NFIELD * 8; ++m)
        if (t == m) s_coef[m] = A.coef[m >> 3][m & 7];
    int x, y;
    const bool act = fused_column<TX, TY>(t, x, y);
    const bool own = __builtin_amdgcn_readfirstlane(t >> 6) < TY;  // the tile's waves
    const int i = i0 + x, j = j0 + y;
    const bool in = act && i >= 0 && i < nx && j >= 0 && j < ny;
    const unsigned oc = in ? (unsigned)(i + sy * j) * (unsigned)sizeof(T) : kOOB;
    const unsigned ow = own ? oc : kOOB;  // own-tile samples only
    const int br = F::b_index(x, y), bw = act ? br : F::NB;
    const int er = F::e_index(x, y), ew = act ? er : F::NE;
    const int om = y * MX + x, mw = own ? om : F::NM;

    // ring cells of the old-state planes and of the mu planes
    const Slot hxx = ring_slot<T, TX, TY, -3, TX + 4, -2, TY + 2, 320>(t, i0, j0, nx, ny, sy);
    const Slot hyy = ring_slot<T, TX, TY, -2, TX + 2, -3, TY + 4, 256>(t, i0, j0, nx, ny, sy);
    const Slot hxy = ring_slot<T, TX, TY, -4, TX + 3, -4, TY + 3, 0>(t, i0, j0, nx, ny, sy);
    const Slot hxz = ring_slot<T, TX, TY, -4, TX + 3, -2, TY + 2, 384>(t, i0, j0, nx, ny, sy);
    const Slot hyz = ring_slot<T, TX, TY, -2, TX + 2, -4, TY + 3, 512>(t, i0, j0, nx, ny, sy);
    const Slot hr = ring_slot<T, TX, TY, -2, TX + 3, -2, TY + 3, 448>(t, i0, j0, nx, ny, sy);
    const Slot hm = mu_slot<T, TX, TY, 640>(t, i0, j0, nx, ny, sy);

    const T rdx = A.rdx, rdy = A.rdy, rdz = A.rdz, dt = A.dt;
    const T s = A.wavelet ? sload(A.wavelet, A.n) : T(0);
    const T gxh = in ? A.gx[1][i] : T(0), gxi = in ? A.gx[0][i] : T(0);
    const T gyh = in ? A.gy[1][j] : T(0), gyi = in ? A.gy[0][j] : T(0);
    const bool mvx = in && i <= nx - 2, mvy = in && j <= ny - 2;
    const bool pxy = i <= nx - 2 && j <= ny - 2, pxz = i <= nx - 2, pyz = j <= ny - 2;

    // source tap of component q at (i, j, k) (-1: none) and its coefficient; srcw: a tap
    // of some component lies in this workgroup's columns and planes (uniform)
    auto tap = [&](int q, int kk) -> int {
        const unsigned a = (unsigned)(i - A.origin[0][stag(q, 0)]), b = (unsigned)(j - A.origin[1][stag(q, 1)]);
        const unsigned d = (unsigned)(kk - A.origin[2][stag(q, 2)]);
        return (((A.mask >> q) & 1) && a < 2u && b < 2u && d < 2u) ? (int)(a + 2u * b + 4u * d) : -1;
    };
    auto coef = [&](int q, int tp) -> T { return tp >= 0 ? s_coef[q * 8 + (tp & 7)] : T(0); };
    bool srcw = A.mask != 0 && A.wavelet != nullptr;
    {
        const int lo[3] = {i0 - 2, j0 - 2, k0 - 2}, hi[3] = {i0 + TX + 1, j0 + TY + 1, k1 + 1};
        for (int a = 0; a < 3; ++a) {
            const int o0 = min(A.origin[a][0], A.origin[a][1]), o1 = max(A.origin[a][0], A.origin[a][1]) + 1;
            srcw = srcw && o1 >= lo[a] && o0 <= hi[a];
        }
    }

    // descriptors of the inputs over the sweep's planes; offset of plane kk (kSkip: skipped)
    const Window w = window<T>(k0, k1, nz, sz);
    rsrc_t Fin[NFIELD];
#pragma unroll
    for (int q = 0; q < NFIELD; ++q) Fin[q] = wfield(A.in + q * fs, w);
    const rsrc_t Flam = wfield(A.lam, w), Fmu = wfield(A.mu, w), Frho = wfield(A.rho, w);
    auto po = [&](int kk, bool ok) -> unsigned { return wplane(w, kk, ok); };
    auto stq = [&](int q, int kk, bool ok, unsigned off, T v) { st(wfield(A.out + q * fs, w), off + po(kk, ok), v); };
    // old sxz / syz / szz at plane kk, with the odd images above a free surface
    auto zsh = [&](int q, int kk, bool ok) -> T {
        if (FS && kk < 0) return -ld<T>(Fin[q], oc + po(-1 - kk, ok));
        return ld<T>(Fin[q], oc + po(kk, ok));
    };
    auto zzz = [&](int kk, bool ok) -> T {
        if (FS && kk < 0) return -ld<T>(Fin[SZZ], oc + po(-kk, ok));
        return ld<T>(Fin[SZZ], oc + po(kk, ok));
    };

    // loads of velocity plane q: old stress of plane q (own column and ring), queue heads,
    // old velocity, rho; lambda of stress plane q - 2 and mu of plane q - 1
    struct Pre {
        T xx, yy, xy, xz1, yz1, zz2, r1, vx, vy, vz, hxx, hyy, hxy, hxz, hyz, hr, lam, mu, hmu;
    };
    auto load = [&](int q, bool ok, Pre &P) {
        const unsigned pq = po(q, ok), o = oc + pq;
        P.xx = ld<T>(Fin[SXX], o);
        P.yy = ld<T>(Fin[SYY], o);
        P.xy = ld<T>(Fin[SXY], o);
        P.xz1 = zsh(SXZ, q + 1, ok);
        P.yz1 = zsh(SYZ, q + 1, ok);
        P.zz2 = zzz(q + 2, ok);
        P.r1 = ld<T>(Frho, oc + po(q + 1, ok));
        P.vx = ld<T>(Fin[VX], o);
        P.vy = ld<T>(Fin[VY], o);
        P.vz = ld<T>(Fin[VZ], o);
        P.hxx = ld<T>(Fin[SXX], hxx.off + pq);
        P.hyy = ld<T>(Fin[SYY], hyy.off + pq);
        P.hxy = ld<T>(Fin[SXY], hxy.off + pq);
        P.hxz = ld<T>(Fin[SXZ], hxz.off + pq);
        P.hyz = ld<T>(Fin[SYZ], hyz.off + pq);
        P.hr = ld<T>(Frho, hr.off + pq);
        P.lam = ld<T>(Flam, ow + po(q - 2, ok));
        const unsigned pm = po(q - 1, ok);
        P.mu = ld<T>(Fmu, ow + pm);
        P.hmu = ld<T>(Fmu, hm.off + pm);
    };

    // register queues (entry m holds plane p - 2 + m of the current velocity plane p)
    const int p0 = k0 - 2;
    T qxz[4], qyz[4], qzz[5];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        qxz[m] = zsh(SXZ, p0 - 2 + m, true);
        qyz[m] = zsh(SYZ, p0 - 2 + m, true);
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) qzz[m] = zzz(p0 - 2 + m, true);
    qxz[3] = qyz[3] = qzz[4] = T(0);
    T dxx[3] = {T(0), T(0), T(0)}, dyy[3] = {T(0), T(0), T(0)}, dxy[3] = {T(0), T(0), T(0)};  // planes p-2, p-1, p
    T qvx[4] = {T(0), T(0), T(0), T(0)}, qvy[4] = {T(0), T(0), T(0), T(0)};  // new v, planes p-3 .. p
    T qvz[5] = {T(0), T(0), T(0), T(0), T(0)};                               // new vz, planes p-4 .. p
    T r0 = ld<T>(Frho, oc + po(p0, true)), r1 = T(0);
    Pre P;
    load(p0, true, P);

    for (int it = 0, p = p0; p < k1 + 2; ++it, ++p) {
        qxz[3] = P.xz1;
        qyz[3] = P.yz1;
        qzz[4] = P.zz2;
        r1 = P.r1;
        dxx[2] = P.xx;
        dyy[2] = P.yy;
        dxy[2] = P.xy;
        const T vx0 = P.vx, vy0 = P.vy, vz0 = P.vz, l = P.lam;
        T *Lxx = s_old[it & 1][0], *Lyy = s_old[it & 1][1], *Lxy = s_old[it & 1][2];
        T *Lxz = s_old[it & 1][3], *Lyz = s_old[it & 1][4], *Lr = s_old[it & 1][5];
        T *M1 = s_mu[it % 3];              // mu of plane k + 1 = p - 1
        const T *M0 = s_mu[(it + 2) % 3];  // mu of plane k
        Lxx[bw] = dxx[2];
        Lyy[bw] = dyy[2];
        Lxy[bw] = dxy[2];
        Lxz[bw] = qxz[2];
        Lyz[bw] = qyz[2];
        Lr[bw] = r0;
        Lxx[hxx.lds] = P.hxx;
        Lyy[hyy.lds] = P.hyy;
        Lxy[hxy.lds] = P.hxy;
        Lxz[hxz.lds] = P.hxz;
        Lyz[hyz.lds] = P.hyz;
        Lr[hr.lds] = P.hr;
        M1[mw] = P.mu;
        M1[hm.lds] = P.hmu;
        load(p + 1, p + 1 < k1 + 2, P);
        const bool pin = p >= 0 && p < nz;
        const T gz_i = pin ? sload(A.gz[0], p) : T(0), gz_h = pin ? sload(A.gz[1], p) : T(0);
        const int k = p - 2;
        const bool sdo = own && k >= k0;  // stress plane k of this chunk (k < k1 always)
        const T gk_i = k >= k0 ? sload(A.gz[0], k) : T(0), gk_h = k >= k0 ? sload(A.gz[1], k) : T(0);
        __syncthreads();

        // new velocity at plane p (zero outside the grid and at pinned samples)
        const bool vstore = own && p >= k0 && p < k1;
        T vxn, vyn, vzn;
        {
            const T d = dstag(Lxx[br + 1], Lxx[br], Lxx[br + 2], Lxx[br - 1], rdx)
                      + dstag(Lxy[br], Lxy[br - BX], Lxy[br + BX], Lxy[br - 2 * BX], rdy)
                      + dstag(qxz[2], qxz[1], qxz[3], qxz[0], rdz);
            const T bb = buoy(r0, Lr[br + 1]);
            T v = vx0 + dt * bb * d;
            if (srcw) v += bb * coef(VX, tap(VX, p)) * s;
            v = v * (gxh * gyi * gz_i);
            vxn = (pin && mvx) ? v : T(0);
        }
        {
            const T d = dstag(Lxy[br], Lxy[br - 1], Lxy[br + 1], Lxy[br - 2], rdx)
                      + dstag(Lyy[br + BX], Lyy[br], Lyy[br + 2 * BX], Lyy[br - BX], rdy)
                      + dstag(qyz[2], qyz[1], qyz[3], qyz[0], rdz);
            const T bb = buoy(r0, Lr[br + BX]);
            T v = vy0 + dt * bb * d;
            if (srcw) v += bb * coef(VY, tap(VY, p)) * s;
            v = v * (gxi * gyh * gz_i);
            vyn = (pin && mvy) ? v : T(0);
        }
        {
            const T d = dstag(Lxz[br], Lxz[br - 1], Lxz[br + 1], Lxz[br - 2], rdx)
                      + dstag(Lyz[br], Lyz[br - BX], Lyz[br + BX], Lyz[br - 2 * BX], rdy)
                      + dstag(qzz[3], qzz[2], qzz[4], qzz[1], rdz);
            const T bb = buoy(r0, r1);
            T v = vz0 + dt * bb * d;
            if (srcw) v += bb * coef(VZ, tap(VZ, p)) * s;
            v = v * (gxi * gyi * gz_h);
            vzn = (in && p >= 0 && p <= nz - 2) ? v : T(0);
        }
        s_v[it % 3][0][ew] = vxn;
        s_v[it % 3][1][ew] = vyn;
        s_v[it % 3][2][ew] = vzn;
        stq(VX, p, vstore, ow, vxn);
        stq(VY, p, vstore, ow, vyn);
        stq(VZ, p, vstore, ow, vzn);
        qvx[0] = qvx[1]; qvx[1] = qvx[2]; qvx[2] = qvx[3]; qvx[3] = vxn;
        qvy[0] = qvy[1]; qvy[1] = qvy[2]; qvy[2] = qvy[3]; qvy[3] = vyn;
        qvz[0] = qvz[1]; qvz[1] = qvz[2]; qvz[2] = qvz[3]; qvz[3] = qvz[4]; qvz[4] = vzn;

        // new stress at plane k from the new velocity of planes k-2 .. k+2
        if (sdo) {
            const T *Vx = s_v[(it + 1) % 3][0], *Vy = s_v[(it + 1) % 3][1], *Vz = s_v[(it + 1) % 3][2];
            const T mm = M0[om];
            const T exx = dstag(Vx[er], Vx[er - 1], Vx[er + 1], Vx[er - 2], rdx);
            const T eyy = dstag(Vy[er], Vy[er - EX], Vy[er + EX], Vy[er - 2 * EX], rdy);
            T ezz;
            if (FS && k == 0) ezz = -l / (l + T(2) * mm) * (exx + eyy);
            else if (FS && k == 1) ezz = (qvz[2] - qvz[1]) * rdz;
            else ezz = dstag(qvz[2], qvz[1], qvz[3], qvz[0], rdz);
            const T gn = gxi * gyi * gk_i;
            const T exy = dstag(Vx[er + EX], Vx[er], Vx[er + 2 * EX], Vx[er - EX], rdy)
                        + dstag(Vy[er + 1], Vy[er], Vy[er + 2], Vy[er - 1], rdx);
            const T dzvx = (FS && k == 0) ? (qvx[2] - qvx[1]) * rdz : dstag(qvx[2], qvx[1], qvx[3], qvx[0], rdz);
            const T exz = dzvx + dstag(Vz[er + 1], Vz[er], Vz[er + 2], Vz[er - 1], rdx);
            const T dzvy = (FS && k == 0) ? (qvy[2] - qvy[1]) * rdz : dstag(qvy[2], qvy[1], qvy[3], qvy[0], rdz);
            const T eyz = dzvy + dstag(Vz[er + EX], Vz[er], Vz[er + 2 * EX], Vz[er - EX], rdy);
            const T g_xy = gxh * gyh * gk_i, g_xz = gxh * gyi * gk_h, g_yz = gxi * gyh * gk_h;
            const T tr = exx + eyy + ezz;
            T nxx = dxx[0] + dt * (l * tr + T(2) * mm * exx);
            T nyy = dyy[0] + dt * (l * tr + T(2) * mm * eyy);
            T nzz = qzz[0] + dt * (l * tr + T(2) * mm * ezz);
            if (srcw) {
                const int tp = tap(SXX, k);
                nxx += coef(SXX, tp) * s;
                nyy += coef(SYY, tp) * s;
                nzz += coef(SZZ, tp) * s;
            }
            stq(SXX, k, true, ow, nxx * gn);
            stq(SYY, k, true, ow, nyy * gn);
            stq(SZZ, k, true, ow, (FS && k == 0) ? T(0) : nzz * gn);
            {
                const T mxy = ((M0[om] + M0[om + 1]) + (M0[om + MX] + M0[om + MX + 1])) / T(4);
                T v = dxy[0] + dt * mxy * exy;
                if (srcw) v += coef(SXY, tap(SXY, k)) * s;
                stq(SXY, k, true, ow, pxy ? v * g_xy : T(0));
            }
            {
                const T mxz = ((M0[om] + M0[om + 1]) + (M1[om] + M1[om + 1])) / T(4);
                T v = qxz[0] + dt * mxz * exz;
                if (srcw) v += coef(SXZ, tap(SXZ, k)) * s;
                stq(SXZ, k, true, ow, (pxz && k <= nz - 2) ? v * g_xz : T(0));
            }
            {
                const T myz = ((M0[om] + M0[om + MX]) + (M1[om] + M1[om + MX])) / T(4);
                T v = qyz[0] + dt * myz * eyz;
                if (srcw) v += coef(SYZ, tap(SYZ, k)) * s;
                stq(SYZ, k, true, ow, (pyz && k <= nz - 2) ? v * g_yz : T(0));
            }
        }
        qxz[0] = qxz[1]; qxz[1] = qxz[2]; qxz[2] = qxz[3];
        qyz[0] = qyz[1]; qyz[1] = qyz[2]; qyz[2] = qyz[3];
        qzz[0] = qzz[1]; qzz[1] = qzz[2]; qzz[2] = qzz[3]; qzz[3] = qzz[4];
        dxx[0] = dxx[1]; dxx[1] = dxx[2];
        dyy[0] = dyy[1]; dyy[1] = dyy[2];
        dxy[0] = dxy[1]; dxy[1] = dxy[2];
        r0 = r1;
    }
}

template <typename T, int TX, int TY, bool FS>
__global__ void __launch_bounds__((Fused<TX, TY>::NT)) step_fused(FusedArgs<T> A, TileMap tm)
{
    int i0, j0, k0, k1;
    tile_coords(tm, xcd_remap(blockIdx.x, gridDim.x), i0, j0, k0, k1, TX, TY, A.nz);
    fused_body<T, TX, TY, FS>(A, i0, j0, k0, k1);
}

} // namespace fd3d
