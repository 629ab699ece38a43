// Tiled forward passes: LDS-staged (x, y) halo planes, register-streamed z sweep.
//
// A workgroup owns a TX x TY column tile and sweeps a chunk of z planes.  Per plane,
// every field is read from HBM once: the owner thread loads its own sample, a few
// threads load the x/y halo of the LDS plane, and the z neighbours come from a
// per-thread register queue.  All loads of plane k+1 are issued before the compute of
// plane k (software pipelining), so one barrier per plane is the only stall.  LDS
// planes are double-buffered (a ring of three for the two-plane mu window).
//
// Memory access is branch-free: fields are read and written through raw buffer
// descriptors, one per z plane.  A sample outside the grid gets an out-of-range byte
// offset (the load returns 0, the store is dropped) and a plane outside the chunk gets
// an empty descriptor, so the loop body has no divergent memory operations and the
// compiler can wait on exactly the loads each step needs.  Uniform per-plane values
// (damping profile along z, wavelet sample) come through the scalar cache.
//
// Workgroup ids are remapped so that each XCD receives a contiguous block of tiles
// (hardware dispatches consecutive ids round-robin over the 8 XCDs), which keeps the
// halo rows shared by neighbouring tiles inside one XCD's L2.
#pragma once

#include "common.h"

namespace fd3d {

// Tile decomposition of a grid: ntx x nty column tiles, nzc z-chunks of zc planes.
struct TileMap {
    int ntx, nty, nzc, zc;
};

typedef __amdgpu_buffer_rsrc_t rsrc_t;

constexpr unsigned kOOB = 0x80000000u;  // byte offset past every plane (< 2 GiB per plane)
constexpr int kRsrcWord3 = 0x00020000;  // raw buffer descriptor, gfx9-family word 3

// Descriptor over plane kk of field f; empty (every access out of range) unless ok.
template <typename T>
__device__ __forceinline__ rsrc_t plane(const T *f, int kk, long sz, bool ok)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)(f + (ok ? kk * sz : 0)), (short)0,
                                             ok ? (int)(sz * (long)sizeof(T)) : 0, kRsrcWord3);
}

// The planes one z sweep of a workgroup touches, [max(k0-4, 0), min(k1+4, nz)): one
// descriptor per field covers them and a plane is selected by the lane offset, so a
// plane costs a vector add per distinct offset instead of a scalar descriptor per field.
// For windows of at most 1 GiB the offsets need no selects: kOOB (a sample outside the
// grid) plus any plane offset stays out of range, a skipped plane gets the plane offset
// kSkip, and a plane below the window wraps around to the top of the 32-bit range.
constexpr unsigned kSkip = 0x40000000u;
constexpr long kMaxWindowBytes = 1L << 30;

struct Window {
    int b0;       // first plane
    int bytes;    // descriptor size
    unsigned pb;  // bytes per plane
    long sz;      // samples per plane
};

template <typename T> __device__ __forceinline__ Window window(int k0, int k1, int nz, long sz)
{
    Window w;
    w.b0 = max(k0 - 4, 0);
    w.pb = (unsigned)(sz * (long)sizeof(T));
    w.bytes = (int)((long)(min(k1 + 4, nz) - w.b0) * (long)w.pb);
    w.sz = sz;
    return w;
}

// Descriptor of field f over the window (empty unless ok).
template <typename T> __device__ __forceinline__ rsrc_t wfield(const T *f, const Window &w, bool ok = true)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)(f + (ok ? w.b0 * w.sz : 0)), (short)0, ok ? w.bytes : 0,
                                             kRsrcWord3);
}

// Offset of plane kk in the window (kSkip: every sample out of range).
__device__ __forceinline__ unsigned wplane(const Window &w, int kk, bool ok)
{
    return ok ? (unsigned)(kk - w.b0) * w.pb : kSkip;
}

constexpr int kNT = 2;  // buffer instruction cache policy: nt (non-temporal)

__device__ __forceinline__ float bload(rsrc_t r, unsigned off, float)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ double bload(rsrc_t r, unsigned off, double)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <typename T> __device__ __forceinline__ T ld(rsrc_t r, unsigned off) { return bload(r, off, T(0)); }

// Loads of the model arrays, and the gradient's stored velocities and accumulators, under
// a cache policy chosen per launch (the NTP template argument of the tile bodies: 0 plain,
// 1 streaming all of them, 2 streaming the gradient's data but not the model; see
// stream_model on the host): streamed accesses carry the non-temporal bit (nt = 2 on
// gfx950).  The model arrays are read by one pass per step each, the recompute's
// v^{n+1/2} only by the adjoint, many steps later, and an accumulator by one pass per
// step; on grids whose working set exceeds the 256 MB Infinity Cache, streaming them
// leaves more of it to the fields the next pass reads (256^3 forward 43.6-43.9 ->
// 44.7-45.0 Gcell-steps/s, stress pass 0.213 -> 0.204 ms; gradient -3.6 % per shot; the
// stored velocities' and accumulators' stores and loads a further -3.2 %).  On grids that
// fit the plain policy keeps the model cached between uses; batched gradient launches,
// whose shots share one model, stream the gradient's data only (-2.9 % per shot).
template <int AUX> __device__ __forceinline__ float bload_p(rsrc_t r, unsigned off, float)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, AUX));
}
template <int AUX> __device__ __forceinline__ double bload_p(rsrc_t r, unsigned off, double)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, AUX));
}
template <bool NTP, typename T> __device__ __forceinline__ T ldm(rsrc_t r, unsigned off)
{
    return bload_p<NTP ? kNT : 0>(r, off, T(0));
}

__device__ __forceinline__ void st(rsrc_t r, unsigned off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st(rsrc_t r, unsigned off, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}
template <bool NTP> __device__ __forceinline__ void stm(rsrc_t r, unsigned off, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, NTP ? kNT : 0);
}
template <bool NTP> __device__ __forceinline__ void stm(rsrc_t r, unsigned off, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, NTP ? kNT : 0);
}

// Uniform value through the scalar cache.
template <typename T> __device__ __forceinline__ T sload(const T *p, int idx)
{
    typedef const __attribute__((address_space(4))) T cT;
    return ((cT *)p)[idx];
}

__device__ __forceinline__ int xcd_remap(int b, int nwg)
{
    const int q = nwg >> 3, r = nwg & 7;
    const int x = b & 7, local = b >> 3;
    return x * q + (x < r ? x : r) + local;
}

// One halo element of an LDS plane owned by this thread: LDS index (the array's dummy
// slot when the thread has none) and in-plane byte offset (kOOB outside the grid).
struct Slot {
    int lds;
    unsigned off;
};

// x-halo element e of a plane of width TX+LEFT+RIGHT whose TY core rows start at row OY.
template <typename T, int TX, int TY, int LEFT, int RIGHT, int OY>
__device__ __forceinline__ Slot xslot(int e, int i0, int j0, int nx, int ny, int sy, int dummy)
{
    constexpr int W = TX + LEFT + RIGHT;
    constexpr int NH = (LEFT + RIGHT) * TY;
    Slot s{dummy, kOOB};
    if (e < NH) {
        const int row = e / (LEFT + RIGHT), c = e % (LEFT + RIGHT);
        const int col = c < LEFT ? c : TX + c;
        const int gi = i0 - LEFT + col, gj = j0 + row;
        s.lds = (row + OY) * W + col;
        if (gi >= 0 && gi < nx && gj < ny) s.off = (unsigned)(gi + sy * gj) * (unsigned)sizeof(T);
    }
    return s;
}

// y-halo element e of a plane with TOP/BOT halo rows over the TX core columns at column OX.
template <typename T, int TX, int TY, int TOP, int BOT, int OX, int W>
__device__ __forceinline__ Slot yslot(int e, int i0, int j0, int nx, int ny, int sy, int dummy)
{
    constexpr int NH = (TOP + BOT) * TX;
    Slot s{dummy, kOOB};
    if (e < NH) {
        const int r = e / TX, col = e % TX;
        const int row = r < TOP ? r : TY + r;
        const int gi = i0 + col, gj = j0 - TOP + row;
        s.lds = row * W + col + OX;
        if (gi < nx && gj >= 0 && gj < ny) s.off = (unsigned)(gi + sy * gj) * (unsigned)sizeof(T);
    }
    return s;
}

// Bottom-right corner element of a (+1, +1) plane, owned by one thread.
template <typename T, int TX, int TY>
__device__ __forceinline__ Slot cslot(bool mine, int i0, int j0, int nx, int ny, int sy, int dummy)
{
    Slot s{dummy, kOOB};
    if (mine) {
        s.lds = TY * (TX + 1) + TX;
        const int gi = i0 + TX, gj = j0 + TY;
        if (gi < nx && gj < ny) s.off = (unsigned)(gi + sy * gj) * (unsigned)sizeof(T);
    }
    return s;
}

// Whether any lane of the wave holds a halo slot of a field (wave-uniform): waves without
// one skip that field's halo load and LDS store (the halo threads are the first and the
// last ones of the workgroup, so most waves hold none of the x-halo slots).
__device__ __forceinline__ bool wave_holds(const Slot &s, int dummy)
{
    return __builtin_amdgcn_ballot_w64(s.lds != dummy) != 0;
}

// The halo slot of a field that this thread actually holds, when the x-halo threads (the
// last ones), the y-halo threads (the first ones) and the corner thread are disjoint,
// which holds for every supported tile shape (3 TX + 3 TY < TX TY).
__device__ __forceinline__ Slot either(const Slot &a, const Slot &b, int dummy) { return a.lds != dummy ? a : b; }

__device__ __forceinline__ void tile_coords(const TileMap &tm, int t, int &i0, int &j0, int &k0, int &k1, int TX,
                                            int TY, int nz)
{
    const int tz = t % tm.nzc;
    t /= tm.nzc;
    const int bx = t % tm.ntx, by = t / tm.ntx;
    i0 = bx * TX;
    j0 = by * TY;
    k0 = tz * tm.zc;
    k1 = min(k0 + tm.zc, nz);
}

// What a tile body computes.  kFwd: the forward pass; kFwdSave (velocity-type body): the
// forward velocity pass that writes v^{n+1/2} through the grid's save pointers instead of
// over v^{n-1/2} (the gradient's segment recompute, whose steps read v^{n-1/2} from the
// previous step's slot).  For the velocity-type body, kAdjA: the adjoint velocity
// update A_v = U' - dt D_S(X) (X = C G_s A_s, precomputed; U' = Y' rho_eff, the damped
// adjoint velocity of the step after, held as Y'), then at the own sample the buoyancy
// gradient's share g_b -= v^{n+1/2} rho_eff dt D_S(X) and Y = b G_v A_v, written over Y'
// (A_v itself is not stored).  For the stress-type body, kAdjA: gradients of C from
// E(v^{n+1/2}) and T = G_s A_s, X = C T; kAdjB: A_s <- G_s A_s - dt E(Y); kAdjM: kAdjB of
// the step after (Y of that step in io.y) then kAdjA of this step, in one sweep (the
// updated A_s is stored and feeds T directly).  The adjoint modes read and write the
// arrays named by the grid (f[] pointing at the adjoint, stored or scratch fields) and by
// TileIO.  The Born (tangent-linear) modes step the background and the perturbation in
// one sweep: kBornV is the background's forward velocity update, then the perturbation's,
// whose velocity (io.out[0..2]) first takes the source term dt db (D_S sigma) + db c s
// formed from the background's derivatives (db = -b^2 drho_eff, drho in io.acc[0]) and
// then its own forward update from its stress (io.pin[0..5], staged like the
// background's); kBornS is the background's forward stress update, then the perturbation's
// stress (io.out[0..5]) takes dt (dC E v) (dlam, dmu in io.acc[0], io.acc[1]; no damping,
// no source) and then its own forward update from its velocity (io.pin[0..2]).  Each
// perturbation sample sees the operations of a separate source pass followed by a forward
// pass, in that order.
enum { kFwd = 0, kAdjA = 1, kAdjB = 2, kFwdSave = 3, kBornV = 4, kBornS = 5, kAdjM = 6 };

// Sweep direction of each pass (true: upward, decreasing k), chosen so that a pass starts
// where the pass before it ended and finds those planes still in the last-level cache:
// forward velocity down, stress up; adjoint stress-M (and stress-A) down, velocity-A up;
// the adjoint's closing stress-B up, after the last velocity-A; Born velocity down, Born
// stress up.  A pass that sweeps up also takes its tiles in reverse order, so that when
// the tiles run in several rounds its first round covers the last round of the pass
// before.
template <int MODE> constexpr bool vel_sweeps_up() { return MODE == kAdjA; }
template <int MODE> constexpr bool stress_sweeps_up() { return MODE == kFwd || MODE == kAdjB || MODE == kBornS; }

// Waits for every outstanding memory operation of the wave (s_waitcnt with all counters
// zero).  Called once between a sweep's prologue loads and its plane loop: the compiler
// places the loop header's waits for the state of both paths into the header, and when a
// prologue load is still in flight there it puts a full vmcnt(0) at the top of every
// iteration, which then also waits for the previous plane's stores to be acknowledged
// before the next plane's loads can be issued.  With the prologue drained, each iteration
// waits only for its own plane's loads and leaves the stores in flight.
__device__ __forceinline__ void drain_loads() { __builtin_amdgcn_s_waitcnt(0); }

// Tile of workgroup b of nwg (XCD-contiguous ranges), reversed for upward passes.
__device__ __forceinline__ int tile_of(int b, int nwg, bool reverse)
{
    const int t = xcd_remap(b, nwg);
    return reverse ? nwg - 1 - t : t;
}

template <typename T> struct TileIO {
    T *out[6];  // X (stress-A), or the Born perturbation's velocity (3) or stress (6)
    T *acc[5];  // gradient accumulators: stress-A's (gl, gm, g_mu_xy, g_mu_xz, g_mu_yz),
                // velocity-A's (g_bx, g_by, g_bz); or the Born model perturbation (drho;
                // dlam, dmu)
    const T *vst[3];  // velocity-A: stored v^{n+1/2}
    const T *y[3];    // stress-M: Y of the step after
    const T *pin[6];  // Born: the perturbation's stress (velocity sweep) or velocity (stress
                      // sweep), read with halos
};

// Source coefficients of NC consecutive components starting at C0, staged in LDS when a
// tap lies in the tile (on, uniform), so that the sweep reads them with LDS loads: a
// global load inside the loop would make the wait for it also wait for the next plane's
// prefetched loads.  Visible after the sweep's first barrier.
template <typename T, int C0, int NC>
__device__ __forceinline__ void stage_coef(T *lds, const Inject<T> &src, bool on, int tid)
{
    if (on && tid < NC * 8) lds[tid] = src.coef[C0 * 8 + tid];
}

// ---------------------------------------------------------------------------------
// (V) velocity pass, tiled.  Same arithmetic per sample as vel_cell.
// CM (forward only): the medium is a coarse node grid read by trilinear samples at the
// velocity samples' own positions (CoarseAxis); the node density plane and queue are not
// read.
template <typename T, int TX, int TY, bool FS, int MODE = kFwd, bool VAC = false, int NTP = 0, bool CM = false>
__device__ __forceinline__ void vel_tile_body(const Grid<T> &G, const Inject<T> &src, int n, int i0, int j0, int k0,
                                              int k1, const TileIO<T> &io = TileIO<T>{})
{
    static_assert(!CM || MODE == kFwd, "the coarse medium is read by the forward passes only");
    static_assert(MODE == kFwd || MODE == kFwdSave || MODE == kAdjA || MODE == kBornV, "velocity-type modes");
    constexpr int NT = TX * TY;
    // LDS plane shapes: sxx x(-1,+2); sxy x(-2,+1) y(-2,+1); sxz x(-2,+1); syy y(-1,+2);
    // syz y(-2,+1); rho x(+1) y(+1) with the corner.  The last element is a dummy slot.
    constexpr int W3 = TX + 3, H3 = TY + 3, WR = TX + 1, HR = TY + 1;
    constexpr int NXX = TY * W3, NXY = H3 * W3, NXZ = TY * W3, NYY = H3 * TX, NYZ = H3 * TX, NR = HR * WR;
    __shared__ T s_xx[2][NXX + 1];
    __shared__ T s_xy[2][NXY + 1];
    __shared__ T s_xz[2][NXZ + 1];
    __shared__ T s_yy[2][NYY + 1];
    __shared__ T s_yz[2][NYZ + 1];
    __shared__ T s_r[2][NR + 1];
    constexpr bool born = MODE == kBornV;
    static_assert(!born || (!FS && !VAC && !CM), "Born: damped boundaries, node medium");
    __shared__ T s_dr[2][born ? NR + 1 : 1];  // drho plane of the Born source term
    // Born: the perturbation's stress planes, with the shapes and halo slots of the
    // background's
    __shared__ T s_pxx[2][born ? NXX + 1 : 1];
    __shared__ T s_pxy[2][born ? NXY + 1 : 1];
    __shared__ T s_pxz[2][born ? NXZ + 1 : 1];
    __shared__ T s_pyy[2][born ? NYY + 1 : 1];
    __shared__ T s_pyz[2][born ? NYZ + 1 : 1];

    const int nx = G.nx, ny = G.ny, nz = G.nz;
    const int sy = (int)G.sy;
    const long sz = G.sz;
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int i = i0 + tx, j = j0 + ty;
    const bool in = i < nx && j < ny;
    const SurfacePlanes sp = VAC ? surface_planes(G, i, j) : SurfacePlanes{0, 0, 0};  // vacuum planes of this column
    const unsigned oc = in ? (unsigned)(i + sy * j) * (unsigned)sizeof(T) : kOOB;  // own column

    // halo slots (fixed over the sweep); x-halo work on the last threads, y-halo on the first
    const int ex = NT - 1 - tid;
    const Slot hxx = xslot<T, TX, TY, 1, 2, 0>(ex, i0, j0, nx, ny, sy, NXX);
    const Slot hxy = either(xslot<T, TX, TY, 2, 1, 2>(ex, i0, j0, nx, ny, sy, NXY),
                            yslot<T, TX, TY, 2, 1, 2, W3>(tid, i0, j0, nx, ny, sy, NXY), NXY);
    const Slot hxz = xslot<T, TX, TY, 2, 1, 0>(ex, i0, j0, nx, ny, sy, NXZ);
    const Slot hyy = yslot<T, TX, TY, 1, 2, 0, TX>(tid, i0, j0, nx, ny, sy, NYY);
    const Slot hyz = yslot<T, TX, TY, 2, 1, 0, TX>(tid, i0, j0, nx, ny, sy, NYZ);
    const Slot hr = either(either(xslot<T, TX, TY, 0, 1, 0>(ex, i0, j0, nx, ny, sy, NR),
                                  yslot<T, TX, TY, 0, 1, 0, WR>(tid, i0, j0, nx, ny, sy, NR), NR),
                           cslot<T, TX, TY>(tid == NT / 2, i0, j0, nx, ny, sy, NR), NR);
    const int own_c3 = ty * W3;  // row base in the x-halo planes without y halo
    // (the coarse-medium instantiations issue every halo access: their own branches make
    // the skip cost more than it saves)
    const bool wxx = CM || wave_holds(hxx, NXX), wxy = CM || wave_holds(hxy, NXY), wxz = CM || wave_holds(hxz, NXZ);
    const bool wyy = CM || wave_holds(hyy, NYY), wyz = CM || wave_holds(hyz, NYZ), wr = CM || wave_holds(hr, NR);

    const T *fxx = G.f[SXX], *fyy = G.f[SYY], *fzz = G.f[SZZ];
    const T *fxy = G.f[SXY], *fxz = G.f[SXZ], *fyz = G.f[SYZ];
    const T *rho = G.rho;
    const T *pxx = io.pin[0], *pyy = io.pin[1], *pzz = io.pin[2];  // Born: the perturbation's stress
    const T *pxy = io.pin[3], *pxz = io.pin[4], *pyz = io.pin[5];
    const T rdx = G.rdx, rdy = G.rdy, rdz = G.rdz, dt = G.dt;
    const T s = src.on ? sload(src.wavelet, n) : T(0);
    const T gxh = in ? G.g[0][1][i] : T(0), gxi = in ? G.g[0][0][i] : T(0);
    const T gyh = in ? G.g[1][1][j] : T(0), gyi = in ? G.g[1][0][j] : T(0);
    const unsigned st_vx = (in && i <= nx - 2) ? oc : kOOB;
    const unsigned st_vy = (in && j <= ny - 2) ? oc : kOOB;
    // a force-source tap in this tile (uniform): elsewhere the source terms are skipped
    const bool srcv = src.on && (taps_in(src, VX, i0, i0 + TX, j0, j0 + TY, k0, k1) ||
                                 taps_in(src, VY, i0, i0 + TX, j0, j0 + TY, k0, k1) ||
                                 taps_in(src, VZ, i0, i0 + TX, j0, j0 + TY, k0, k1));
    __shared__ T s_coef[3 * 8];
    stage_coef<T, VX, 3>(s_coef, src, srcv, tid);
    auto cf = [&](int c, int t) -> T { return t >= 0 ? s_coef[(c - VX) * 8 + (t & 7)] : T(0); };
    constexpr bool fwd = MODE == kFwd || MODE == kFwdSave || MODE == kBornV;
    constexpr bool adj = MODE == kAdjA;
    constexpr bool use_rho = !CM;
    constexpr bool up = vel_sweeps_up<MODE>();
    static_assert(!(up && FS), "upward velocity sweeps have no free-surface images");
    const int kfirst = up ? k1 - 1 : k0;

    const Window w = window<T>(k0, k1, nz, sz);
    auto zld = [&](const T *f, int kk, bool ok) -> T { return ld<T>(wfield(f, w), oc + wplane(w, kk, ok)); };

    // z queues at the first plane (with the free-surface odd images above k = 0)
    T qxz[4], qyz[4], qzz[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int kk = kfirst - 2 + m;
        if (FS && kk < 0) {
            qxz[m] = -zld(fxz, -1 - kk, true);
            qyz[m] = -zld(fyz, -1 - kk, true);
        } else {
            qxz[m] = zld(fxz, kk, true);
            qyz[m] = zld(fyz, kk, true);
        }
        const int kz = kfirst - 1 + m;
        qzz[m] = (FS && kz < 0) ? -zld(fzz, -kz, true) : zld(fzz, kz, true);
    }
    T pqxz[4] = {}, pqyz[4] = {}, pqzz[4] = {};  // Born: the perturbation's queues
    if constexpr (born) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            pqxz[m] = zld(pxz, kfirst - 2 + m, true);
            pqyz[m] = zld(pyz, kfirst - 2 + m, true);
            pqzz[m] = zld(pzz, kfirst - 1 + m, true);
        }
    }
    T r0 = T(0), r1 = T(0);
    if constexpr (!CM) {
        r0 = ldm<NTP == 1, T>(wfield(rho, w), oc + wplane(w, kfirst, use_rho));
        r1 = ldm<NTP == 1, T>(wfield(rho, w), oc + wplane(w, kfirst + 1, use_rho));
    }
    // coarse medium: per-column coarse coordinates of the vx (i + 1/2, j), vy (i, j + 1/2)
    // and vz (i, j) columns, and the bilinear density samples of the coarse planes that
    // the current plane's z positions (k for vx, vy; k + 1/2 for vz) lie between,
    // recomputed only when those coarse planes change (a uniform branch)
    const int cmx = CM ? G.cm[0] : 0, cmxy = CM ? G.cm[0] * G.cm[1] : 0;
    CoarseAxis<T> cxn{}, cxh{}, cyn{}, cyh{};
    if constexpr (CM) {
        cxn = coarse_axis<T>(T(i), G.cs[0], G.cm[0]);
        cxh = coarse_axis<T>(T(i) + T(0.5), G.cs[0], G.cm[0]);
        cyn = coarse_axis<T>(T(j), G.cs[1], G.cm[1]);
        cyh = coarse_axis<T>(T(j) + T(0.5), G.cs[1], G.cm[1]);
    }
    int ck_int = -1, ck_half = -1;
    T cbx0 = T(0), cbx1 = T(0), cby0 = T(0), cby1 = T(0), cbz0 = T(0), cbz1 = T(0);
    T dr0 = T(0), dr1 = T(0);
    if constexpr (born) {
        dr0 = zld(io.acc[0], kfirst, true);
        dr1 = zld(io.acc[0], kfirst + 1, true);
    }

    // plane registers, loaded one plane ahead
    struct Plane {
        T cxx, cyy, cxy, vx, vy, vz, xx, xy, xz, yy, yz, r, dr, dvx, dvy, dvz;
        T s[3], gb[3];  // velocity-A: stored v^{n+1/2}, buoyancy gradients
        T qcxx, qcyy, qcxy, qxx, qxy, qxz, qyy, qyz;  // Born: the perturbation's own and halo stress
    };
    auto loadplane = [&](int kk, bool ok, Plane &P) {
        const unsigned pk = wplane(w, kk, ok), pr = wplane(w, kk, ok && use_rho), o = oc + pk;
        const rsrc_t bxx = wfield(fxx, w), byy = wfield(fyy, w), bxy = wfield(fxy, w);
        const rsrc_t bxz = wfield(fxz, w), byz = wfield(fyz, w), br = wfield(rho, w);
        if constexpr (born) {
            P.dvx = ld<T>(wfield(io.out[0], w), o);
            P.dvy = ld<T>(wfield(io.out[1], w), o);
            P.dvz = ld<T>(wfield(io.out[2], w), o);
            P.qcxx = ld<T>(wfield(pxx, w), o);
            P.qcyy = ld<T>(wfield(pyy, w), o);
            P.qcxy = ld<T>(wfield(pxy, w), o);
        }
        if constexpr (adj) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                P.s[c] = ldm<NTP != 0, T>(wfield(io.vst[c], w), o);
                P.gb[c] = ldm<NTP != 0, T>(wfield(io.acc[c], w), o);
            }
        }
        P.cxx = ld<T>(bxx, o);
        P.cyy = ld<T>(byy, o);
        P.cxy = ld<T>(bxy, o);
        P.vx = ld<T>(wfield(G.f[VX], w), o);
        P.vy = ld<T>(wfield(G.f[VY], w), o);
        P.vz = ld<T>(wfield(G.f[VZ], w), o);
        if (wxx) P.xx = ld<T>(bxx, hxx.off + pk);
        if (wxy) P.xy = ld<T>(bxy, hxy.off + pk);
        if (wxz) P.xz = ld<T>(bxz, hxz.off + pk);
        if (wyy) P.yy = ld<T>(byy, hyy.off + pk);
        if (wyz) P.yz = ld<T>(byz, hyz.off + pk);
        if constexpr (!CM) {
            if (wr) P.r = ldm<NTP == 1, T>(br, hr.off + pr);
        }
        if constexpr (born) {
            if (wr) P.dr = ld<T>(wfield(io.acc[0], w), hr.off + pr);
            if (wxx) P.qxx = ld<T>(wfield(pxx, w), hxx.off + pk);
            if (wxy) P.qxy = ld<T>(wfield(pxy, w), hxy.off + pk);
            if (wxz) P.qxz = ld<T>(wfield(pxz, w), hxz.off + pk);
            if (wyy) P.qyy = ld<T>(wfield(pyy, w), hyy.off + pk);
            if (wyz) P.qyz = ld<T>(wfield(pyz, w), hyz.off + pk);
        }
    };
    Plane P{};
    loadplane(kfirst, true, P);
    drain_loads();

    for (int it = 0; it < k1 - k0; ++it) {
        const int k = up ? k1 - 1 - it : k0 + it;
        const int b = it & 1;
        T *Lxx = s_xx[b], *Lxy = s_xy[b], *Lxz = s_xz[b], *Lyy = s_yy[b], *Lyz = s_yz[b], *Lr = s_r[b];
        // own samples and halos of plane k
        Lxx[own_c3 + tx + 1] = P.cxx;
        Lxy[(ty + 2) * W3 + tx + 2] = P.cxy;
        Lxz[own_c3 + tx + 2] = qxz[2];
        Lyy[(ty + 1) * TX + tx] = P.cyy;
        Lyz[(ty + 2) * TX + tx] = qyz[2];
        Lr[ty * WR + tx] = r0;
        if (wxx) Lxx[hxx.lds] = P.xx;
        if (wxy) Lxy[hxy.lds] = P.xy;
        if (wxz) Lxz[hxz.lds] = P.xz;
        if (wyy) Lyy[hyy.lds] = P.yy;
        if (wyz) Lyz[hyz.lds] = P.yz;
        if (wr) Lr[hr.lds] = P.r;
        T *Ldr = s_dr[b];
        T *Qxx = s_pxx[b], *Qxy = s_pxy[b], *Qxz = s_pxz[b], *Qyy = s_pyy[b], *Qyz = s_pyz[b];
        if constexpr (born) {
            Ldr[ty * WR + tx] = dr0;
            if (wr) Ldr[hr.lds] = P.dr;
            Qxx[own_c3 + tx + 1] = P.qcxx;
            Qxy[(ty + 2) * W3 + tx + 2] = P.qcxy;
            Qxz[own_c3 + tx + 2] = pqxz[2];
            Qyy[(ty + 1) * TX + tx] = P.qcyy;
            Qyz[(ty + 2) * TX + tx] = pqyz[2];
            if (wxx) Qxx[hxx.lds] = P.qxx;
            if (wxy) Qxy[hxy.lds] = P.qxy;
            if (wxz) Qxz[hxz.lds] = P.qxz;
            if (wyy) Qyy[hyy.lds] = P.qyy;
            if (wyz) Qyz[hyz.lds] = P.qyz;
        }
        const T vx0 = P.vx, vy0 = P.vy, vz0 = P.vz;
        const T bvx0 = P.dvx, bvy0 = P.dvy, bvz0 = P.dvz;  // the perturbation's velocity (kBornV)
        T st0[3], gb0[3];  // velocity-A's own-sample inputs of this plane
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            st0[c] = P.s[c];
            gb0[c] = P.gb[c];
        }
        // buoyancy at the three velocity samples: node means (Sec. 2.2.1), or the coarse
        // medium sampled at each sample's own position (its loads issued before the next
        // plane's, so that waiting for them leaves the prefetch in flight)
        T bvx_c = T(0), bvy_c = T(0), bvz_c = T(0);
        if constexpr (CM) {
            const CoarseAxis<T> zi = coarse_axis<T>(T(k), G.cs[2], G.cm[2]);
            const CoarseAxis<T> zh = coarse_axis<T>(T(k) + T(0.5), G.cs[2], G.cm[2]);
            if (zi.lo != ck_int) {
                cbx0 = coarse_bil(rho, cmx, cmxy, cxh, cyn, zi.lo);
                cbx1 = coarse_bil(rho, cmx, cmxy, cxh, cyn, zi.lo + 1);
                cby0 = coarse_bil(rho, cmx, cmxy, cxn, cyh, zi.lo);
                cby1 = coarse_bil(rho, cmx, cmxy, cxn, cyh, zi.lo + 1);
                ck_int = zi.lo;
            }
            if (zh.lo != ck_half) {
                cbz0 = coarse_bil(rho, cmx, cmxy, cxn, cyn, zh.lo);
                cbz1 = coarse_bil(rho, cmx, cmxy, cxn, cyn, zh.lo + 1);
                ck_half = zh.lo;
            }
            bvx_c = rcp_rho(lerp_w(cbx0, cbx1, zi.f));
            bvy_c = rcp_rho(lerp_w(cby0, cby1, zi.f));
            bvz_c = rcp_rho(lerp_w(cbz0, cbz1, zh.f));
        }
        // loads of the next plane of the sweep and the queue heads (skipped past the chunk)
        const bool more = it + 1 < k1 - k0;
        loadplane(up ? k - 1 : k + 1, more, P);
        const T nxz = zld(fxz, up ? k - 3 : k + 2, more), nyz = zld(fyz, up ? k - 3 : k + 2, more);
        const T nzz = zld(fzz, up ? k - 2 : k + 3, more);
        const T nr = CM ? T(0) : ldm<NTP == 1, T>(wfield(rho, w), oc + wplane(w, up ? k - 1 : k + 2, more && use_rho));
        const T ndr = born ? zld(io.acc[0], up ? k - 1 : k + 2, more) : T(0);
        const T npxz = born ? zld(pxz, up ? k - 3 : k + 2, more) : T(0);
        const T npyz = born ? zld(pyz, up ? k - 3 : k + 2, more) : T(0);
        const T npzz = born ? zld(pzz, up ? k - 2 : k + 3, more) : T(0);
        const T gz_i = sload(G.g[2][0], k), gz_h = sload(G.g[2][1], k);
        // second order next to a vacuum surface: vx, vy at integer k, vz at k + 1/2 (only in
        // the instantiations for grids with a vacuum surface)
        const bool vxo = VAC && o2_int(sp.x, k), vyo = VAC && o2_int(sp.y, k), vzo = VAC && o2_half(sp.n, k);
        __syncthreads();

        const unsigned pw = wplane(w, k, true);
        const rsrc_t ovx = wfield(G.f[VX], w), ovy = wfield(G.f[VY], w), ovz = wfield(G.f[VZ], w);
        const rsrc_t bvx = wfield(io.out[0], w), bvy = wfield(io.out[1], w), bvz = wfield(io.out[2], w);
        // velocity-A at component c's sample: y0 = Y' there, ra, rb the two densities of its
        // mean, g its damping factor, d the divergence of X; stores Y and g_b (at so)
        auto adj_v = [&](int c, rsrc_t oy, unsigned so, T y0, T ra, T rb, T g, T d) {
            const T re = (ra + rb) * T(0.5);
            const T dd = dt * d;
            st(oy, so, (g * (y0 * re - dd)) * buoy(ra, rb));
            stm<NTP != 0>(wfield(io.acc[c], w), so, gb0[c] - (st0[c] * re) * dd);
        };
        {
            const int o = own_c3 + tx + 1;
            const int ox = (ty + 2) * W3 + tx + 2;
            const T d = dstag(Lxx[o + 1], Lxx[o], Lxx[o + 2], Lxx[o - 1], rdx)
                      + dstag(Lxy[ox], Lxy[ox - W3], Lxy[ox + W3], Lxy[ox - 2 * W3], rdy)
                      + dz_or_o2(vxo, qxz[2], qxz[1], qxz[3], qxz[0], rdz);
            if constexpr (fwd) {
                const T bb = CM ? bvx_c : buoy(r0, Lr[ty * WR + tx + 1]);
                T v = vx0 + dt * bb * d;
                if (srcv) v += bb * cf(VX, tap_of(src, VX, i, j, k)) * s;
                v = v * (gxh * gyi * gz_i);
                if constexpr (MODE == kFwdSave) stm<NTP != 0>(wfield(G.save[VX], w), st_vx + pw, v);
                else st(ovx, st_vx + pw, v);
            }
            if constexpr (born) {  // the source term, then the perturbation's own update
                const T bb = buoy(r0, Lr[ty * WR + tx + 1]);
                const T db = -(bb * bb) * ((dr0 + Ldr[ty * WR + tx + 1]) * T(0.5));
                T add = dt * db * d;
                if (srcv) add += db * cf(VX, tap_of(src, VX, i, j, k)) * s;
                const T pv = bvx0 + add;
                const T pd = dstag(Qxx[o + 1], Qxx[o], Qxx[o + 2], Qxx[o - 1], rdx)
                           + dstag(Qxy[ox], Qxy[ox - W3], Qxy[ox + W3], Qxy[ox - 2 * W3], rdy)
                           + dz_or_o2(false, pqxz[2], pqxz[1], pqxz[3], pqxz[0], rdz);
                const T v = pv + dt * bb * pd;
                st(bvx, st_vx + pw, v * (gxh * gyi * gz_i));
            }
            if constexpr (adj) adj_v(0, ovx, st_vx + pw, vx0, r0, Lr[ty * WR + tx + 1], gxh * gyi * gz_i, d);
        }
        {
            const int ox = (ty + 2) * W3 + tx + 2;
            const int oy = (ty + 1) * TX + tx;
            const T d = dstag(Lxy[ox], Lxy[ox - 1], Lxy[ox + 1], Lxy[ox - 2], rdx)
                      + dstag(Lyy[oy + TX], Lyy[oy], Lyy[oy + 2 * TX], Lyy[oy - TX], rdy)
                      + dz_or_o2(vyo, qyz[2], qyz[1], qyz[3], qyz[0], rdz);
            if constexpr (fwd) {
                const T bb = CM ? bvy_c : buoy(r0, Lr[(ty + 1) * WR + tx]);
                T v = vy0 + dt * bb * d;
                if (srcv) v += bb * cf(VY, tap_of(src, VY, i, j, k)) * s;
                v = v * (gxi * gyh * gz_i);
                if constexpr (MODE == kFwdSave) stm<NTP != 0>(wfield(G.save[VY], w), st_vy + pw, v);
                else st(ovy, st_vy + pw, v);
            }
            if constexpr (born) {
                const T bb = buoy(r0, Lr[(ty + 1) * WR + tx]);
                const T db = -(bb * bb) * ((dr0 + Ldr[(ty + 1) * WR + tx]) * T(0.5));
                T add = dt * db * d;
                if (srcv) add += db * cf(VY, tap_of(src, VY, i, j, k)) * s;
                const T pv = bvy0 + add;
                const T pd = dstag(Qxy[ox], Qxy[ox - 1], Qxy[ox + 1], Qxy[ox - 2], rdx)
                           + dstag(Qyy[oy + TX], Qyy[oy], Qyy[oy + 2 * TX], Qyy[oy - TX], rdy)
                           + dz_or_o2(false, pqyz[2], pqyz[1], pqyz[3], pqyz[0], rdz);
                const T v = pv + dt * bb * pd;
                st(bvy, st_vy + pw, v * (gxi * gyh * gz_i));
            }
            if constexpr (adj) adj_v(1, ovy, st_vy + pw, vy0, r0, Lr[(ty + 1) * WR + tx], gxi * gyh * gz_i, d);
        }
        {
            const int o = own_c3 + tx + 2;
            const int oy = (ty + 2) * TX + tx;
            const T d = dstag(Lxz[o], Lxz[o - 1], Lxz[o + 1], Lxz[o - 2], rdx)
                      + dstag(Lyz[oy], Lyz[oy - TX], Lyz[oy + TX], Lyz[oy - 2 * TX], rdy)
                      + dz_or_o2(vzo, qzz[2], qzz[1], qzz[3], qzz[0], rdz);
            const unsigned st_vz = k <= nz - 2 ? oc : kOOB;
            if constexpr (fwd) {
                const T bb = CM ? bvz_c : buoy(r0, r1);
                T v = vz0 + dt * bb * d;
                if (srcv) v += bb * cf(VZ, tap_of(src, VZ, i, j, k)) * s;
                v = v * (gxi * gyi * gz_h);
                if constexpr (MODE == kFwdSave) stm<NTP != 0>(wfield(G.save[VZ], w), st_vz + pw, v);
                else st(ovz, st_vz + pw, v);
            }
            if constexpr (born) {
                const T bb = buoy(r0, r1);
                const T db = -(bb * bb) * ((dr0 + dr1) * T(0.5));
                T add = dt * db * d;
                if (srcv) add += db * cf(VZ, tap_of(src, VZ, i, j, k)) * s;
                const T pv = bvz0 + add;
                const T pd = dstag(Qxz[o], Qxz[o - 1], Qxz[o + 1], Qxz[o - 2], rdx)
                           + dstag(Qyz[oy], Qyz[oy - TX], Qyz[oy + TX], Qyz[oy - 2 * TX], rdy)
                           + dz_or_o2(false, pqzz[2], pqzz[1], pqzz[3], pqzz[0], rdz);
                const T v = pv + dt * bb * pd;
                st(bvz, st_vz + pw, v * (gxi * gyi * gz_h));
            }
            if constexpr (adj) adj_v(2, ovz, st_vz + pw, vz0, r0, r1, gxi * gyi * gz_h, d);
        }
        if constexpr (up) {
            qxz[3] = qxz[2]; qxz[2] = qxz[1]; qxz[1] = qxz[0]; qxz[0] = nxz;
            qyz[3] = qyz[2]; qyz[2] = qyz[1]; qyz[1] = qyz[0]; qyz[0] = nyz;
            qzz[3] = qzz[2]; qzz[2] = qzz[1]; qzz[1] = qzz[0]; qzz[0] = nzz;
            r1 = r0; r0 = nr;
            dr1 = dr0; dr0 = ndr;
            pqxz[3] = pqxz[2]; pqxz[2] = pqxz[1]; pqxz[1] = pqxz[0]; pqxz[0] = npxz;
            pqyz[3] = pqyz[2]; pqyz[2] = pqyz[1]; pqyz[1] = pqyz[0]; pqyz[0] = npyz;
            pqzz[3] = pqzz[2]; pqzz[2] = pqzz[1]; pqzz[1] = pqzz[0]; pqzz[0] = npzz;
        } else {
            qxz[0] = qxz[1]; qxz[1] = qxz[2]; qxz[2] = qxz[3]; qxz[3] = nxz;
            qyz[0] = qyz[1]; qyz[1] = qyz[2]; qyz[2] = qyz[3]; qyz[3] = nyz;
            qzz[0] = qzz[1]; qzz[1] = qzz[2]; qzz[2] = qzz[3]; qzz[3] = nzz;
            r0 = r1; r1 = nr;
            dr0 = dr1; dr1 = ndr;
            pqxz[0] = pqxz[1]; pqxz[1] = pqxz[2]; pqxz[2] = pqxz[3]; pqxz[3] = npxz;
            pqyz[0] = pqyz[1]; pqyz[1] = pqyz[2]; pqyz[2] = pqyz[3]; pqyz[3] = npyz;
            pqzz[0] = pqzz[1]; pqzz[1] = pqzz[2]; pqzz[2] = pqzz[3]; pqzz[3] = npzz;
        }
    }
}

// ---------------------------------------------------------------------------------
// (S) stress pass, tiled.  Same arithmetic per sample as stress_cell.
// CM (forward only): lambda, mu at the node and mu at the shear samples are trilinear
// samples of a coarse medium at each sample's own position (CoarseAxis); the node
// arrays, their halo and the mu ring are not read.
template <typename T, int TX, int TY, bool FS, int MODE = kFwd, bool VAC = false, int NTP = 0, bool CM = false>
__device__ __forceinline__ void stress_tile_body(const Grid<T> &G, const Inject<T> &src, int n, int i0, int j0,
                                                 int k0, int k1, const TileIO<T> &io = TileIO<T>{})
{
    static_assert(MODE == kFwd || MODE == kAdjA || MODE == kAdjB || MODE == kAdjM || MODE == kBornS,
                  "stress-type modes");
    constexpr bool adjm = MODE == kAdjM;
    static_assert(!adjm || (!FS && !VAC && !CM), "stress-M: damped boundaries, node medium");
    static_assert(!CM || MODE == kFwd, "the coarse medium is read by the forward passes only");
    constexpr int NT = TX * TY;
    // vx x(-2,+1) y(-1,+2); vy x(-1,+2) y(-2,+1); vz x(-1,+2) y(-1,+2); mu x(+1) y(+1) corner
    constexpr int W3 = TX + 3, H3 = TY + 3, WM = TX + 1, HM = TY + 1;
    constexpr int NV = H3 * W3, NM = HM * WM;
    __shared__ T s_vx[2][NV + 1];
    __shared__ T s_vy[2][NV + 1];
    __shared__ T s_vz[2][NV + 1];
    __shared__ T s_yx[2][adjm ? NV + 1 : 1];  // stress-M: Y, with the halos of v
    __shared__ T s_yy[2][adjm ? NV + 1 : 1];
    __shared__ T s_yz[2][adjm ? NV + 1 : 1];
    __shared__ T s_mu[3][NM + 1];
    constexpr bool bsf = MODE == kBornS;
    static_assert(!bsf || (!FS && !VAC && !CM), "Born: damped boundaries, node medium");
    __shared__ T s_dmu[3][bsf ? NM + 1 : 1];  // dmu ring of the Born stress term
    __shared__ T s_pvx[2][bsf ? NV + 1 : 1];  // Born: the perturbation's velocity planes
    __shared__ T s_pvy[2][bsf ? NV + 1 : 1];
    __shared__ T s_pvz[2][bsf ? NV + 1 : 1];

    const int nx = G.nx, ny = G.ny, nz = G.nz;
    const int sy = (int)G.sy;
    const long sz = G.sz;
    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int i = i0 + tx, j = j0 + ty;
    const bool in = i < nx && j < ny;
    const SurfacePlanes sp = VAC ? surface_planes(G, i, j) : SurfacePlanes{0, 0, 0};  // vacuum planes of this column
    const unsigned oc = in ? (unsigned)(i + sy * j) * (unsigned)sizeof(T) : kOOB;

    const int ex = NT - 1 - tid;
    const Slot hvx = either(xslot<T, TX, TY, 2, 1, 1>(ex, i0, j0, nx, ny, sy, NV),
                            yslot<T, TX, TY, 1, 2, 2, W3>(tid, i0, j0, nx, ny, sy, NV), NV);
    const Slot hvy = either(xslot<T, TX, TY, 1, 2, 2>(ex, i0, j0, nx, ny, sy, NV),
                            yslot<T, TX, TY, 2, 1, 1, W3>(tid, i0, j0, nx, ny, sy, NV), NV);
    const Slot hvz = either(xslot<T, TX, TY, 1, 2, 1>(ex, i0, j0, nx, ny, sy, NV),
                            yslot<T, TX, TY, 1, 2, 1, W3>(tid, i0, j0, nx, ny, sy, NV), NV);
    const Slot hm = either(either(xslot<T, TX, TY, 0, 1, 0>(ex, i0, j0, nx, ny, sy, NM),
                                  yslot<T, TX, TY, 0, 1, 0, WM>(tid, i0, j0, nx, ny, sy, NM), NM),
                           cslot<T, TX, TY>(tid == NT / 2, i0, j0, nx, ny, sy, NM), NM);
    // own positions in the planes
    const int ovx = (ty + 1) * W3 + tx + 2;
    const int ovy = (ty + 2) * W3 + tx + 1;
    const int ovz = (ty + 1) * W3 + tx + 1;
    const int om = ty * WM + tx;
    const bool wvx = CM || wave_holds(hvx, NV), wvy = CM || wave_holds(hvy, NV), wvz = CM || wave_holds(hvz, NV);
    const bool wm = CM || wave_holds(hm, NM);

    const T *fvx = G.f[VX], *fvy = G.f[VY], *fvz = G.f[VZ];
    const T *mu = G.mu, *lam = G.lam;
    const T *pvx = io.pin[0], *pvy = io.pin[1], *pvz = io.pin[2];  // Born: the perturbation's velocity
    const T rdx = G.rdx, rdy = G.rdy, rdz = G.rdz, dt = G.dt;
    const T s = src.on ? sload(src.wavelet, n) : T(0);
    const T gxh = in ? G.g[0][1][i] : T(0), gxi = in ? G.g[0][0][i] : T(0);
    const T gyh = in ? G.g[1][1][j] : T(0), gyi = in ? G.g[1][0][j] : T(0);
    const unsigned st_xy = (in && i <= nx - 2 && j <= ny - 2) ? oc : kOOB;
    // a moment-source tap in this tile (uniform): elsewhere the source terms are skipped
    const bool srcs = src.on && (taps_in(src, SXX, i0, i0 + TX, j0, j0 + TY, k0, k1) ||
                                 taps_in(src, SXY, i0, i0 + TX, j0, j0 + TY, k0, k1) ||
                                 taps_in(src, SXZ, i0, i0 + TX, j0, j0 + TY, k0, k1) ||
                                 taps_in(src, SYZ, i0, i0 + TX, j0, j0 + TY, k0, k1));
    __shared__ T s_coef[6 * 8];
    stage_coef<T, SXX, 6>(s_coef, src, srcs, tid);
    auto cf = [&](int c, int t) -> T { return t >= 0 ? s_coef[(c - SXX) * 8 + (t & 7)] : T(0); };
    const unsigned st_xz = (in && i <= nx - 2) ? oc : kOOB;
    const unsigned st_yz = (in && j <= ny - 2) ? oc : kOOB;
    constexpr bool fwd = MODE == kFwd || MODE == kBornS;
    constexpr bool use_model = MODE != kAdjB && !CM;
    // coarse medium: per-column coarse coordinates of the node (i, j), xy (i + 1/2, j + 1/2),
    // xz (i + 1/2, j) and yz (i, j + 1/2) columns; bilinear samples of the coarse planes
    // around z = k (lambda, mu at the node, mu at xy) and z = k + 1/2 (mu at xz, yz),
    // recomputed only when those planes change (a uniform branch)
    const int cmx = CM ? G.cm[0] : 0, cmxy = CM ? G.cm[0] * G.cm[1] : 0;
    CoarseAxis<T> cxn{}, cxh{}, cyn{}, cyh{};
    if constexpr (CM) {
        cxn = coarse_axis<T>(T(i), G.cs[0], G.cm[0]);
        cxh = coarse_axis<T>(T(i) + T(0.5), G.cs[0], G.cm[0]);
        cyn = coarse_axis<T>(T(j), G.cs[1], G.cm[1]);
        cyh = coarse_axis<T>(T(j) + T(0.5), G.cs[1], G.cm[1]);
    }
    int ck_int = -1, ck_half = -1;
    T cl0 = T(0), cl1 = T(0), cm0 = T(0), cm1 = T(0), cxy0 = T(0), cxy1 = T(0);
    T cxz0 = T(0), cxz1 = T(0), cyz0 = T(0), cyz1 = T(0);

    // upward for the forward passes and stress-B (see stress_sweeps_up); the z queues shift
    // the other way and the mu ring takes the new plane at the other end, with the same
    // arithmetic per sample in both directions
    constexpr bool up = stress_sweeps_up<MODE>();
    static_assert(!bsf || up, "the Born stress mode sweeps upward");
    static_assert(!adjm || !up, "stress-M sweeps downward");
    const int kfirst = up ? k1 - 1 : k0;

    const Window w = window<T>(k0, k1, nz, sz);
    auto zld = [&](const T *f, int kk, bool ok) -> T { return ld<T>(wfield(f, w), oc + wplane(w, kk, ok)); };

    // z queues: vx, vy at k-1..k+2; vz at k-2..k+1 (zero above k = 0: never used with FS)
    T qvx[4], qvy[4], qvz[4];
    T qyx[4] = {}, qyy[4] = {}, qyz[4] = {};  // stress-M: the same queues of Y
    T pqvx[4] = {}, pqvy[4] = {}, pqvz[4] = {};  // Born: the same queues of the perturbation
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        qvx[m] = zld(fvx, kfirst - 1 + m, true);
        qvy[m] = zld(fvy, kfirst - 1 + m, true);
        qvz[m] = zld(fvz, kfirst - 2 + m, true);
        if constexpr (bsf) {
            pqvx[m] = zld(pvx, kfirst - 1 + m, true);
            pqvy[m] = zld(pvy, kfirst - 1 + m, true);
            pqvz[m] = zld(pvz, kfirst - 2 + m, true);
        }
        if constexpr (adjm) {
            qyx[m] = zld(io.y[0], kfirst - 1 + m, true);
            qyy[m] = zld(io.y[1], kfirst - 1 + m, true);
            qyz[m] = zld(io.y[2], kfirst - 2 + m, true);
        }
    }
    // downward sweeps: the own mu of each plane is loaded once, one plane ahead, into the
    // ring, which also supplies the node's mu (the upward ring takes it from the plane loads)
    T m1 = (up || CM) ? T(0) : ldm<NTP == 1, T>(wfield(mu, w), oc + wplane(w, k0 + 1, use_model));

    struct Plane {
        T cl, cm, sxx, syy, szz, sxy, sxz, syz, hx, hy, hz, a0, a1, a2, a3, a4, dl, dm, b0, b1, b2, b3, b4, b5;
        T yhx, yhy, yhz;  // stress-M: halo samples of Y
        T phx, phy, phz;  // Born: halo samples of the perturbation's velocity
    };
    auto loadplane = [&](int kk, bool ok, Plane &P) {
        const unsigned pk = wplane(w, kk, ok), o = oc + pk, om_ = oc + wplane(w, kk, ok && use_model);
        const rsrc_t bx = wfield(fvx, w), by = wfield(fvy, w), bz = wfield(fvz, w);
        if constexpr (!CM) {
            P.cl = ldm<NTP == 1, T>(wfield(lam, w), om_);
            P.cm = up ? ldm<NTP == 1, T>(wfield(mu, w), om_) : T(0);
        } else {
            P.cl = P.cm = T(0);
        }
        if constexpr (adjm) {
            if (wvx) P.yhx = ld<T>(wfield(io.y[0], w), hvx.off + pk);
            if (wvy) P.yhy = ld<T>(wfield(io.y[1], w), hvy.off + pk);
            if (wvz) P.yhz = ld<T>(wfield(io.y[2], w), hvz.off + pk);
        }
        if constexpr (MODE == kAdjA || adjm) {
            P.a0 = ldm<NTP != 0, T>(wfield(io.acc[0], w), o);
            P.a1 = ldm<NTP != 0, T>(wfield(io.acc[1], w), o);
            P.a2 = ldm<NTP != 0, T>(wfield(io.acc[2], w), o);
            P.a3 = ldm<NTP != 0, T>(wfield(io.acc[3], w), o);
            P.a4 = ldm<NTP != 0, T>(wfield(io.acc[4], w), o);
        }
        P.sxx = ld<T>(wfield(G.f[SXX], w), o);
        P.syy = ld<T>(wfield(G.f[SYY], w), o);
        P.szz = ld<T>(wfield(G.f[SZZ], w), o);
        P.sxy = ld<T>(wfield(G.f[SXY], w), o);
        P.sxz = ld<T>(wfield(G.f[SXZ], w), o);
        P.syz = ld<T>(wfield(G.f[SYZ], w), o);
        if (wvx) P.hx = ld<T>(bx, hvx.off + pk);
        if (wvy) P.hy = ld<T>(by, hvy.off + pk);
        if (wvz) P.hz = ld<T>(bz, hvz.off + pk);
        if constexpr (bsf) {
            if (wvx) P.phx = ld<T>(wfield(pvx, w), hvx.off + pk);
            if (wvy) P.phy = ld<T>(wfield(pvy, w), hvy.off + pk);
            if (wvz) P.phz = ld<T>(wfield(pvz, w), hvz.off + pk);
            P.dl = ld<T>(wfield(io.acc[0], w), om_);
            P.dm = ld<T>(wfield(io.acc[1], w), om_);
            P.b0 = ld<T>(wfield(io.out[0], w), o);
            P.b1 = ld<T>(wfield(io.out[1], w), o);
            P.b2 = ld<T>(wfield(io.out[2], w), o);
            P.b3 = ld<T>(wfield(io.out[3], w), o);
            P.b4 = ld<T>(wfield(io.out[4], w), o);
            P.b5 = ld<T>(wfield(io.out[5], w), o);
        }
    };
    auto loadmu = [&](int kk, bool ok) -> T {
        return ldm<NTP == 1, T>(wfield(mu, w), hm.off + wplane(w, kk, ok && use_model));
    };
    auto loaddmu = [&](int kk, bool ok) -> T { return ld<T>(wfield(io.acc[1], w), hm.off + wplane(w, kk, ok)); };

    Plane P{};
    loadplane(kfirst, true, P);
    T hmu = T(0), hdmu = T(0);
    if constexpr (CM) {
        // no mu ring
    } else if constexpr (up) {
        // mu plane k1 (below the first plane) complete; plane k1 - 1's halo one ahead
        T *M = s_mu[k1 % 3];
        M[om] = zld(mu, k1, use_model);
        if (wm) {
            M[hm.lds] = loadmu(k1, true);
            hmu = loadmu(k1 - 1, true);
        }
        if constexpr (bsf) {
            T *D = s_dmu[k1 % 3];
            D[om] = zld(io.acc[1], k1, true);
            if (wm) {
                D[hm.lds] = loaddmu(k1, true);
                hdmu = loaddmu(k1 - 1, true);
            }
        }
    } else {
        T *M = s_mu[k0 % 3];
        M[om] = ldm<NTP == 1, T>(wfield(mu, w), oc + wplane(w, k0, use_model));
        if (wm) {
            M[hm.lds] = loadmu(k0, true);
            hmu = loadmu(k0 + 1, true);
        }
    }

    drain_loads();
    for (int it = 0; it < k1 - k0; ++it) {
        const int k = up ? k1 - 1 - it : k0 + it;
        const int b = it & 1;
        T *Lx = s_vx[b], *Ly = s_vy[b], *Lz = s_vz[b];
        T *M0 = s_mu[k % 3], *M1 = s_mu[(k + 1) % 3];
        T *D0 = s_dmu[bsf ? k % 3 : 0], *D1 = s_dmu[bsf ? (k + 1) % 3 : 0];
        Lx[ovx] = qvx[1];
        Ly[ovy] = qvy[1];
        Lz[ovz] = qvz[2];
        if (wvx) Lx[hvx.lds] = P.hx;
        if (wvy) Ly[hvy.lds] = P.hy;
        if (wvz) Lz[hvz.lds] = P.hz;
        T *Yx = s_yx[adjm ? b : 0], *Yy = s_yy[adjm ? b : 0], *Yz = s_yz[adjm ? b : 0];
        if constexpr (adjm) {
            Yx[ovx] = qyx[1];
            Yy[ovy] = qyy[1];
            Yz[ovz] = qyz[2];
            if (wvx) Yx[hvx.lds] = P.yhx;
            if (wvy) Yy[hvy.lds] = P.yhy;
            if (wvz) Yz[hvz.lds] = P.yhz;
        }
        T *Qx = s_pvx[bsf ? b : 0], *Qy = s_pvy[bsf ? b : 0], *Qz = s_pvz[bsf ? b : 0];
        if constexpr (bsf) {
            Qx[ovx] = pqvx[1];
            Qy[ovy] = pqvy[1];
            Qz[ovz] = pqvz[2];
            if (wvx) Qx[hvx.lds] = P.phx;
            if (wvy) Qy[hvy.lds] = P.phy;
            if (wvz) Qz[hvz.lds] = P.phz;
        }
        if constexpr (CM) {
            // the coarse samples replace the ring
        } else if constexpr (up) {  // mu plane k enters the ring (plane k + 1 is there)
            M0[om] = P.cm;
            if (wm) M0[hm.lds] = hmu;
            if constexpr (bsf) {
                D0[om] = P.dm;
                if (wm) D0[hm.lds] = hdmu;
            }
        } else {  // mu plane k + 1 enters the ring (plane k is there)
            M1[om] = m1;
            if (wm) M1[hm.lds] = hmu;
        }
        T l = P.cl, mm = (up || CM) ? P.cm : M0[om];
        // coarse medium samples of this plane (loads issued before the next plane's)
        T cmu_xy = T(0), cmu_xz = T(0), cmu_yz = T(0);
        if constexpr (CM) {
            const CoarseAxis<T> zi = coarse_axis<T>(T(k), G.cs[2], G.cm[2]);
            const CoarseAxis<T> zh = coarse_axis<T>(T(k) + T(0.5), G.cs[2], G.cm[2]);
            if (zi.lo != ck_int) {
                cl0 = coarse_bil(lam, cmx, cmxy, cxn, cyn, zi.lo);
                cl1 = coarse_bil(lam, cmx, cmxy, cxn, cyn, zi.lo + 1);
                cm0 = coarse_bil(mu, cmx, cmxy, cxn, cyn, zi.lo);
                cm1 = coarse_bil(mu, cmx, cmxy, cxn, cyn, zi.lo + 1);
                cxy0 = coarse_bil(mu, cmx, cmxy, cxh, cyh, zi.lo);
                cxy1 = coarse_bil(mu, cmx, cmxy, cxh, cyh, zi.lo + 1);
                ck_int = zi.lo;
            }
            if (zh.lo != ck_half) {
                cxz0 = coarse_bil(mu, cmx, cmxy, cxh, cyn, zh.lo);
                cxz1 = coarse_bil(mu, cmx, cmxy, cxh, cyn, zh.lo + 1);
                cyz0 = coarse_bil(mu, cmx, cmxy, cxn, cyh, zh.lo);
                cyz1 = coarse_bil(mu, cmx, cmxy, cxn, cyh, zh.lo + 1);
                ck_half = zh.lo;
            }
            l = lerp_w(cl0, cl1, zi.f);
            mm = lerp_w(cm0, cm1, zi.f);
            cmu_xy = lerp_w(cxy0, cxy1, zi.f);
            cmu_xz = lerp_w(cxz0, cxz1, zh.f);
            cmu_yz = lerp_w(cyz0, cyz1, zh.f);
        }
        const T o_xx = P.sxx, o_yy = P.syy, o_zz = P.szz, o_xy = P.sxy, o_xz = P.sxz, o_yz = P.syz;
        const T a0 = P.a0, a1 = P.a1, a2 = P.a2, a3 = P.a3, a4 = P.a4;
        const T dl = P.dl, dm = P.dm;
        const T b_xx = P.b0, b_yy = P.b1, b_zz = P.b2, b_xy = P.b3, b_xz = P.b4, b_yz = P.b5;
        // loads of the next plane of the sweep and the queue heads (skipped past the chunk)
        const int kn = up ? k - 1 : k + 1;
        const bool more = it + 1 < k1 - k0;
        loadplane(kn, more, P);
        const T nvx = zld(fvx, up ? k - 2 : k + 3, more), nvy = zld(fvy, up ? k - 2 : k + 3, more);
        const T nvz = zld(fvz, up ? k - 3 : k + 2, more);
        T npvx = T(0), npvy = T(0), npvz = T(0);
        if constexpr (bsf) {
            npvx = zld(pvx, up ? k - 2 : k + 3, more);
            npvy = zld(pvy, up ? k - 2 : k + 3, more);
            npvz = zld(pvz, up ? k - 3 : k + 2, more);
        }
        T nyx = T(0), nyy = T(0), nyz = T(0);
        if constexpr (adjm) {
            nyx = zld(io.y[0], k + 3, more);
            nyy = zld(io.y[1], k + 3, more);
            nyz = zld(io.y[2], k + 2, more);
        }
        const T nm1 = (up || CM) ? T(0) : ldm<NTP == 1, T>(wfield(mu, w), oc + wplane(w, k + 2, more && use_model));
        T nhm = T(0), nhdm = T(0);
        if (!CM && wm) nhm = loadmu(up ? k - 1 : k + 2, more);
        if (bsf && wm) nhdm = loaddmu(k - 1, more);
        const T gz_i = sload(G.g[2][0], k), gz_h = sload(G.g[2][1], k);
        // second order next to a vacuum surface: ezz at integer k, dz vx / dz vy at k + 1/2
        const bool vzo = VAC && o2_int(sp.n, k), vxo = VAC && o2_half(sp.x, k), vyo = VAC && o2_half(sp.y, k);
        const unsigned pw = wplane(w, k, true);
        __syncthreads();

        const T exx = dstag(Lx[ovx], Lx[ovx - 1], Lx[ovx + 1], Lx[ovx - 2], rdx);
        const T eyy = dstag(Ly[ovy], Ly[ovy - W3], Ly[ovy + W3], Ly[ovy - 2 * W3], rdy);
        T ezz;
        if (FS && k == 0) ezz = -l / (l + T(2) * mm) * (exx + eyy);
        else if (FS && k == 1) ezz = (qvz[2] - qvz[1]) * rdz;
        else ezz = dz_or_o2(vzo, qvz[2], qvz[1], qvz[3], qvz[0], rdz);
        const T gn = gxi * gyi * gz_i;
        const T exy = dstag(Lx[ovx + W3], Lx[ovx], Lx[ovx + 2 * W3], Lx[ovx - W3], rdy)
                    + dstag(Ly[ovy + 1], Ly[ovy], Ly[ovy + 2], Ly[ovy - 1], rdx);
        const T dzvx = dz_or_o2((FS && k == 0) || vxo, qvx[2], qvx[1], qvx[3], qvx[0], rdz);
        const T exz = dzvx + dstag(Lz[ovz + 1], Lz[ovz], Lz[ovz + 2], Lz[ovz - 1], rdx);
        const T dzvy = dz_or_o2((FS && k == 0) || vyo, qvy[2], qvy[1], qvy[3], qvy[0], rdz);
        const T eyz = dzvy + dstag(Lz[ovz + W3], Lz[ovz], Lz[ovz + 2 * W3], Lz[ovz - W3], rdy);
        const T g_xy = gxh * gyh * gz_i, g_xz = gxh * gyi * gz_h;
        const T g_yz = gxi * gyh * gz_h;
        const unsigned o_stxz = k <= nz - 2 ? st_xz : kOOB, o_styz = k <= nz - 2 ? st_yz : kOOB;
        if constexpr (fwd) {
            const T tr = exx + eyy + ezz;
            T nxx = o_xx + dt * (l * tr + T(2) * mm * exx);
            T nyy = o_yy + dt * (l * tr + T(2) * mm * eyy);
            T nzz = o_zz + dt * (l * tr + T(2) * mm * ezz);
            const T mxy = CM ? cmu_xy : ((M0[om] + M0[om + 1]) + (M0[om + WM] + M0[om + WM + 1])) / T(4);
            const T mxz = CM ? cmu_xz : ((M0[om] + M0[om + 1]) + (M1[om] + M1[om + 1])) / T(4);
            const T myz = CM ? cmu_yz : ((M0[om] + M0[om + WM]) + (M1[om] + M1[om + WM])) / T(4);
            T nxy = o_xy + dt * mxy * exy;
            T nxz = o_xz + dt * mxz * exz;
            T nyz = o_yz + dt * myz * eyz;
            if (srcs) {  // one uniform branch for all six source terms
                const int t = tap_of(src, SXX, i, j, k);
                nxx += cf(SXX, t) * s;
                nyy += cf(SYY, t) * s;
                nzz += cf(SZZ, t) * s;
                nxy += cf(SXY, tap_of(src, SXY, i, j, k)) * s;
                nxz += cf(SXZ, tap_of(src, SXZ, i, j, k)) * s;
                nyz += cf(SYZ, tap_of(src, SYZ, i, j, k)) * s;
            }
            st(wfield(G.f[SXX], w), oc + pw, nxx * gn);
            st(wfield(G.f[SYY], w), oc + pw, nyy * gn);
            st(wfield(G.f[SZZ], w), oc + pw, (FS && k == 0) ? T(0) : nzz * gn);
            st(wfield(G.f[SXY], w), st_xy + pw, nxy * g_xy);
            st(wfield(G.f[SXZ], w), o_stxz + pw, nxz * g_xz);
            st(wfield(G.f[SYZ], w), o_styz + pw, nyz * g_yz);
            if constexpr (bsf) {
                // the perturbation's stress term: dlam, dmu with the same strain rates
                // (no damping, no source) ...
                const T bxx = b_xx + dt * (dl * tr + T(2) * dm * exx);
                const T byy = b_yy + dt * (dl * tr + T(2) * dm * eyy);
                const T bzz = b_zz + dt * (dl * tr + T(2) * dm * ezz);
                const T dxy = ((D0[om] + D0[om + 1]) + (D0[om + WM] + D0[om + WM + 1])) / T(4);
                const T dxz = ((D0[om] + D0[om + 1]) + (D1[om] + D1[om + 1])) / T(4);
                const T dyz = ((D0[om] + D0[om + WM]) + (D1[om] + D1[om + WM])) / T(4);
                const T bxy = b_xy + dt * dxy * exy, bxz = b_xz + dt * dxz * exz, byz = b_yz + dt * dyz * eyz;
                // ... then its own forward update from its velocity's strain rates
                const T pexx = dstag(Qx[ovx], Qx[ovx - 1], Qx[ovx + 1], Qx[ovx - 2], rdx);
                const T peyy = dstag(Qy[ovy], Qy[ovy - W3], Qy[ovy + W3], Qy[ovy - 2 * W3], rdy);
                const T pezz = dz_or_o2(false, pqvz[2], pqvz[1], pqvz[3], pqvz[0], rdz);
                const T pexy = dstag(Qx[ovx + W3], Qx[ovx], Qx[ovx + 2 * W3], Qx[ovx - W3], rdy)
                             + dstag(Qy[ovy + 1], Qy[ovy], Qy[ovy + 2], Qy[ovy - 1], rdx);
                const T pdzvx = dz_or_o2(false, pqvx[2], pqvx[1], pqvx[3], pqvx[0], rdz);
                const T pexz = pdzvx + dstag(Qz[ovz + 1], Qz[ovz], Qz[ovz + 2], Qz[ovz - 1], rdx);
                const T pdzvy = dz_or_o2(false, pqvy[2], pqvy[1], pqvy[3], pqvy[0], rdz);
                const T peyz = pdzvy + dstag(Qz[ovz + W3], Qz[ovz], Qz[ovz + 2 * W3], Qz[ovz - W3], rdy);
                const T ptr = pexx + peyy + pezz;
                const T pxx_ = bxx + dt * (l * ptr + T(2) * mm * pexx);
                const T pyy_ = byy + dt * (l * ptr + T(2) * mm * peyy);
                const T pzz_ = bzz + dt * (l * ptr + T(2) * mm * pezz);
                const T pxy_ = bxy + dt * mxy * pexy;
                const T pxz_ = bxz + dt * mxz * pexz;
                const T pyz_ = byz + dt * myz * peyz;
                st(wfield(io.out[0], w), oc + pw, pxx_ * gn);
                st(wfield(io.out[1], w), oc + pw, pyy_ * gn);
                st(wfield(io.out[2], w), oc + pw, pzz_ * gn);
                st(wfield(io.out[3], w), st_xy + pw, pxy_ * g_xy);
                st(wfield(io.out[4], w), o_stxz + pw, pxz_ * g_xz);
                st(wfield(io.out[5], w), o_styz + pw, pyz_ * g_yz);
            }
        } else if constexpr (MODE == kAdjA || adjm) {
            // stress-M: first the adjoint stress update of the step after, A_s <- G_s A_s -
            // dt E(Y), stored, and taken as this step's A_s below
            T s_xx = o_xx, s_yy = o_yy, s_zz = o_zz, s_xy = o_xy, s_xz = o_xz, s_yz = o_yz;
            if constexpr (adjm) {
                const T yxx = dstag(Yx[ovx], Yx[ovx - 1], Yx[ovx + 1], Yx[ovx - 2], rdx);
                const T yyy = dstag(Yy[ovy], Yy[ovy - W3], Yy[ovy + W3], Yy[ovy - 2 * W3], rdy);
                const T yzz = dz_or_o2(false, qyz[2], qyz[1], qyz[3], qyz[0], rdz);
                const T yxy = dstag(Yx[ovx + W3], Yx[ovx], Yx[ovx + 2 * W3], Yx[ovx - W3], rdy)
                            + dstag(Yy[ovy + 1], Yy[ovy], Yy[ovy + 2], Yy[ovy - 1], rdx);
                const T yxz = dz_or_o2(false, qyx[2], qyx[1], qyx[3], qyx[0], rdz)
                            + dstag(Yz[ovz + 1], Yz[ovz], Yz[ovz + 2], Yz[ovz - 1], rdx);
                const T yyz = dz_or_o2(false, qyy[2], qyy[1], qyy[3], qyy[0], rdz)
                            + dstag(Yz[ovz + W3], Yz[ovz], Yz[ovz + 2 * W3], Yz[ovz - W3], rdy);
                s_xx = gn * o_xx - dt * yxx;
                s_yy = gn * o_yy - dt * yyy;
                s_zz = gn * o_zz - dt * yzz;
                s_xy = g_xy * o_xy - dt * yxy;
                s_xz = g_xz * o_xz - dt * yxz;
                s_yz = g_yz * o_yz - dt * yyz;
                st(wfield(G.f[SXX], w), oc + pw, s_xx);
                st(wfield(G.f[SYY], w), oc + pw, s_yy);
                st(wfield(G.f[SZZ], w), oc + pw, s_zz);
                st(wfield(G.f[SXY], w), st_xy + pw, s_xy);
                st(wfield(G.f[SXZ], w), o_stxz + pw, s_xz);
                st(wfield(G.f[SYZ], w), o_styz + pw, s_yz);
            }
            // gradients of C and X = C T with T = G_s A_s
            const T txx = gn * s_xx, tyy = gn * s_yy, tzz = gn * s_zz;
            const T trT = (txx + tyy) + tzz;
            stm<NTP != 0>(wfield(io.acc[0], w), oc + pw, a0 + dt * ((exx + eyy) + ezz) * trT);
            stm<NTP != 0>(wfield(io.acc[1], w), oc + pw, a1 + dt * T(2) * ((exx * txx + eyy * tyy) + ezz * tzz));
            st(wfield(io.out[0], w), oc + pw, l * trT + T(2) * mm * txx);
            st(wfield(io.out[1], w), oc + pw, l * trT + T(2) * mm * tyy);
            st(wfield(io.out[2], w), oc + pw, l * trT + T(2) * mm * tzz);
            const T txy = g_xy * s_xy, txz = g_xz * s_xz, tyz = g_yz * s_yz;
            stm<NTP != 0>(wfield(io.acc[2], w), st_xy + pw, a2 + dt * exy * txy);
            stm<NTP != 0>(wfield(io.acc[3], w), o_stxz + pw, a3 + dt * exz * txz);
            stm<NTP != 0>(wfield(io.acc[4], w), o_styz + pw, a4 + dt * eyz * tyz);
            const T mxy = CM ? cmu_xy : ((M0[om] + M0[om + 1]) + (M0[om + WM] + M0[om + WM + 1])) / T(4);
            const T mxz = CM ? cmu_xz : ((M0[om] + M0[om + 1]) + (M1[om] + M1[om + 1])) / T(4);
            const T myz = CM ? cmu_yz : ((M0[om] + M0[om + WM]) + (M1[om] + M1[om + WM])) / T(4);
            st(wfield(io.out[3], w), st_xy + pw, mxy * txy);
            st(wfield(io.out[4], w), o_stxz + pw, mxz * txz);
            st(wfield(io.out[5], w), o_styz + pw, myz * tyz);
        } else {
            // A_s <- G_s A_s - dt E(Y)
            st(wfield(G.f[SXX], w), oc + pw, gn * o_xx - dt * exx);
            st(wfield(G.f[SYY], w), oc + pw, gn * o_yy - dt * eyy);
            st(wfield(G.f[SZZ], w), oc + pw, gn * o_zz - dt * ezz);
            st(wfield(G.f[SXY], w), st_xy + pw, g_xy * o_xy - dt * exy);
            st(wfield(G.f[SXZ], w), o_stxz + pw, g_xz * o_xz - dt * exz);
            st(wfield(G.f[SYZ], w), o_styz + pw, g_yz * o_yz - dt * eyz);
        }
        if constexpr (up) {
            qvx[3] = qvx[2]; qvx[2] = qvx[1]; qvx[1] = qvx[0]; qvx[0] = nvx;
            qvy[3] = qvy[2]; qvy[2] = qvy[1]; qvy[1] = qvy[0]; qvy[0] = nvy;
            qvz[3] = qvz[2]; qvz[2] = qvz[1]; qvz[1] = qvz[0]; qvz[0] = nvz;
            pqvx[3] = pqvx[2]; pqvx[2] = pqvx[1]; pqvx[1] = pqvx[0]; pqvx[0] = npvx;
            pqvy[3] = pqvy[2]; pqvy[2] = pqvy[1]; pqvy[1] = pqvy[0]; pqvy[0] = npvy;
            pqvz[3] = pqvz[2]; pqvz[2] = pqvz[1]; pqvz[1] = pqvz[0]; pqvz[0] = npvz;
        } else {
            qvx[0] = qvx[1]; qvx[1] = qvx[2]; qvx[2] = qvx[3]; qvx[3] = nvx;
            qvy[0] = qvy[1]; qvy[1] = qvy[2]; qvy[2] = qvy[3]; qvy[3] = nvy;
            qvz[0] = qvz[1]; qvz[1] = qvz[2]; qvz[2] = qvz[3]; qvz[3] = nvz;
            if constexpr (adjm) {
                qyx[0] = qyx[1]; qyx[1] = qyx[2]; qyx[2] = qyx[3]; qyx[3] = nyx;
                qyy[0] = qyy[1]; qyy[1] = qyy[2]; qyy[2] = qyy[3]; qyy[3] = nyy;
                qyz[0] = qyz[1]; qyz[1] = qyz[2]; qyz[2] = qyz[3]; qyz[3] = nyz;
            }
            m1 = nm1;
        }
        hmu = nhm;
        hdmu = nhdm;
    }
}

// ---------------------------------------------------------------------------------
// Single-grid launches: one workgroup per tile.
template <typename T, int TX, int TY, bool FS, int MODE = kFwd, bool VAC = false, bool NTP = false, bool CM = false>
__global__ void __launch_bounds__(TX *TY) vel_tile(Grid<T> G, Inject<T> src, int n, TileMap tm)
{
    int i0, j0, k0, k1;
    tile_coords(tm, tile_of(blockIdx.x, gridDim.x, vel_sweeps_up<MODE>()), i0, j0, k0, k1, TX, TY, G.nz);
    vel_tile_body<T, TX, TY, FS, MODE, VAC, NTP, CM>(G, src, n, i0, j0, k0, k1);
}

// The stress pass only reads v^{n+1/2}, so workgroups past the grid's tiles sample the
// receivers of the step (rec.nq work items) in the same launch.
template <typename T, int TX, int TY, bool FS, int MODE = kFwd, bool VAC = false, bool NTP = false, bool CM = false>
__global__ void __launch_bounds__(TX *TY) stress_tile(Grid<T> G, Inject<T> src, int n, TileMap tm, RecJob<T> rec)
{
    const int nwg = tm.ntx * tm.nty * tm.nzc;
    if ((int)blockIdx.x >= nwg) {
        const int q = ((int)blockIdx.x - nwg) * (TX * TY) + (int)threadIdx.x;
        if (q < rec.nq) sample_receiver(rec, q, n);
        return;
    }
    int i0, j0, k0, k1;
    tile_coords(tm, tile_of(blockIdx.x, nwg, stress_sweeps_up<MODE>()), i0, j0, k0, k1, TX, TY, G.nz);
    stress_tile_body<T, TX, TY, FS, MODE, VAC, NTP, CM>(G, src, n, i0, j0, k0, k1);
}

// Born stress pass (kBornS): the background's and the perturbation's stress updates in
// one sweep; the workgroups past the tiles sample the background's receivers (rec), then
// the perturbation's (prec).
template <typename T, int TX, int TY, bool NTP = false>
__global__ void __launch_bounds__(TX *TY) stress_tile_born(Grid<T> G, Inject<T> src, int n, TileMap tm, TileIO<T> io,
                                                           RecJob<T> rec, RecJob<T> prec)
{
    const int nwg = tm.ntx * tm.nty * tm.nzc;
    if ((int)blockIdx.x >= nwg) {
        const int q = ((int)blockIdx.x - nwg) * (TX * TY) + (int)threadIdx.x;
        if (q < rec.nq) sample_receiver(rec, q, n);
        else if (q - rec.nq < prec.nq) sample_receiver(prec, q - rec.nq, n);
        return;
    }
    int i0, j0, k0, k1;
    tile_coords(tm, tile_of(blockIdx.x, nwg, stress_sweeps_up<kBornS>()), i0, j0, k0, k1, TX, TY, G.nz);
    stress_tile_body<T, TX, TY, false, kBornS, false, NTP>(G, src, n, i0, j0, k0, k1, io);
}

// Adjoint passes, one workgroup per tile (no free surface).
template <typename T, int TX, int TY, int MODE, bool NTP = false>
__global__ void __launch_bounds__(TX *TY) vel_tile_adj(Grid<T> G, Inject<T> src, int n, TileMap tm, TileIO<T> io)
{
    int i0, j0, k0, k1;
    tile_coords(tm, tile_of(blockIdx.x, gridDim.x, vel_sweeps_up<MODE>()), i0, j0, k0, k1, TX, TY, G.nz);
    vel_tile_body<T, TX, TY, false, MODE, false, NTP>(G, src, n, i0, j0, k0, k1, io);
}

template <typename T, int TX, int TY, int MODE, bool NTP = false>
__global__ void __launch_bounds__(TX *TY) stress_tile_adj(Grid<T> G, Inject<T> src, TileMap tm, TileIO<T> io)
{
    int i0, j0, k0, k1;
    tile_coords(tm, tile_of(blockIdx.x, gridDim.x, stress_sweeps_up<MODE>()), i0, j0, k0, k1, TX, TY, G.nz);
    stress_tile_body<T, TX, TY, false, MODE, false, NTP>(G, src, 0, i0, j0, k0, k1, io);
}

// ---------------------------------------------------------------------------------
// Many grids in one persistent launch.  Every shot contributes its tiles to one flat
// work list (shot-major); the list is cut into 8 contiguous chunks, one per XCD, and
// the workgroups of an XCD walk their chunk with a stride of the XCD's workgroup count.
// A workgroup loads the descriptor of the shot its tile belongs to (uniform, scalar).
template <typename T> struct ShotFwd {
    Grid<T> G;
    Inject<T> src;
    TileIO<T> io;
    TileMap tm;
    int base;  // first work item of this shot
    int alt;   // the batch's second tile shape covers this shot
};

// Work item range [lo, hi) and stride of this workgroup in the XCD-chunked order of a
// persistent grid of wgs workgroups.
__device__ __forceinline__ void work_range(int total, int wgs, int &w0, int &hi, int &stride)
{
    const int x = blockIdx.x & 7, l = blockIdx.x >> 3;
    const int per = wgs >> 3;  // wgs is a multiple of 8
    const int lo = (int)((long)total * x / 8);
    hi = (int)((long)total * (x + 1) / 8);
    w0 = lo + l;
    stride = per;
}

// Stride in ints between the .base members of consecutive descriptors.
template <typename D> constexpr int base_stride() { return (int)(sizeof(D) / sizeof(int)); }

// A batch may use a second tile shape with the same workgroup size (TX2 x TY2, 0: none)
// for the shots whose descriptor sets `alt`, so that grids of different widths all get a
// tile shape that covers them without idle columns.
template <typename T, int TX, int TY, int TX2, int TY2, bool FS, int MODE = kFwd, bool VAC = false, int NTP = 0>
__global__ void __launch_bounds__(TX *TY) vel_tile_multi(const ShotFwd<T> *__restrict__ shots, int nshot, int total,
                                                          int n)
{
    static_assert(TX2 == 0 || TX2 * TY2 == TX * TY, "both tile shapes need the same workgroup size");
    __shared__ int s_base[kMaxShots];
    load_bases(s_base, &shots[0].base, base_stride<ShotFwd<T>>(), nshot);
    int w0, hi, stride;
    work_range(total, (int)gridDim.x, w0, hi, stride);
    for (; w0 < hi; w0 += stride) {
        const int w = vel_sweeps_up<MODE>() ? total - 1 - w0 : w0;
        const int s = shot_of(s_base, nshot, w);
        const ShotFwd<T> &d = shots[s];
        const Grid<T> G = d.G;
        const Inject<T> src = d.src;
        const TileMap tm = d.tm;
        const TileIO<T> io = d.io;
        int i0, j0, k0, k1;
        if constexpr (TX2 != 0) {
            if (d.alt) {
                tile_coords(tm, w - d.base, i0, j0, k0, k1, TX2, TY2, G.nz);
                vel_tile_body<T, TX2, TY2, FS, MODE, VAC, NTP>(G, src, n, i0, j0, k0, k1, io);
                __syncthreads();
                continue;
            }
        }
        tile_coords(tm, w - d.base, i0, j0, k0, k1, TX, TY, G.nz);
        vel_tile_body<T, TX, TY, FS, MODE, VAC, NTP>(G, src, n, i0, j0, k0, k1, io);
        __syncthreads();
    }
}

// Workgroups past rec.wgs sample the receivers of the step (the stress pass only reads
// the velocity).
template <typename T, int TX, int TY, int TX2, int TY2, bool FS, int MODE = kFwd, bool VAC = false, int NTP = 0>
__global__ void __launch_bounds__(TX *TY) stress_tile_multi(const ShotFwd<T> *__restrict__ shots, int nshot, int total,
                                                          int n, RecMulti<T> rec)
{
    static_assert(TX2 == 0 || TX2 * TY2 == TX * TY, "both tile shapes need the same workgroup size");
    __shared__ int s_base[kMaxShots];
    if ((int)blockIdx.x >= rec.wgs) {
        sample_batch_receivers(rec, s_base, n);
        return;
    }
    load_bases(s_base, &shots[0].base, base_stride<ShotFwd<T>>(), nshot);
    int w0, hi, stride;
    work_range(total, rec.wgs, w0, hi, stride);
    for (; w0 < hi; w0 += stride) {
        const int w = stress_sweeps_up<MODE>() ? total - 1 - w0 : w0;
        const int s = shot_of(s_base, nshot, w);
        const ShotFwd<T> &d = shots[s];
        const Grid<T> G = d.G;
        const Inject<T> src = d.src;
        const TileMap tm = d.tm;
        const TileIO<T> io = d.io;
        int i0, j0, k0, k1;
        if constexpr (TX2 != 0) {
            if (d.alt) {
                tile_coords(tm, w - d.base, i0, j0, k0, k1, TX2, TY2, G.nz);
                stress_tile_body<T, TX2, TY2, FS, MODE, VAC, NTP>(G, src, n, i0, j0, k0, k1, io);
                __syncthreads();
                continue;
            }
        }
        tile_coords(tm, w - d.base, i0, j0, k0, k1, TX, TY, G.nz);
        stress_tile_body<T, TX, TY, FS, MODE, VAC, NTP>(G, src, n, i0, j0, k0, k1, io);
        __syncthreads();
    }
}

} // namespace fd3d
