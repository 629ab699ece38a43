// Host side of the fd3d library (C ABI of include/fd3d.h): the context, its workspace
// layout and the helpers the translation units share.
//
//   runtime.hip   contexts, options, workspace layout, model check, damping profiles,
//                 source and receiver staging, state access, the allocation-free entry
//   forward.hip   the step loop (Sec. 2.2 update order), kernel selection and its tuner
//   gradient.hip  checkpointed discrete adjoint and the FWI gradient
//   batch.hip     batches of shots, persistent launches, graphs, the batched gradient
//   born.hip      tangent-linear (Born) forward
#pragma once

#include "fd3d.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "common.h"
#include "fwd_cell.h"
#include "fwd_tile.h"
#include "adj_cell.h"
#include "util_kernels.h"

namespace fd3d {

// Message of the last failed call on this thread (fd3d_last_error).
extern thread_local std::string g_err;

// Records msg as the thread's last error and returns code.
int fail(int code, const std::string &msg);

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(FD3D_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
constexpr int kDefaultMaxRec = 4096;

inline size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

inline size_t rectap_bytes(int tsize) { return 8 * sizeof(int) + 8 * (size_t)tsize; }

// Workspace layout (byte offsets).  Two copies of the state: the fused step reads one and
// writes the other.  The fields are stored in one of two forms:
//  * separate arrays: each field x fastest and unpadded, padded to 4 KiB plus a 1 KiB
//    skew so that the nine streams of a pass do not start on the same HBM channel; the
//    model arrays are the caller's;
//  * interleaved rows: one block of kRows rows per (y, z) row index, row q holding field q
//    ([nz][ny][kRows][nx]), so that the rows of the nine fields a tile reads lie side by
//    side; the model is copied once into a block of the same shape (rows 0-2: lam, mu,
//    rho; rows 3-5: a Born perturbation), so every array of a pass has the same strides.
// A group of nine fields (a state copy, the adjoint state, a checkpoint, ...) is one block
// of interleaved rows, or nine padded arrays.
constexpr int kRows = 9;

struct Layout {
    bool rows;              // interleaved rows
    size_t field[2][NFIELD];
    size_t model;           // interleaved rows without a coarse medium: the model block
    size_t prof[3][2];
    size_t src;     // source coefficients [NFIELD][8]
    size_t rec;
    size_t colors;  // receiver order grouped by colour (tap-disjoint sets), int[max_rec]
    size_t part;
    size_t stats;
    size_t flag;
    size_t total;
    size_t field_bytes;     // bytes of one field's samples
    size_t fstep;           // bytes from one field of a group to the next
    size_t group;           // bytes of a group of up to nine fields
    size_t chunk;           // bytes from one field-sized chunk of a group to the next (copies)
};

// Workspace layout of a grid under the given options (field storage chosen by opts.layout).
Layout layout_of(int nx, int ny, int nz, const fd3d_opts &o);

int check_opts(const fd3d_opts *o);
fd3d_opts default_opts();

inline int max_rec_of(const fd3d_opts &o) { return o.max_receivers > 0 ? o.max_receivers : kDefaultMaxRec; }

// The medium arrays are a coarse grid read by trilinear samples (opts.coarse).
inline bool coarse_on(const fd3d_opts &o) { return o.coarse[0] > 0; }

} // namespace fd3d

// A context (fd3d_create): one grid, its model and options, its workspace layout, the
// host staging of sources and receivers, the kernel choice and the gradient state.
struct fd3d_ctx {
    int n[3];
    int nt;
    int tsize;
    double dx, dy, dz, dt;  // spacing per axis (m), time step (s)
    fd3d_opts opts;
    const void *lam, *mu, *rho;
    char *ws;
    size_t ws_bytes;
    fd3d::Layout L;
    double info[4];
    std::vector<unsigned char> prof_host;  // typed profiles, kept for the async upload
    std::vector<unsigned char> src_host;   // source coefficients, kept for the async upload
    std::vector<unsigned char> rec_host;   // receiver descriptors, kept for the async upload
    std::vector<int> color_host;           // receivers grouped by colour, kept for the async upload
    std::vector<int> color_off;            // colour c holds color_host[color_off[c] .. color_off[c+1])
    std::vector<unsigned char> src_dev;    // source coefficients now in the workspace
    std::vector<double> rec_dev;           // receiver positions whose descriptors are in the workspace
    bool rec_dev_valid;                    // rec_dev describes the workspace's descriptors
    hipEvent_t staged;     // marks the end of the uploads from the host staging buffers;
                           // null in a context that must create no HIP objects (its call
                           // synchronises the stream before the buffers are released)
    bool staged_pending;
    // optional per-kernel timing of the step loop
    int prof_on;
    std::vector<hipEvent_t> prof_ev;  // pairs: [2*q] before, [2*q+1] after launch q
    std::vector<int> prof_pass;       // pass of launch q
    int prof_used;
    // kernel selection for the step loop
    int variant;  // FD3D_KERNEL_CELL, FD3D_KERNEL_TILE or FD3D_KERNEL_FUSED
    int cur;      // state copy holding the current state (0 or 1)
    int tile_x;   // columns of a tile (64, 128, 256)
    int tile_y;   // rows of a tile (4, 8, 16)
    int zchunk;   // z planes per workgroup sweep
    // gradient state: checkpoints written by fd3d_forward_ckpt into a caller workspace
    const char *grad_ws;
    int grad_k;
    int grad_ready;
    int adj_done;  // an adjoint has run on grad_ws since its checkpointed forward
    int grad_y;    // the last adjoint was the tiled one: the adjoint velocity is held as Y
};

namespace fd3d {

template <typename T> Grid<T> make_grid(const fd3d_ctx *c)
{
    Grid<T> G;
    G.nx = c->n[0];
    G.ny = c->n[1];
    G.nz = c->n[2];
    G.sy = c->L.rows ? (long)kRows * G.nx : G.nx;
    G.sz = G.sy * G.ny;
    G.dt = (T)c->dt;
    G.rdx = (T)(1.0 / c->dx);
    G.rdy = (T)(1.0 / c->dy);
    G.rdz = (T)(1.0 / c->dz);
    G.ks = c->opts.vacuum_top;
    G.ksmap = (const int *)c->opts.vacuum_map;
    for (int a = 0; a < 3; ++a) {
        G.cm[a] = coarse_on(c->opts) ? c->opts.coarse[a] : 0;
        G.cs[a] = G.cm[a] ? (T)((double)(G.cm[a] - 1) / (double)(c->n[a] - 1)) : T(0);
    }
    if (c->L.model) {  // the model's copy in interleaved rows
        G.lam = (const T *)(c->ws + c->L.model);
        G.mu = (const T *)(c->ws + c->L.model + c->L.fstep);
        G.rho = (const T *)(c->ws + c->L.model + 2 * c->L.fstep);
    } else {
        G.lam = (const T *)c->lam;
        G.mu = (const T *)c->mu;
        G.rho = (const T *)c->rho;
    }
    for (int f = 0; f < NFIELD; ++f) G.f[f] = (T *)(c->ws + c->L.field[c->cur][f]);
    for (int a = 0; a < 3; ++a)
        for (int h = 0; h < 2; ++h) G.g[a][h] = (const T *)(c->ws + c->L.prof[a][h]);
    for (int f = 0; f < NFIELD; ++f) G.save[f] = nullptr;
    return G;
}

// Both state copies (the first bytes of the workspace; not the model block after them).
template <typename T> void zero_fields(fd3d_ctx *c, hipStream_t st)
{
    fill_zero<T><<<2048, 256, 0, st>>>((T *)c->ws, (long)(2 * c->L.group / sizeof(T)));
}

// Strided copy of field-shaped arrays between node arrays (x fastest, unpadded) and the
// workspace's field storage, pinned slots of component `comp` zeroed (-1: a plain copy).
template <typename T>
void copy_field(const fd3d_ctx *c, T *dst, bool dst_fields, const T *src, bool src_fields, int comp, hipStream_t st)
{
    const long nx = c->n[0], ny = c->n[1];
    const long fsy = c->L.rows ? kRows * nx : nx;
    const long dsy = dst_fields ? fsy : nx, ssy = src_fields ? fsy : nx;
    const int sx = comp >= 0 ? stag(comp, 0) : 0, sy = comp >= 0 ? stag(comp, 1) : 0, sz = comp >= 0 ? stag(comp, 2) : 0;
    copy_masked<T><<<1024, 256, 0, st>>>(dst, dsy, dsy * ny, src, ssy, ssy * ny, c->n[0], c->n[1], c->n[2], sx, sy, sz);
}

// Both state copies zeroed, for either element type.
void zero_fields_any(fd3d_ctx *c, hipStream_t st);

// Builds the source (tap boxes into inj) and the receiver descriptors and colours, and
// uploads them from the context's host staging buffers (after the previous call's
// uploads from those buffers are done).  Defined for float and double.
template <typename T>
int stage_inputs(fd3d_ctx *c, const fd3d_source *src, Inject<T> &inj, int nrec, const double *rec_pos,
                 hipStream_t st);

// Event pair around one launch when timing is on.
struct Timer {
    fd3d_ctx *c;
    hipStream_t st;
    void begin(int pass)
    {
        if (!c->prof_on) return;
        const int q = c->prof_used;
        if ((size_t)(2 * q + 2) > c->prof_ev.size()) {
            hipEvent_t a = nullptr, b = nullptr;
            (void)hipEventCreate(&a);
            (void)hipEventCreate(&b);
            c->prof_ev.push_back(a);
            c->prof_ev.push_back(b);
            c->prof_pass.push_back(pass);
        }
        c->prof_pass[q] = pass;
        (void)hipEventRecord(c->prof_ev[2 * q], st);
    }
    void end()
    {
        if (!c->prof_on) return;
        (void)hipEventRecord(c->prof_ev[2 * c->prof_used + 1], st);
        ++c->prof_used;
    }
};

inline TileMap tile_map(const fd3d_ctx *c)
{
    TileMap tm;
    tm.ntx = (c->n[0] + c->tile_x - 1) / c->tile_x;
    tm.nty = (c->n[1] + c->tile_y - 1) / c->tile_y;
    tm.zc = c->zchunk;
    tm.nzc = (c->n[2] + c->zchunk - 1) / c->zchunk;
    return tm;
}

// Supported tile shapes: 64x{4,8,16}, 128x{4,8}, 256x4 (FP64: 64x{4,8}, 128x4).
inline bool tile_supported(int tsize, int tx, int ty)
{
    if (tsize == 8) return (tx == 64 && (ty == 4 || ty == 8)) || (tx == 128 && ty == 4);
    return (tx == 64 && (ty == 4 || ty == 8 || ty == 16)) || (tx == 128 && (ty == 4 || ty == 8)) ||
           (tx == 256 && ty == 4);
}

// Calls f(TX, TY) with the tile shape as integral constants (64x8 for a shape that is
// not compiled for T).
template <typename T, typename F> decltype(auto) with_tile(int tx, int ty, F &&f)
{
    using X64 = std::integral_constant<int, 64>;
    using X128 = std::integral_constant<int, 128>;
    using X256 = std::integral_constant<int, 256>;
    using Y4 = std::integral_constant<int, 4>;
    using Y8 = std::integral_constant<int, 8>;
    using Y16 = std::integral_constant<int, 16>;
    const int key = tx * 100 + ty;
    if constexpr (sizeof(T) == 8) {
        switch (key) {
        case 6404: return f(X64{}, Y4{});
        case 12804: return f(X128{}, Y4{});
        default: return f(X64{}, Y8{});
        }
    } else {
        switch (key) {
        case 6404: return f(X64{}, Y4{});
        case 6416: return f(X64{}, Y16{});
        case 12804: return f(X128{}, Y4{});
        case 12808: return f(X128{}, Y8{});
        case 25604: return f(X256{}, Y4{});
        default: return f(X64{}, Y8{});
        }
    }
}

// Passes of a step.  Forward: velocity, stress.  Adjoint step (reverse order of the
// forward step): stress-A (C gradients, X = C G_s A_s), velocity-A (A_v update, b
// gradient, Y = G_v A_v / rho_eff), stress-B (A_s update from Y); the tiled adjoint runs
// stress-B of step n+1 and stress-A of step n as one pass, stress-M, and a last stress-B
// after step 0.  The velocity pass also comes in a variant for the gradient's segment
// recompute: the tile kernels write v^{n+1/2} through the grid's save pointers instead of
// over v^{n-1/2}, the cell kernel writes it to both.
enum Pass { kPassVel = 0, kPassStress = 1, kPassStressA, kPassVelA, kPassStressB, kPassVelSave, kPassStressM };

// Tile and fused sweeps address a window of at most zchunk + 8 planes (and at most the
// grid's nz) through one buffer descriptor per field, of at most 1 GiB.
inline bool window_ok(const fd3d_ctx *c, int zc)
{
    const long rows = c->L.rows ? kRows : 1, planes = std::min(zc + 8, c->n[2]);
    return planes * rows * (long)c->n[0] * (long)c->n[1] * (long)c->tsize <= kMaxWindowBytes;
}

// Cache policy of a context's single-grid tile launches: the model arrays and the
// gradient's stored velocities and accumulators are streamed (non-temporal) when the
// grid's working set, nine fields and three model arrays, exceeds the 256 MB Infinity
// Cache.  Below that the whole working set can stay cached from step to step, and
// streaming would evict the model.
constexpr double kInfinityCacheBytes = 256.0 * 1024 * 1024;
inline bool stream_model(const fd3d_ctx *c)
{
    if (coarse_on(c->opts)) return false;  // the coarse medium is small and stays cached
    return 12.0 * (double)c->n[0] * (double)c->n[1] * (double)c->n[2] * (double)c->tsize > kInfinityCacheBytes;
}

// rec (stress passes of the forward only): the step's receiver sampling, carried by the
// tile launch or launched after the cell kernel.  Forward passes (velocity, stress and
// their storing variants); defined for float and double, with and without free surface.
template <typename T, bool FS>
void launch_pass(const fd3d_ctx *c, const Grid<T> &G, const Inject<T> &inj, int n, int pass, hipStream_t st,
                 const TileIO<T> &io = TileIO<T>{}, const RecJob<T> &rec = RecJob<T>{});

// The receiver sampling of a grid's velocity (none when nrec is 0).
template <typename T> RecJob<T> rec_job(const T *vx, const T *vy, const T *vz, const RecTap<T> *taps, int nrec,
                                        int nt, T *traces)
{
    RecJob<T> r{};
    if (nrec <= 0) return r;
    r.v[0] = vx;
    r.v[1] = vy;
    r.v[2] = vz;
    r.taps = taps;
    r.traces = traces;
    r.nq = 3 * nrec;
    r.nt = nt;
    return r;
}

// One forward step: velocity pass, then the stress pass, which samples the receivers.
template <typename T, bool FS>
void step(fd3d_ctx *c, const Grid<T> &G, const Inject<T> &inj, int n, int nrec, const RecTap<T> *taps, T *traces,
          hipStream_t st, Timer &tm);

// Fused tile shapes: FP32 64x4 and 64x8, FP64 64x4.
bool fused_supported(const fd3d_ctx *c, int tx, int ty);

// Gradient workspace (byte offsets): adjoint state, staggered-point gradient
// accumulators, the tiled adjoint's intermediate fields, checkpoints every k steps, the
// stored velocities of one k-step segment, a copy of the segment's checkpoint (the cell
// adjoint's v^{n-1/2} of the segment's first step), and the residual buffer of
// fd3d_gradient.
// Every group of fields has the layout of the context's state (one block of interleaved
// rows, or padded arrays): field q of a group at q * fstep.
struct GradLayout {
    size_t fstep;   // bytes from one field of a group to the next
    size_t group;   // bytes of a group of nine fields
    size_t chunk;   // bytes from one field-sized chunk of a group to the next (copies)
    size_t adj;     // 9 fields: A_v, A_s
    size_t acc;     // 8 fields: gl, gm, g_mu_xy, g_mu_xz, g_mu_yz, g_bx, g_by, g_bz
    size_t scr;     // 9 fields: X = C G_s A_s (6, stress layout), Y = G_v A_v / rho_eff (3)
    size_t ckpt;    // nseg groups: state at the start of steps 0, k, 2k, ...
    size_t seg;     // ceil(k/3) groups: v^{n+1/2} of three steps of a segment per group
    size_t prev;    // one group: a copy of the segment's checkpoint (cell adjoint)
    size_t res;     // residual [max_rec][3][nt]
    size_t misfit;  // one T
    size_t total;
    int nseg, k;
};

// Gradient workspace layout for checkpoints every k steps.
GradLayout make_grad_layout(const fd3d_ctx *c, int k);

// Stored v^{n+1/2} of step m of a segment (m < k): fields 3 (m mod 3) .. +2 of group m / 3.
inline char *seg_slot(char *gws, const GradLayout &GL, int m)
{
    return gws + GL.seg + (size_t)(m / 3) * GL.group + (size_t)(3 * (m % 3)) * GL.fstep;
}

// Bytes of a checkpoint group copied to the segment's prev group: the velocity fields (the
// first three separate arrays), or the whole block of interleaved rows.
inline size_t prev_copy_bytes(const fd3d_ctx *c, const GradLayout &GL)
{
    return c->L.rows ? GL.group : 3 * GL.fstep;
}

// v^{n-1/2} of segment step m: the previous step's stored v^{n+1/2}, or for m = 0 the
// velocity fields of the copy of the segment's checkpoint.
inline char *prev_velocity(char *gws, const GradLayout &GL, int m)
{
    return m > 0 ? seg_slot(gws, GL, m - 1) : gws + GL.prev;
}

// The q-th field-sized chunk of the current state (q < 9): field q of separate arrays, or
// the q-th ninth of the block of interleaved rows.  Checkpoints copy a state chunk by
// chunk into a group of the same layout.
template <typename T> char *state_chunk(const fd3d_ctx *c, const Grid<T> &G, int q)
{
    return c->L.rows ? (char *)G.f[0] + (size_t)q * c->L.chunk : (char *)G.f[q];
}

// The nt-step forward of a context (checkpoints into gws with GL); float and double.
template <typename T>
int forward_impl(fd3d_ctx *c, const fd3d_source *src, int nrec, const double *rec_pos, void *traces, int flags,
                 hipStream_t st, char *gws = nullptr, const GradLayout *GL = nullptr);

template <typename T> AdjGrid<T> make_adj(char *gws, const GradLayout &GL)
{
    AdjGrid<T> A;
    for (int f = 0; f < NFIELD; ++f) A.a[f] = (T *)(gws + GL.adj + f * GL.fstep);
    T *acc[8];
    for (int q = 0; q < 8; ++q) acc[q] = (T *)(gws + GL.acc + q * GL.fstep);
    A.gl = acc[0];
    A.gm = acc[1];
    for (int q = 0; q < 3; ++q) {
        A.gs[q] = acc[2 + q];
        A.gb[q] = acc[5 + q];
    }
    for (int q = 0; q < 3; ++q) A.vst[q] = A.vprev[q] = nullptr;
    return A;
}

// The stored velocities of segment step m for the one-thread-per-cell adjoint (the tiled
// adjoint reads v^{n+1/2} only).
template <typename T> void set_stored_velocity(AdjGrid<T> &A, char *gws, const GradLayout &GL, int m)
{
    const char *slot = seg_slot(gws, GL, m), *prev = prev_velocity(gws, GL, m);
    for (int q = 0; q < 3; ++q) {
        A.vst[q] = (const T *)(slot + q * GL.fstep);
        A.vprev[q] = (const T *)(prev + q * GL.fstep);
    }
}

// Fields of the three tiled adjoint passes of segment step m: grids (f[] re-pointed) and
// tile outputs.  The tiled adjoint holds Y = G_v A_v / rho_eff (intermediate fields 6-8)
// in place of A_v.
template <typename T> struct AdjTiles {
    Grid<T> g[3];     // stress-A (or stress-M), velocity-A, stress-B
    TileIO<T> io[3];
};

template <typename T> AdjTiles<T> adj_tiles(const Grid<T> &G, char *gws, const GradLayout &GL, int m)
{
    auto fld = [&](size_t base, int q) { return (T *)(gws + base + q * GL.fstep); };
    const char *slot = seg_slot(gws, GL, m);
    AdjTiles<T> P;
    for (int p = 0; p < 3; ++p) {
        P.g[p] = G;
        for (int f = 0; f < NFIELD; ++f) P.g[p].save[f] = nullptr;
        std::memset(&P.io[p], 0, sizeof P.io[p]);
    }
    for (int q = 0; q < 3; ++q) {
        P.g[0].f[VX + q] = (T *)(slot + q * GL.fstep);  // stored v^{n+1/2}
        P.g[1].f[VX + q] = fld(GL.scr, 6 + q);            // Y
        P.g[2].f[VX + q] = fld(GL.scr, 6 + q);
        P.io[1].acc[q] = fld(GL.acc, 5 + q);              // g_b
        P.io[1].vst[q] = (const T *)(slot + q * GL.fstep);
        P.io[0].y[q] = fld(GL.scr, 6 + q);                // Y of the step after (stress-M)
    }
    for (int q = 0; q < 6; ++q) {
        P.g[0].f[SXX + q] = fld(GL.adj, SXX + q);  // A_s
        P.g[1].f[SXX + q] = fld(GL.scr, q);        // X
        P.g[2].f[SXX + q] = fld(GL.adj, SXX + q);
        P.io[0].out[q] = fld(GL.scr, q);
    }
    for (int q = 0; q < 5; ++q) P.io[0].acc[q] = fld(GL.acc, q);  // gl, gm, g_mu_xy, g_mu_xz, g_mu_yz
    return P;
}

// What the tiled adjoint's residual injection of segment step m updates.
template <typename T> TapAdjoint<T> tap_adjoint(const Grid<T> &G, char *gws, const GradLayout &GL, int m)
{
    const AdjTiles<T> P = adj_tiles<T>(G, gws, GL, m);
    TapAdjoint<T> A;
    for (int q = 0; q < 3; ++q) {
        A.y[q] = P.g[1].f[VX + q];
        A.gb[q] = P.io[1].acc[q];
        A.vst[q] = P.io[1].vst[q];
    }
    A.rho = G.rho;
    for (int a = 0; a < 3; ++a)
        for (int h = 0; h < 2; ++h) A.g[a][h] = G.g[a][h];
    A.sy = G.sy;
    A.sz = G.sz;
    return A;
}

// The tiled adjoint's last term of the gradient of b, from the initial velocity (the
// velocity fields of checkpoint 0) and the first step's Y.
template <typename T> void launch_gb_initial(const Grid<T> &G, const AdjGrid<T> &A, char *gws, const GradLayout &GL,
                                             hipStream_t st)
{
    auto v0 = [&](int q) { return (const T *)(gws + GL.ckpt + q * GL.fstep); };
    auto y = [&](int q) { return (const T *)(gws + GL.scr + (6 + q) * GL.fstep); };
    const dim3 blk(64, 4, 1), grd((G.nx + 63) / 64, (G.ny + 3) / 4, G.nz);
    gb_initial_velocity<T><<<grd, blk, 0, st>>>(G, v0(0), v0(1), v0(2), y(0), y(1), y(2), A.gb[0], A.gb[1], A.gb[2]);
}

// Zero the adjoint state, accumulators and intermediate fields, and the segment slots
// (whose samples at the pinned staggered positions are never stored and must read 0).
template <typename T> void zero_grad_fields(char *gws, const GradLayout &GL, hipStream_t st)
{
    fill_zero<T><<<2048, 256, 0, st>>>((T *)(gws + GL.adj), (long)((GL.ckpt - GL.adj) / sizeof(T)));
    fill_zero<T><<<2048, 256, 0, st>>>((T *)(gws + GL.seg), (long)((GL.res - GL.seg) / sizeof(T)));
}

// Validates a caller's gradient workspace for checkpoints every k steps.
int check_gws(const fd3d_ctx *ctx, void *gws, size_t gws_bytes, int k);

} // namespace fd3d
