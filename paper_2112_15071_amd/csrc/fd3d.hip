// fd3d.hip -- host side of the C ABI declared in include/fd3d.h.
//
// Validation, workspace layout, damping profiles, point-operator weights and the
// step loop that enqueues the velocity pass, the receiver sampling and the
// stress pass of every step on the caller's stream (Sec. 2.2 update order).
#include "fd3d.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <string>
#include <vector>

#include "common.h"
#include "fwd_cell.h"
#include "fwd_tile.h"
#include "fwd_fused.h"
#include "adj_cell.h"
#include "born_cell.h"
#include "util_kernels.h"

#include <unordered_set>

using namespace fd3d;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(FD3D_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
constexpr int kDefaultMaxRec = 4096;

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

size_t rectap_bytes(int tsize) { return 8 * sizeof(int) + 8 * (size_t)tsize; }

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

Layout make_layout(int nx, int ny, int nz, int tsize, int max_rec, bool rows, bool model_block)
{
    Layout L{};
    size_t off = 0;
    L.rows = rows;
    L.field_bytes = (size_t)nx * ny * nz * tsize;
    const size_t stride = round_up(L.field_bytes, 4096) + 1024;
    L.fstep = rows ? (size_t)nx * tsize : stride;
    L.group = rows ? round_up(kRows * L.field_bytes, 4096) + 1024 : NFIELD * stride;
    L.chunk = rows ? L.field_bytes : stride;
    for (int b = 0; b < 2; ++b) {
        for (int f = 0; f < NFIELD; ++f) L.field[b][f] = off + f * L.fstep;
        off += L.group;
    }
    L.model = 0;
    if (rows && model_block) {
        L.model = off;
        off += L.group;
    }
    const int n[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a)
        for (int h = 0; h < 2; ++h) {
            L.prof[a][h] = off;
            off += round_up((size_t)n[a] * tsize, kAlign);
        }
    L.src = off;
    off += round_up((size_t)NFIELD * 8 * tsize, kAlign);
    L.rec = off;
    off += round_up((size_t)max_rec * 3 * rectap_bytes(tsize), kAlign);
    L.colors = off;
    off += round_up((size_t)max_rec * sizeof(int), kAlign);
    L.part = off;
    off += round_up((size_t)kReduceBlocks * kStats * sizeof(double), kAlign);
    L.stats = off;
    off += round_up(kStats * sizeof(double), kAlign);
    L.flag = off;
    off += kAlign;
    L.total = off;
    return L;
}

int check_opts(const fd3d_opts *o)
{
    if (o->dtype != FD3D_F32 && o->dtype != FD3D_F64) return fail(FD3D_EINVAL, "opts.dtype must be FD3D_F32 or FD3D_F64");
    for (int f = 0; f < 6; ++f)
        if (o->sponge[f] < 0) return fail(FD3D_EINVAL, "opts.sponge widths must be >= 0");
    if (!std::isfinite(o->sponge_alpha)) return fail(FD3D_EINVAL, "opts.sponge_alpha must be finite");
    if (!(o->dy >= 0.0) || !(o->dz >= 0.0) || !std::isfinite(o->dy) || !std::isfinite(o->dz))
        return fail(FD3D_EINVAL, "opts.dy and opts.dz must be finite and >= 0 (0: dx)");
    if (o->vacuum_top < 0) return fail(FD3D_EINVAL, "opts.vacuum_top must be >= 0");
    if (o->vacuum_top > 0 && o->free_surface)
        return fail(FD3D_EINVAL, "opts.vacuum_top and opts.free_surface exclude each other");
    if (o->vacuum_map && o->vacuum_top <= 0) return fail(FD3D_EINVAL, "opts.vacuum_map needs opts.vacuum_top > 0");
    if (o->layout < FD3D_LAYOUT_AUTO || o->layout > FD3D_LAYOUT_ROWS)
        return fail(FD3D_EINVAL, "opts.layout must be FD3D_LAYOUT_AUTO, _SEPARATE or _ROWS");
    if (o->coarse[0] || o->coarse[1] || o->coarse[2]) {
        for (int a = 0; a < 3; ++a)
            if (o->coarse[a] < 2) return fail(FD3D_EINVAL, "opts.coarse needs >= 2 nodes per axis (or all 0)");
        if (o->vacuum_top > 0) return fail(FD3D_EINVAL, "opts.coarse with opts.vacuum_top is not supported");
    }
    return FD3D_OK;
}

fd3d_opts default_opts()
{
    fd3d_opts o;
    std::memset(&o, 0, sizeof o);
    o.dtype = FD3D_F32;
    o.max_receivers = kDefaultMaxRec;
    return o;
}

int max_rec_of(const fd3d_opts &o) { return o.max_receivers > 0 ? o.max_receivers : kDefaultMaxRec; }

// The medium arrays are a coarse grid read by trilinear samples (opts.coarse).
bool coarse_on(const fd3d_opts &o) { return o.coarse[0] > 0; }

// Field storage of a grid (opts.layout).  Automatic: interleaved rows when a tile sweep
// over the whole depth fits one buffer window, separate arrays otherwise.  Measured on
// MI355X with the same tile sweeps, interleaved rows run the step 4-5 % faster (256^3,
// 256^2 x 128; 2-3 % at 128^3); on larger planes the window caps rows at shorter sweeps
// (64 planes at 512^2), and separate arrays with whole-depth sweeps run faster there.
bool rows_fit(int nx, int ny, int nz, int tsize, int planes)
{
    const double row_samples = (double)kRows * nx * ny;
    return row_samples * nz < 2147483647.0 &&  // receiver tap indices are int
           (double)planes * row_samples * tsize <= (double)kMaxWindowBytes;
}

bool rows_layout(int nx, int ny, int nz, int tsize, const fd3d_opts &o)
{
    if (o.layout == FD3D_LAYOUT_SEPARATE) return false;
    if (o.layout == FD3D_LAYOUT_ROWS) return true;
    return rows_fit(nx, ny, nz, tsize, nz);
}

Layout layout_of(int nx, int ny, int nz, const fd3d_opts &o)
{
    const int tsize = o.dtype == FD3D_F64 ? 8 : 4;
    const bool rows = rows_layout(nx, ny, nz, tsize, o);
    return make_layout(nx, ny, nz, tsize, max_rec_of(o), rows, rows && !coarse_on(o));
}

// Cerjan factor of one face at distance d (cells) from it.
double face_factor(double d, int width, double alpha)
{
    if (width <= 0 || d >= width) return 1.0;
    const double a = alpha > 0.0 ? alpha : 0.3 / width;
    const double t = a * (width - d);
    return std::exp(-t * t);
}

// Eight trilinear taps of point p on component c's subgrid; false when a tap is not
// an active sample.
bool point_taps(int c, const double p[3], const int n[3], int base[3], double w[8])
{
    double fr[3];
    for (int a = 0; a < 3; ++a) {
        if (!std::isfinite(p[a])) return false;
        const double q = p[a] - 0.5 * stag(c, a);
        const double b = std::floor(q);
        const int last = n[a] - 1 - stag(c, a);
        if (b < 0.0 || b + 1.0 > (double)last) return false;
        base[a] = (int)b;
        fr[a] = q - b;
    }
    int m = 0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx)
                w[m++] = (dx ? fr[0] : 1.0 - fr[0]) * (dy ? fr[1] : 1.0 - fr[1]) * (dz ? fr[2] : 1.0 - fr[2]);
    return true;
}

} // namespace

struct fd3d_ctx {
    int n[3];
    int nt;
    int tsize;
    double dx, dy, dz, dt;  // spacing per axis (m), time step (s)
    fd3d_opts opts;
    const void *lam, *mu, *rho;
    char *ws;
    size_t ws_bytes;
    Layout L;
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
};

namespace {

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

template <typename T> int upload_profiles(fd3d_ctx *c, hipStream_t st)
{
    const int top = c->opts.free_surface ? 0 : c->opts.sponge[4];
    const int width[3][2] = {{c->opts.sponge[0], c->opts.sponge[1]},
                             {c->opts.sponge[2], c->opts.sponge[3]},
                             {top, c->opts.sponge[5]}};
    size_t total = 0;
    for (int a = 0; a < 3; ++a) total += 2 * (size_t)c->n[a];
    c->prof_host.assign(total * sizeof(T), 0);
    T *h = (T *)c->prof_host.data();
    size_t off = 0;
    for (int a = 0; a < 3; ++a)
        for (int half = 0; half < 2; ++half) {
            const int n = c->n[a];
            for (int i = 0; i < n; ++i) {
                const double pos = i + 0.5 * half;
                h[off + i] = (T)(face_factor(pos, width[a][0], c->opts.sponge_alpha) *
                                 face_factor((n - 1) - pos, width[a][1], c->opts.sponge_alpha));
            }
            HIP_TRY(hipMemcpyAsync(c->ws + c->L.prof[a][half], h + off, n * sizeof(T), hipMemcpyHostToDevice, st));
            off += n;
        }
    return FD3D_OK;
}

template <typename T> int model_check(fd3d_ctx *c, hipStream_t st)
{
    // statistics over the medium's own nodes; with a coarse medium every sample is a convex
    // combination of coarse nodes, so their extremes bound the sampled ones (vp, vs by the
    // mediant inequality)
    const fd3d_opts &o = c->opts;
    const long N = coarse_on(o) ? (long)o.coarse[0] * o.coarse[1] * o.coarse[2] : (long)c->n[0] * c->n[1] * c->n[2];
    double *part = (double *)(c->ws + c->L.part);
    double *out = (double *)(c->ws + c->L.stats);
    model_stats<T><<<kReduceBlocks, kReduceThreads, 0, st>>>((const T *)c->lam, (const T *)c->mu,
                                                            (const T *)c->rho, N, part);
    stats_final<<<1, kReduceThreads, 0, st>>>(part, kReduceBlocks, out);
    HIP_TRY(hipGetLastError());
    double s[kStats];
    HIP_TRY(hipMemcpyAsync(s, out, sizeof s, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (s[5] != 0.0) return fail(FD3D_EMODEL, "model holds a non-finite value");
    if (!(s[2] > 0.0)) return fail(FD3D_EMODEL, "rho must be > 0 everywhere");
    if (s[3] < 0.0) return fail(FD3D_EMODEL, "mu must be >= 0 everywhere");
    if (c->opts.vacuum_top > 0) {
        if (!(s[4] >= 0.0)) return fail(FD3D_EMODEL, "lambda + 2 mu must be >= 0 everywhere");
    } else if (!(s[4] > 0.0)) {
        return fail(FD3D_EMODEL, "lambda + 2 mu must be > 0 everywhere");
    }
    // von Neumann bound of the O(2,4) scheme: dt vp sqrt(sum 1/h_a^2) <= 1 / (9/8 + 1/24)
    const double inv = std::sqrt(1.0 / (c->dx * c->dx) + 1.0 / (c->dy * c->dy) + 1.0 / (c->dz * c->dz));
    c->info[0] = s[0];
    c->info[1] = s[1] < 1e299 ? s[1] : 0.0;
    c->info[2] = s[2];
    c->info[3] = (6.0 / 7.0) / (s[0] * inv);
    if (c->dt > c->info[3] * (1.0 + 1e-12))
        return fail(FD3D_ECFL, "dt = " + std::to_string(c->dt) + " exceeds the stability bound " +
                                   std::to_string(c->info[3]) + " ((6/7) / (vp_max sqrt(sum 1/h^2)))");
    return FD3D_OK;
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

// The model's copy into interleaved rows (rows 0-2 of the model block; the rest zeroed).
template <typename T> void copy_model(fd3d_ctx *c, hipStream_t st)
{
    if (!c->L.model) return;
    T *m = (T *)(c->ws + c->L.model);
    fill_zero<T><<<2048, 256, 0, st>>>(m, (long)(c->L.group / sizeof(T)));
    const void *src[3] = {c->lam, c->mu, c->rho};
    for (int q = 0; q < 3; ++q)
        copy_field<T>(c, (T *)((char *)m + q * c->L.fstep), true, (const T *)src[q], false, -1, st);
}

void zero_fields_any(fd3d_ctx *c, hipStream_t st);

// The source's tap boxes into inj and its coefficients into the host staging buffer
// (uploaded by stage_inputs).
template <typename T> int build_source(fd3d_ctx *c, const fd3d_source *src, Inject<T> &inj)
{
    std::memset(&inj, 0, sizeof inj);
    c->src_host.assign((size_t)NFIELD * 8 * sizeof(T), 0);
    T *coef = (T *)c->src_host.data();
    inj.coef = (const T *)(c->ws + c->L.src);
    for (int f = 0; f < NFIELD; ++f) inj.i0[f] = inj.j0[f] = inj.k0[f] = -(1 << 28);
    if (!src) return FD3D_OK;
    const double h3 = c->dx * c->dy * c->dz;  // cell volume
    int base[3];
    double w[8];
    bool any = false;
    for (int q = 0; q < 3; ++q) {
        if (src->force[q] == 0.0) continue;
        if (!std::isfinite(src->force[q])) return fail(FD3D_EINVAL, "source force must be finite");
        if (!point_taps(VX + q, src->pos, c->n, base, w))
            return fail(FD3D_ERANGE, "force source taps leave the active samples of v" + std::string(1, "xyz"[q]));
        inj.i0[VX + q] = base[0]; inj.j0[VX + q] = base[1]; inj.k0[VX + q] = base[2];
        for (int m = 0; m < 8; ++m) coef[(VX + q) * 8 + m] = (T)(c->dt * w[m] * src->force[q] / h3);
        any = true;
    }
    for (int q = 0; q < 6; ++q)
        if (!std::isfinite(src->moment[q])) return fail(FD3D_EINVAL, "source moment must be finite");
    if (src->moment[0] != 0.0 || src->moment[1] != 0.0 || src->moment[2] != 0.0) {
        if (!point_taps(SXX, src->pos, c->n, base, w))
            return fail(FD3D_ERANGE, "moment source taps leave the normal-stress grid");
        for (int q = 0; q < 3; ++q) {
            inj.i0[SXX + q] = base[0]; inj.j0[SXX + q] = base[1]; inj.k0[SXX + q] = base[2];
            for (int m = 0; m < 8; ++m) coef[(SXX + q) * 8 + m] = (T)(-c->dt * w[m] * src->moment[q] / h3);
        }
        any = true;
    }
    for (int q = 3; q < 6; ++q) {
        if (src->moment[q] == 0.0) continue;
        const int comp = SXY + (q - 3);
        if (!point_taps(comp, src->pos, c->n, base, w))
            return fail(FD3D_ERANGE, "moment source taps leave the shear-stress grid");
        inj.i0[comp] = base[0]; inj.j0[comp] = base[1]; inj.k0[comp] = base[2];
        for (int m = 0; m < 8; ++m) coef[(comp) * 8 + m] = (T)(-c->dt * w[m] * src->moment[q] / h3);
        any = true;
    }
    if (any && !src->wavelet && c->nt > 0) return fail(FD3D_EINVAL, "source wavelet pointer is NULL");
    inj.on = any ? 1 : 0;
    inj.wavelet = (const T *)src->wavelet;
    return FD3D_OK;
}

// Builds the source (tap boxes into inj) and the receiver descriptors and colours, and
// uploads them from the context's host staging buffers (after the previous call's
// uploads from those buffers are done).
template <typename T>
int stage_inputs(fd3d_ctx *c, const fd3d_source *src, Inject<T> &inj, int nrec, const double *rec_pos,
                 hipStream_t st)
{
    if (c->staged_pending) {
        HIP_TRY(hipEventSynchronize(c->staged));
        c->staged_pending = false;
    }
    int rc = build_source<T>(c, src, inj);
    if (rc) return rc;
    // inputs equal to the ones already in the workspace (a repeated shot) are not staged again
    if (c->src_host != c->src_dev) {
        HIP_TRY(hipMemcpyAsync(c->ws + c->L.src, c->src_host.data(), c->src_host.size(), hipMemcpyHostToDevice, st));
        c->src_dev = c->src_host;
        if (c->staged) {
            HIP_TRY(hipEventRecord(c->staged, st));
            c->staged_pending = true;
        }
    }
    if (nrec == 0) return FD3D_OK;
    if (c->rec_dev_valid && c->rec_dev.size() == (size_t)nrec * 3 &&
        std::memcmp(c->rec_dev.data(), rec_pos, (size_t)nrec * 3 * sizeof(double)) == 0)
        return FD3D_OK;
    c->rec_dev_valid = false;
    c->rec_host.assign((size_t)nrec * 3 * sizeof(RecTap<T>), 0);
    RecTap<T> *t = (RecTap<T> *)c->rec_host.data();
    const long sy = c->L.rows ? (long)kRows * c->n[0] : c->n[0], sz = sy * c->n[1];  // field strides
    int base[3];
    double w[8];
    for (int r = 0; r < nrec; ++r)
        for (int q = 0; q < 3; ++q) {
            if (!point_taps(VX + q, rec_pos + 3 * r, c->n, base, w))
                return fail(FD3D_ERANGE, "receiver " + std::to_string(r) + " taps leave the active samples of v" +
                                             std::string(1, "xyz"[q]));
            RecTap<T> &d = t[r * 3 + q];
            int m = 0;
            for (int dz = 0; dz < 2; ++dz)
                for (int dy = 0; dy < 2; ++dy)
                    for (int dx = 0; dx < 2; ++dx) {
                        d.idx[m] = (int)((base[0] + dx) + sy * (base[1] + dy) + sz * (base[2] + dz));
                        d.w[m] = (T)w[m];
                        ++m;
                    }
        }
    // colours: receivers in one colour share no tap, so their adjoint injections can run
    // as one launch without write conflicts (greedy, in receiver order)
    std::vector<std::unordered_set<long>> used;  // keys 3 * index + component
    std::vector<std::vector<int>> members;
    for (int r = 0; r < nrec; ++r) {
        size_t col = 0;
        for (;; ++col) {
            if (col == used.size()) {
                used.emplace_back();
                members.emplace_back();
            }
            bool clash = false;
            for (int q = 0; q < 3 && !clash; ++q)
                for (int m = 0; m < 8 && !clash; ++m) clash = used[col].count(3L * t[r * 3 + q].idx[m] + q) > 0;
            if (!clash) break;
        }
        for (int q = 0; q < 3; ++q)
            for (int m = 0; m < 8; ++m) used[col].insert(3L * t[r * 3 + q].idx[m] + q);
        members[col].push_back(r);
    }
    c->color_host.clear();
    c->color_off.assign(1, 0);
    for (auto &mm : members) {
        c->color_host.insert(c->color_host.end(), mm.begin(), mm.end());
        c->color_off.push_back((int)c->color_host.size());
    }
    HIP_TRY(hipMemcpyAsync(c->ws + c->L.rec, c->rec_host.data(), c->rec_host.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(c->ws + c->L.colors, c->color_host.data(), c->color_host.size() * sizeof(int),
                           hipMemcpyHostToDevice, st));
    c->rec_dev.assign(rec_pos, rec_pos + (size_t)nrec * 3);
    c->rec_dev_valid = true;
    if (c->staged) {
        HIP_TRY(hipEventRecord(c->staged, st));
        c->staged_pending = true;
    }
    return FD3D_OK;
}

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

void zero_fields_any(fd3d_ctx *c, hipStream_t st)
{
    if (c->tsize == 8) zero_fields<double>(c, st);
    else zero_fields<float>(c, st);
}

TileMap tile_map(const fd3d_ctx *c)
{
    TileMap tm;
    tm.ntx = (c->n[0] + c->tile_x - 1) / c->tile_x;
    tm.nty = (c->n[1] + c->tile_y - 1) / c->tile_y;
    tm.zc = c->zchunk;
    tm.nzc = (c->n[2] + c->zchunk - 1) / c->zchunk;
    return tm;
}

// Supported tile shapes: 64x{4,8,16}, 128x{4,8}, 256x4 (FP64: 64x{4,8}, 128x4).
bool tile_supported(int tsize, int tx, int ty)
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
// forward step): stress-A (C gradients, X = C G_s A_s), velocity-A (A_v update),
// velocity-B (b gradient, Y = G_v A_v / rho_eff), stress-B (A_s update).
// The forward passes also come in a variant that stores v^{n+1/2} and sigma^n through the
// grid's save pointers (the gradient's segment recompute).
enum Pass { kPassVel = 0, kPassStress = 1, kPassStressA, kPassVelA, kPassVelB, kPassStressB, kPassVelSave,
            kPassStressSave };

// Tile and fused sweeps address a window of at most zchunk + 8 planes (and at most the
// grid's nz) through one buffer descriptor per field, of at most 1 GiB.
bool window_ok(const fd3d_ctx *c, int zc)
{
    const long rows = c->L.rows ? kRows : 1, planes = std::min(zc + 8, c->n[2]);
    return planes * rows * (long)c->n[0] * (long)c->n[1] * (long)c->tsize <= kMaxWindowBytes;
}

// Cache policy of a context's single-grid tile launches: the model arrays and the
// gradient's stored states are streamed (non-temporal) when the grid's working set, nine
// fields and three model arrays, exceeds the 256 MB Infinity Cache.  Below that the whole
// working set can stay cached from step to step, and streaming would evict the model.
constexpr double kInfinityCacheBytes = 256.0 * 1024 * 1024;
inline bool stream_model(const fd3d_ctx *c)
{
    if (coarse_on(c->opts)) return false;  // the coarse medium is small and stays cached
    return 12.0 * (double)c->n[0] * (double)c->n[1] * (double)c->n[2] * (double)c->tsize > kInfinityCacheBytes;
}

// rec: receiver sampling carried by a forward stress launch (extra workgroups).
// NTP: cache policy of the model loads and stored states (see stream_model).
template <typename T, int TX, int TY, bool FS, bool NTP>
void launch_tiles(const Grid<T> &G, const Inject<T> &inj, int n, const TileMap &tm, int pass, hipStream_t st,
                  const TileIO<T> &io = TileIO<T>{}, const RecJob<T> &rec = RecJob<T>{})
{
    const int nwg = tm.ntx * tm.nty * tm.nzc;
    constexpr int NT = TX * TY;
    const int nws = nwg + rec_blocks(rec, NT);
    if (G.save[VX] != nullptr && pass == kPassVel) pass = kPassVelSave;
    if (G.save[VX] != nullptr && pass == kPassStress) pass = kPassStressSave;
    if (G.cm[0] > 0) {  // coarse medium: instantiations of their own (forward passes only)
        if (pass == kPassVel) vel_tile<T, TX, TY, FS, kFwd, false, false, true><<<nwg, NT, 0, st>>>(G, inj, n, tm);
        else stress_tile<T, TX, TY, FS, kFwd, false, false, true><<<nws, NT, 0, st>>>(G, inj, n, tm, rec);
        return;
    }
    if constexpr (!FS) {  // the vacuum surface has instantiations of its own (forward only)
        if (G.ks > 0 && pass == kPassVel) {
            vel_tile<T, TX, TY, false, kFwd, true, NTP><<<nwg, NT, 0, st>>>(G, inj, n, tm);
            return;
        }
        if (G.ks > 0 && pass == kPassStress) {
            stress_tile<T, TX, TY, false, kFwd, true, NTP><<<nws, NT, 0, st>>>(G, inj, n, tm, rec);
            return;
        }
    }
    switch (pass) {
    case kPassVel: vel_tile<T, TX, TY, FS, kFwd, false, NTP><<<nwg, NT, 0, st>>>(G, inj, n, tm); break;
    case kPassStress: stress_tile<T, TX, TY, FS, kFwd, false, NTP><<<nws, NT, 0, st>>>(G, inj, n, tm, rec); break;
    case kPassVelSave: vel_tile<T, TX, TY, FS, kFwdSave, false, NTP><<<nwg, NT, 0, st>>>(G, inj, n, tm); break;
    case kPassStressSave:
        stress_tile<T, TX, TY, FS, kFwdSave, false, NTP><<<nws, NT, 0, st>>>(G, inj, n, tm, rec);
        break;
    case kPassStressA: stress_tile_adj<T, TX, TY, kAdjA, NTP><<<nwg, NT, 0, st>>>(G, inj, tm, io); break;
    case kPassVelA: vel_tile_adj<T, TX, TY, kAdjA, NTP><<<nwg, NT, 0, st>>>(G, inj, n, tm, io); break;
    case kPassVelB: vel_tile_adj<T, TX, TY, kAdjB, NTP><<<nwg, NT, 0, st>>>(G, inj, n, tm, io); break;
    default: stress_tile_adj<T, TX, TY, kAdjB, NTP><<<nwg, NT, 0, st>>>(G, inj, tm, io); break;
    }
}

// rec (stress passes of the forward only): the step's receiver sampling, carried by the
// tile launch or launched after the cell kernel.
template <typename T, bool FS>
void launch_pass(const fd3d_ctx *c, const Grid<T> &G, const Inject<T> &inj, int n, int pass, hipStream_t st,
                 const TileIO<T> &io = TileIO<T>{}, const RecJob<T> &rec = RecJob<T>{})
{
    if (c->variant == FD3D_KERNEL_CELL) {
        const dim3 blk(64, 4, 1);
        const dim3 grd((G.nx + 63) / 64, (G.ny + 3) / 4, G.nz);
        if (pass == kPassVel) vel_cell<T, FS><<<grd, blk, 0, st>>>(G, inj, n);
        else stress_cell<T, FS><<<grd, blk, 0, st>>>(G, inj, n);
        if (rec.nq > 0) record<T><<<rec_blocks(rec, 256), 256, 0, st>>>(rec, n);
        return;
    }
    const TileMap tm = tile_map(c);
    with_tile<T>(c->tile_x, c->tile_y, [&](auto tx, auto ty) {
        constexpr int TX = decltype(tx)::value, TY = decltype(ty)::value;
        // FP64 (the debug mode) keeps the plain policy and needs no second instantiation
        if (sizeof(T) == 4 && stream_model(c))
            launch_tiles<T, TX, TY, FS, sizeof(T) == 4>(G, inj, n, tm, pass, st, io, rec);
        else
            launch_tiles<T, TX, TY, FS, false>(G, inj, n, tm, pass, st, io, rec);
    });
}

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

template <typename T, bool FS>
void step(fd3d_ctx *c, const Grid<T> &G, const Inject<T> &inj, int n, int nrec, const RecTap<T> *taps, T *traces,
          hipStream_t st, Timer &tm)
{
    tm.begin(0);
    launch_pass<T, FS>(c, G, inj, n, kPassVel, st);
    tm.end();
    tm.begin(2);  // the stress launch also samples the receivers
    launch_pass<T, FS>(c, G, inj, n, kPassStress, st, TileIO<T>{},
                       rec_job<T>(G.f[VX], G.f[VY], G.f[VZ], taps, nrec, c->nt, traces));
    tm.end();
}

// Fused tile shapes: FP32 64x4 and 64x8, FP64 64x4.
bool fused_supported(const fd3d_ctx *c, int tx, int ty)
{
    return c->opts.vacuum_top == 0 && !coarse_on(c->opts) && tx == 64 && (ty == 4 || (ty == 8 && c->tsize == 4));
}

// Arguments of one fused step from the current state copy into the other one.
template <typename T> FusedArgs<T> fused_args(const fd3d_ctx *c, const Inject<T> &inj, int n)
{
    FusedArgs<T> A;
    std::memset(&A, 0, sizeof A);
    const Grid<T> G = make_grid<T>(c);
    A.in = G.f[0];
    A.out = (T *)(c->ws + c->L.field[1 - c->cur][0]);
    A.fs = (long)((c->L.field[0][1] - c->L.field[0][0]) / sizeof(T));
    A.nx = G.nx;
    A.ny = G.ny;
    A.nz = G.nz;
    A.sy = (int)G.sy;
    A.sz = G.sz;
    A.dt = G.dt;
    A.rdx = G.rdx;
    A.rdy = G.rdy;
    A.rdz = G.rdz;
    A.lam = G.lam;
    A.mu = G.mu;
    A.rho = G.rho;
    for (int h = 0; h < 2; ++h) {
        A.gx[h] = G.g[0][h];
        A.gy[h] = G.g[1][h];
        A.gz[h] = G.g[2][h];
    }
    A.wavelet = inj.on ? inj.wavelet : nullptr;
    A.n = n;
    for (int a = 0; a < 3; ++a) A.origin[a][0] = A.origin[a][1] = -(1 << 28);
    for (int q = 0; q < NFIELD; ++q) {
        if (inj.i0[q] == -(1 << 28)) continue;  // component without source taps
        A.mask |= 1 << q;
        A.origin[0][stag(q, 0)] = inj.i0[q];
        A.origin[1][stag(q, 1)] = inj.j0[q];
        A.origin[2][stag(q, 2)] = inj.k0[q];
        for (int m = 0; m < 8; ++m) A.coef[q][m] = ((const T *)c->src_host.data())[q * 8 + m];
    }
    return A;
}

template <typename T, bool FS>
void launch_fused(const fd3d_ctx *c, const FusedArgs<T> &A, hipStream_t st)
{
    const TileMap tm = tile_map(c);
    const int nwg = tm.ntx * tm.nty * tm.nzc;
    if constexpr (sizeof(T) == 4) {
        if (c->tile_y == 8) {
            step_fused<T, 64, 8, FS><<<nwg, Fused<64, 8>::NT, 0, st>>>(A, tm);
            return;
        }
    }
    step_fused<T, 64, 4, FS><<<nwg, Fused<64, 4>::NT, 0, st>>>(A, tm);
}

// One fused step from the current state copy into the other one (which becomes current);
// the receivers sample the new velocity.
template <typename T, bool FS>
void fused_step(fd3d_ctx *c, const Inject<T> &inj, int n, int nrec, const RecTap<T> *taps, T *traces,
                hipStream_t st, Timer &tm)
{
    const FusedArgs<T> A = fused_args<T>(c, inj, n);
    tm.begin(3);
    launch_fused<T, FS>(c, A, st);
    tm.end();
    if (nrec > 0) {
        tm.begin(1);
        const RecJob<T> r = rec_job<T>(A.out + VX * A.fs, A.out + VY * A.fs, A.out + VZ * A.fs, taps, nrec, c->nt,
                                       traces);
        record<T><<<rec_blocks(r, 256), 256, 0, st>>>(r, n);
        tm.end();
    }
    c->cur ^= 1;
}

// Gradient workspace (byte offsets): adjoint state, staggered-point gradient
// accumulators, the tiled adjoint's intermediate fields, checkpoints every k steps, one
// k-step segment of stored fields, and the residual buffer of fd3d_gradient.  Every group
// of fields has the layout of the context's state (one block of interleaved rows, or
// padded arrays): field q of a group at q * fstep.
struct GradLayout {
    size_t fstep;   // bytes from one field of a group to the next
    size_t group;   // bytes of a group of nine fields
    size_t chunk;   // bytes from one field-sized chunk of a group to the next (copies)
    size_t adj;     // 9 fields: A_v, A_s
    size_t acc;     // 8 fields: gl, gm, g_mu_xy, g_mu_xz, g_mu_yz, g_bx, g_by, g_bz
    size_t scr;     // 9 fields: X = C G_s A_s (6, stress layout), Y = G_v A_v / rho_eff (3)
    size_t ckpt;    // nseg groups: state at the start of steps 0, k, 2k, ...
    size_t seg;     // k groups: v^{n+1/2} (3) then sigma^n (6) per step of a segment
    size_t res;     // residual [max_rec][3][nt]
    size_t misfit;  // one T
    size_t total;
    int nseg, k;
};

GradLayout make_grad_layout(const fd3d_ctx *c, int k)
{
    GradLayout g{};
    g.k = k;
    g.nseg = (c->nt + k - 1) / k;
    g.fstep = c->L.fstep;
    g.group = c->L.group;
    g.chunk = c->L.chunk;
    size_t off = 0;
    g.adj = off;
    off += g.group;
    g.acc = off;
    off += c->L.rows ? g.group : 8 * g.fstep;
    g.scr = off;
    off += g.group;
    g.ckpt = off;
    off += (size_t)g.nseg * g.group;
    g.seg = off;
    off += (size_t)k * g.group;
    g.res = off;
    off += round_up((size_t)c->opts.max_receivers * 3 * (size_t)(c->nt > 0 ? c->nt : 1) * c->tsize, kAlign);
    g.misfit = off;
    off += kAlign;
    g.total = off;
    return g;
}

// The q-th field-sized chunk of the current state (q < 9): field q of separate arrays, or
// the q-th ninth of the block of interleaved rows.  Checkpoints copy a state chunk by
// chunk into a group of the same layout.
template <typename T> char *state_chunk(const fd3d_ctx *c, const Grid<T> &G, int q)
{
    return c->L.rows ? (char *)G.f[0] + (size_t)q * c->L.chunk : (char *)G.f[q];
}

template <typename T>
int forward_impl(fd3d_ctx *c, const fd3d_source *src, int nrec, const double *rec_pos, void *traces, int flags,
                 hipStream_t st, char *gws = nullptr, const GradLayout *GL = nullptr)
{
    Inject<T> inj;
    int rc = stage_inputs<T>(c, src, inj, nrec, rec_pos, st);
    if (rc) return rc;
    if (!(flags & FD3D_KEEP_STATE)) zero_fields<T>(c, st);
    const RecTap<T> *taps = (const RecTap<T> *)(c->ws + c->L.rec);
    const bool fused = c->variant == FD3D_KERNEL_FUSED;
    Timer tm{c, st};
    c->prof_used = 0;
    for (int n = 0; n < c->nt; ++n) {
        const Grid<T> G = make_grid<T>(c);
        if (GL && n % GL->k == 0) {
            char *dst = gws + GL->ckpt + (size_t)(n / GL->k) * GL->group;
            for (int q = 0; q < NFIELD; ++q)
                HIP_TRY(hipMemcpyAsync(dst + q * GL->chunk, state_chunk<T>(c, G, q), c->L.field_bytes,
                                       hipMemcpyDeviceToDevice, st));
        }
        if (fused && c->opts.free_surface) fused_step<T, true>(c, inj, n, nrec, taps, (T *)traces, st, tm);
        else if (fused) fused_step<T, false>(c, inj, n, nrec, taps, (T *)traces, st, tm);
        else if (c->opts.free_surface) step<T, true>(c, G, inj, n, nrec, taps, (T *)traces, st, tm);
        else step<T, false>(c, G, inj, n, nrec, taps, (T *)traces, st, tm);
    }
    HIP_TRY(hipGetLastError());
    const Grid<T> G = make_grid<T>(c);
    if (c->opts.check_finite) {
        int *flag = (int *)(c->ws + c->L.flag);
        fill_zero<int><<<1, 64, 0, st>>>(flag, 1);
        finite_check<T><<<1024, 256, 0, st>>>(G, flag);
        HIP_TRY(hipGetLastError());
        int h = 0;
        HIP_TRY(hipMemcpyAsync(&h, flag, sizeof h, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (h) return fail(FD3D_ENONFINITE, "non-finite value in the final state");
    }
    return FD3D_OK;
}

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
    for (int q = 0; q < 3; ++q) A.vst[q] = nullptr;
    for (int q = 0; q < 6; ++q) A.sst[q] = nullptr;
    return A;
}

// Fields of the four tiled adjoint passes of one step whose stored v^{n+1/2}, sigma^n
// sit in segment slot `slot`: grids (f[] re-pointed) and tile outputs.
template <typename T> struct AdjTiles {
    Grid<T> g[4];     // stress-A, velocity-A, velocity-B, stress-B
    TileIO<T> io[4];
};

template <typename T> AdjTiles<T> adj_tiles(const Grid<T> &G, char *gws, const GradLayout &GL, const char *slot)
{
    auto fld = [&](size_t base, int q) { return (T *)(gws + base + q * GL.fstep); };
    AdjTiles<T> P;
    for (int p = 0; p < 4; ++p) {
        P.g[p] = G;
        for (int f = 0; f < NFIELD; ++f) P.g[p].save[f] = nullptr;
        std::memset(&P.io[p], 0, sizeof P.io[p]);
    }
    for (int q = 0; q < 3; ++q) {
        P.g[0].f[VX + q] = (T *)(slot + q * GL.fstep);  // stored v^{n+1/2}
        P.g[1].f[VX + q] = fld(GL.adj, VX + q);           // A_v
        P.g[2].f[VX + q] = fld(GL.adj, VX + q);
        P.g[3].f[VX + q] = fld(GL.scr, 6 + q);            // Y
        P.io[2].acc[q] = fld(GL.acc, 5 + q);              // g_b
        P.io[2].out[q] = fld(GL.scr, 6 + q);
    }
    for (int q = 0; q < 6; ++q) {
        P.g[0].f[SXX + q] = fld(GL.adj, SXX + q);           // A_s
        P.g[1].f[SXX + q] = fld(GL.scr, q);                 // X
        P.g[2].f[SXX + q] = (T *)(slot + (3 + q) * GL.fstep);  // stored sigma^n
        P.g[3].f[SXX + q] = fld(GL.adj, SXX + q);
        P.io[0].out[q] = fld(GL.scr, q);
    }
    for (int q = 0; q < 5; ++q) P.io[0].acc[q] = fld(GL.acc, q);  // gl, gm, g_mu_xy, g_mu_xz, g_mu_yz
    return P;
}

// Zero the adjoint state, accumulators and intermediate fields, and the segment slots
// (whose samples at the pinned staggered positions are never stored and must read 0).
template <typename T> void zero_grad_fields(char *gws, const GradLayout &GL, hipStream_t st)
{
    fill_zero<T><<<2048, 256, 0, st>>>((T *)(gws + GL.adj), (long)((GL.ckpt - GL.adj) / sizeof(T)));
    fill_zero<T><<<2048, 256, 0, st>>>((T *)(gws + GL.seg), (long)((size_t)GL.k * GL.group / sizeof(T)));
}

// Reverse sweep over the checkpointed segments: recompute each segment (storing
// v^{n+1/2} and sigma^n per step), then run the adjoint steps backwards; finally map
// the staggered-point gradients to the node arrays (accumulated into g_*).
template <typename T>
int adjoint_impl(fd3d_ctx *c, const fd3d_source *src, int nrec, const double *rec_pos, const T *residual, T *g_lam,
                 T *g_mu, T *g_rho, char *gws, const GradLayout &GL, hipStream_t st)
{
    Inject<T> inj;
    int rc = stage_inputs<T>(c, src, inj, nrec, rec_pos, st);
    if (rc) return rc;
    Grid<T> G = make_grid<T>(c);
    AdjGrid<T> A = make_adj<T>(gws, GL);
    zero_grad_fields<T>(gws, GL, st);
    const RecTap<T> *taps = (const RecTap<T> *)(c->ws + c->L.rec);
    const int *colors = (const int *)(c->ws + c->L.colors);
    const dim3 blk(64, 4, 1), grd((G.nx + 63) / 64, (G.ny + 3) / 4, G.nz);
    const bool tiled = c->variant != FD3D_KERNEL_CELL;  // the fused variant recomputes with tiles
    Timer tm{c, st};
    Inject<T> none;
    std::memset(&none, 0, sizeof none);
    for (int f = 0; f < NFIELD; ++f) none.i0[f] = none.j0[f] = none.k0[f] = -(1 << 28);
    auto inject = [&](int n) {
        for (size_t col = 0; col + 1 < c->color_off.size(); ++col) {
            const int cnt = c->color_off[col + 1] - c->color_off[col];
            inject_residual<T><<<(3 * cnt + 255) / 256, 256, 0, st>>>(A.a[VX], A.a[VY], A.a[VZ], taps,
                                                                     colors + c->color_off[col], cnt, residual,
                                                                     c->nt, n);
        }
    };
    for (int sgi = GL.nseg - 1; sgi >= 0; --sgi) {
        const int n0 = sgi * GL.k, n1 = std::min(n0 + GL.k, c->nt);
        const char *ck = gws + GL.ckpt + (size_t)sgi * GL.group;
        for (int q = 0; q < NFIELD; ++q)
            HIP_TRY(hipMemcpyAsync(state_chunk<T>(c, G, q), ck + q * GL.chunk, c->L.field_bytes,
                                   hipMemcpyDeviceToDevice, st));
        for (int n = n0; n < n1; ++n) {
            char *slot = gws + GL.seg + (size_t)(n - n0) * GL.group;
            Grid<T> Gs = G;
            for (int f = 0; f < NFIELD; ++f) Gs.save[f] = (T *)(slot + f * GL.fstep);
            if (c->opts.free_surface) step<T, true>(c, Gs, inj, n, 0, taps, nullptr, st, tm);
            else step<T, false>(c, Gs, inj, n, 0, taps, nullptr, st, tm);
        }
        for (int n = n1 - 1; n >= n0; --n) {
            const char *slot = gws + GL.seg + (size_t)(n - n0) * GL.group;
            if (tiled) {
                const AdjTiles<T> P = adj_tiles<T>(G, gws, GL, slot);
                launch_pass<T, false>(c, P.g[0], none, n, kPassStressA, st, P.io[0]);
                launch_pass<T, false>(c, P.g[1], none, n, kPassVelA, st, P.io[1]);
                inject(n);
                launch_pass<T, false>(c, P.g[2], inj, n, kPassVelB, st, P.io[2]);
                launch_pass<T, false>(c, P.g[3], none, n, kPassStressB, st, P.io[3]);
            } else {
                for (int q = 0; q < 3; ++q) A.vst[q] = (const T *)(slot + q * GL.fstep);
                for (int q = 0; q < 6; ++q) A.sst[q] = (const T *)(slot + (3 + q) * GL.fstep);
                adj_stress_cell<T><<<grd, blk, 0, st>>>(G, A);
                inject(n);
                adj_vel_cell<T><<<grd, blk, 0, st>>>(G, A, inj, n);
            }
        }
    }
    grad_finalize<T><<<grd, blk, 0, st>>>(G, A, g_lam, g_mu, g_rho);
    HIP_TRY(hipGetLastError());
    return FD3D_OK;
}

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

template <typename T> int set_state_impl(fd3d_ctx *c, const void *const fields[9], hipStream_t st)
{
    const Grid<T> G = make_grid<T>(c);
    for (int f = 0; f < NFIELD; ++f) copy_field<T>(c, G.f[f], true, (const T *)fields[f], false, f, st);
    HIP_TRY(hipGetLastError());
    return FD3D_OK;
}

} // namespace

// ---------------------------------------------------------------------------------
// Batches: many contexts (uneven grids, own models, sources and receivers) stepped
// together, one persistent launch per pass for all shots, optionally captured once as
// a hipGraph holding the whole nt-step sequence.
//
// Schedules.  Lockstep: every launch covers every shot, and the shots advance one step
// at a time together.  Cache-blocked groups: the shots, taken from the smallest working
// set (nine fields and three model arrays) to the largest, are cut into runs whose
// working sets add up to at most a given number of bytes; one group runs all its nt
// steps (one launch per pass over the group's shots) before the next group starts.  Sized to the last-level (Infinity)
// cache, a group's fields stay resident from one step to the next.  Shots are
// independent, so both schedules give every shot the same result bit for bit.

// Shots at positions [s0, s0 + ns) of the batch's schedule order, stepped by one launch per pass: their work items and
// receiver components (counted from the group's first), the persistent grid size and
// the tile shapes of the launch (tx2 = 0: one shape).
struct BatchGroup {
    int s0, ns, tiles, recs, wgs;
    int tx, ty, tx2, ty2;
    int vac;  // some shot of the group has a vacuum surface
    int ntp;  // cache policy of the group's forward passes (see group_streams)
};

struct fd3d_batch {
    int nshot;
    std::vector<fd3d_ctx *> ctx;
    int tsize, nt, fs;
    char *ws;
    size_t ws_bytes;
    size_t off_fwd, off_rec;
    int tile_x, tile_y, wgs_req;
    int tile2_x, tile2_y;  // optional second tile shape (same workgroup size), 0: none
    size_t group_bytes;    // 0: lockstep; otherwise the cache-blocked group budget
    std::vector<BatchGroup> groups;
    std::vector<int> order;  // shot at each position of the descriptor arrays
    std::vector<unsigned char> fwd_host, rec_host;
    hipEvent_t staged;
    bool staged_pending;
    hipStream_t cap;
    std::vector<unsigned char> grad_host;  // batched-gradient descriptors, kept for the async upload
    hipGraph_t graph;
    hipGraphExec_t gexec;
    bool graph_valid;
    long graph_key;
};

namespace {

size_t batch_desc_bytes(int nshot, int tsize)
{
    const size_t f = tsize == 8 ? sizeof(ShotFwd<double>) : sizeof(ShotFwd<float>);
    const size_t r = tsize == 8 ? sizeof(ShotRec<double>) : sizeof(ShotRec<float>);
    return round_up((size_t)nshot * f, kAlign) + round_up((size_t)nshot * r, kAlign);
}

// Supported pairs of batch tile shapes (primary, second; equal workgroup sizes): FP32
// 256x4 + 64x16, 128x8 + 64x16, 256x4 + 128x8, 128x4 + 64x8; FP64 128x4 + 64x8.
bool pair_supported(int tsize, int tx, int ty, int tx2, int ty2)
{
    const long key = ((long)tx * 1000 + ty) * 1000000 + tx2 * 1000 + ty2;
    if (key == 128004064008L) return true;
    if (tsize == 8) return false;
    return key == 256004064016L || key == 128008064016L || key == 256004128008L;
}

// Calls f(TX, TY, TX2, TY2) with a launch's tile shapes as integral constants (TX2 = 0:
// one shape).
template <typename T, typename F> decltype(auto) with_batch_tiles(const BatchGroup &b, F &&f)
{
    using Z = std::integral_constant<int, 0>;
    if (b.tx2 == 0)
        return with_tile<T>(b.tx, b.ty, [&](auto tx, auto ty) { return f(tx, ty, Z{}, Z{}); });
    using X64 = std::integral_constant<int, 64>;
    using X128 = std::integral_constant<int, 128>;
    using X256 = std::integral_constant<int, 256>;
    using Y4 = std::integral_constant<int, 4>;
    using Y8 = std::integral_constant<int, 8>;
    using Y16 = std::integral_constant<int, 16>;
    if constexpr (sizeof(T) == 4) {
        if (b.tx == 256 && b.tx2 == 64) return f(X256{}, Y4{}, X64{}, Y16{});
        if (b.tx == 128 && b.ty == 8) return f(X128{}, Y8{}, X64{}, Y16{});
        if (b.tx == 256 && b.tx2 == 128) return f(X256{}, Y4{}, X128{}, Y8{});
    }
    return f(X128{}, Y4{}, X64{}, Y8{});
}

// Two contexts whose passes read the same model arrays (the caller's, in place: a context
// with interleaved rows reads its own copy).
bool shares_model(const fd3d_ctx *a, const fd3d_ctx *b)
{
    return !a->L.model && !b->L.model && (a->lam == b->lam || a->mu == b->mu || a->rho == b->rho);
}

// Streaming (non-temporal) policy for the forward passes of a group of contexts, as
// stream_model for one grid: FP32, the group's working sets add up to more than the
// Infinity Cache, and no two of its shots share a model array (a shared model is re-read
// by the other shots' tiles of the same launch).
bool group_streams(const fd3d_ctx *const *ctx, int ns)
{
    if (ns < 1 || ctx[0]->tsize != 4) return false;
    double bytes = 0.0;
    for (int q = 0; q < ns; ++q) {
        bytes += 12.0 * (double)ctx[q]->n[0] * (double)ctx[q]->n[1] * (double)ctx[q]->n[2] * (double)ctx[q]->tsize;
        for (int r = 0; r < q; ++r)
            if (shares_model(ctx[q], ctx[r])) return false;
    }
    return bytes > kInfinityCacheBytes;
}

// The batch's own tile shapes as one group covering every shot (counts not filled in).
BatchGroup whole_batch(const fd3d_batch *b)
{
    BatchGroup g{};
    g.s0 = 0;
    g.ns = b->nshot;
    g.tx = b->tile_x;
    g.ty = b->tile_y;
    g.tx2 = b->tile2_x;
    g.ty2 = b->tile2_y;
    g.ntp = group_streams(b->ctx.data(), b->nshot);
    return g;
}

// Tile map of one shot of a launch, and whether it uses the launch's second tile shape
// (when that covers its rows with fewer idle columns).
TileMap shot_tiles(const BatchGroup &b, const fd3d_ctx *c, int &alt)
{
    int tx = b.tx, ty = b.ty;
    alt = 0;
    if (b.tx2 > 0) {
        const int pad1 = (c->n[0] + tx - 1) / tx * tx, pad2 = (c->n[0] + b.tx2 - 1) / b.tx2 * b.tx2;
        if (pad2 < pad1) {
            alt = 1;
            tx = b.tx2;
            ty = b.ty2;
        }
    }
    TileMap tm;
    tm.ntx = (c->n[0] + tx - 1) / tx;
    tm.nty = (c->n[1] + ty - 1) / ty;
    tm.zc = c->zchunk;
    tm.nzc = (c->n[2] + c->zchunk - 1) / c->zchunk;
    return tm;
}

// One pass over the shots of group gr; d points at the group's first descriptor.  A
// forward stress pass given r (the group's receiver descriptors) also samples them.
template <typename T, int TX, int TY, int TX2, int TY2, bool FS>
int launch_multi(const BatchGroup &gr, const ShotFwd<T> *d, int n, int pass, hipStream_t st,
                 const ShotRec<T> *r = nullptr, int nt = 0)
{
    const int g = gr.wgs, S = gr.ns, W = gr.tiles;
    constexpr int NT = TX * TY;
    const RecMulti<T> rec{r, S, (r && pass == kPassStress) ? gr.recs : 0, nt, g};
    const RecMulti<T> none{nullptr, 0, 0, 0, g};
    const int gs = g + rec_blocks(rec, NT);
    if constexpr (!FS) {  // groups with a vacuum surface: the forward passes' own instantiations
        if (gr.vac && pass == kPassVel) {
            vel_tile_multi<T, TX, TY, TX2, TY2, false, kFwd, true><<<g, NT, 0, st>>>(d, S, W, n);
            return FD3D_OK;
        }
        if (gr.vac && pass == kPassStress) {
            stress_tile_multi<T, TX, TY, TX2, TY2, false, kFwd, true><<<gs, NT, 0, st>>>(d, S, W, n, rec);
            return FD3D_OK;
        }
    }
    if constexpr (sizeof(T) == 4) {  // forward passes of a streaming group (see group_streams)
        if (gr.ntp && pass == kPassVel) {
            vel_tile_multi<T, TX, TY, TX2, TY2, FS, kFwd, false, true><<<g, NT, 0, st>>>(d, S, W, n);
            return FD3D_OK;
        }
        if (gr.ntp && pass == kPassStress) {
            stress_tile_multi<T, TX, TY, TX2, TY2, FS, kFwd, false, true><<<gs, NT, 0, st>>>(d, S, W, n, rec);
            return FD3D_OK;
        }
    }
    switch (pass) {
    case kPassVel: vel_tile_multi<T, TX, TY, TX2, TY2, FS><<<g, NT, 0, st>>>(d, S, W, n); break;
    case kPassStress: stress_tile_multi<T, TX, TY, TX2, TY2, FS><<<gs, NT, 0, st>>>(d, S, W, n, rec); break;
    case kPassVelSave: vel_tile_multi<T, TX, TY, TX2, TY2, FS, kFwdSave><<<g, NT, 0, st>>>(d, S, W, n); break;
    case kPassStressSave:
        stress_tile_multi<T, TX, TY, TX2, TY2, FS, kFwdSave><<<g, NT, 0, st>>>(d, S, W, n, none);
        break;
    case kPassStressA: stress_tile_multi<T, TX, TY, TX2, TY2, false, kAdjA><<<g, NT, 0, st>>>(d, S, W, n, none); break;
    case kPassVelA: vel_tile_multi<T, TX, TY, TX2, TY2, false, kAdjA><<<g, NT, 0, st>>>(d, S, W, n); break;
    case kPassVelB: vel_tile_multi<T, TX, TY, TX2, TY2, false, kAdjB><<<g, NT, 0, st>>>(d, S, W, n); break;
    default: stress_tile_multi<T, TX, TY, TX2, TY2, false, kAdjB><<<g, NT, 0, st>>>(d, S, W, n, none); break;
    }
    return FD3D_OK;
}

template <typename T, bool FS>
int multi_pass(const BatchGroup &b, const ShotFwd<T> *d, int n, int pass, hipStream_t st, const ShotRec<T> *r = nullptr,
               int nt = 0)
{
    return with_batch_tiles<T>(b, [&](auto tx, auto ty, auto tx2, auto ty2) {
        return launch_multi<T, decltype(tx)::value, decltype(ty)::value, decltype(tx2)::value, decltype(ty2)::value,
                            FS>(b, d, n, pass, st, r, nt);
    });
}

template <typename T, bool FS> int multi_occupancy(const BatchGroup &b)
{
    return with_batch_tiles<T>(b, [&](auto tx, auto ty, auto tx2, auto ty2) {
        constexpr int TX = decltype(tx)::value, TY = decltype(ty)::value;
        constexpr int TX2 = decltype(tx2)::value, TY2 = decltype(ty2)::value;
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, vel_tile_multi<T, TX, TY, TX2, TY2, FS>, TX * TY, 0) !=
            hipSuccess)
            occ = 1;
        return occ > 0 ? occ : 1;
    });
}

// The whole nt-step sequence of a batch on one stream (also what a graph captures):
// group after group, each through all its steps.
template <typename T> int batch_sequence(fd3d_batch *b, int flags, hipStream_t st)
{
    if (!(flags & FD3D_KEEP_STATE))
        for (fd3d_ctx *c : b->ctx) zero_fields<T>(c, st);
    for (const BatchGroup &g : b->groups) {
        const ShotRec<T> *r = (const ShotRec<T> *)(b->ws + b->off_rec) + g.s0;
        const ShotFwd<T> *d = (const ShotFwd<T> *)(b->ws + b->off_fwd) + g.s0;
        for (int n = 0; n < b->nt; ++n) {
            if (b->fs) multi_pass<T, true>(g, d, n, kPassVel, st);
            else multi_pass<T, false>(g, d, n, kPassVel, st);
            // the stress launch also samples the receivers
            if (b->fs) multi_pass<T, true>(g, d, n, kPassStress, st, r, b->nt);
            else multi_pass<T, false>(g, d, n, kPassStress, st, r, b->nt);
        }
    }
    HIP_TRY(hipGetLastError());
    return FD3D_OK;
}

// Working set of one shot in the step loop: nine fields and the three model arrays.
size_t shot_footprint(const fd3d_ctx *c) { return (size_t)12 * c->n[0] * c->n[1] * c->n[2] * c->tsize; }

// Groups of the batch's schedule and their tile shapes.  A cache-blocked group whose
// shots all run the tile kernel with one shape of their own uses that shape (each
// shot's tuned kernel); otherwise a group uses the batch's shapes.
void make_groups(fd3d_batch *b)
{
    b->groups.clear();
    b->order.resize(b->nshot);
    for (int s = 0; s < b->nshot; ++s) b->order[s] = s;
    const BatchGroup all = whole_batch(b);
    if (b->group_bytes == 0) {
        b->groups.push_back(all);
        return;
    }
    std::stable_sort(b->order.begin(), b->order.end(),
                     [&](int x, int y) { return shot_footprint(b->ctx[x]) < shot_footprint(b->ctx[y]); });
    auto ctx_at = [&](int p) { return b->ctx[b->order[p]]; };
    int s = 0;
    while (s < b->nshot) {
        BatchGroup g = all;
        g.s0 = s;
        size_t bytes = shot_footprint(ctx_at(s));
        int e = s + 1;
        while (e < b->nshot && bytes + shot_footprint(ctx_at(e)) <= b->group_bytes) bytes += shot_footprint(ctx_at(e++));
        g.ns = e - s;
        std::vector<const fd3d_ctx *> members;
        for (int q = s; q < e; ++q) members.push_back(ctx_at(q));
        g.ntp = group_streams(members.data(), g.ns);
        const fd3d_ctx *c0 = ctx_at(s);
        bool same = c0->variant == FD3D_KERNEL_TILE;
        for (int q = s + 1; q < e && same; ++q)
            same = ctx_at(q)->variant == FD3D_KERNEL_TILE && ctx_at(q)->tile_x == c0->tile_x &&
                   ctx_at(q)->tile_y == c0->tile_y;
        if (same && tile_supported(b->tsize, c0->tile_x, c0->tile_y)) {
            g.tx = c0->tile_x;
            g.ty = c0->tile_y;
            g.tx2 = g.ty2 = 0;
        }
        b->groups.push_back(g);
        s = e;
    }
}

template <typename T>
int batch_forward_impl(fd3d_batch *b, const fd3d_source *srcs, const int *nrec, const double *const *rec_pos,
                       void *const *traces, int flags, int use_graph, hipStream_t st)
{
    std::vector<ShotFwd<T>> fw(b->nshot);
    std::vector<ShotRec<T>> rr(b->nshot);
    make_groups(b);
    size_t gi = 0;
    int tiles = 0, recs = 0;
    for (int p = 0; p < b->nshot; ++p) {  // position p of the schedule order holds shot s
        const int s = b->order[p];
        fd3d_ctx *c = b->ctx[s];
        BatchGroup &grp = b->groups[gi];
        if (p == grp.s0) tiles = recs = grp.vac = 0;  // work items and receivers count from the group's first
        if (c->opts.vacuum_top > 0) grp.vac = 1;
        if (!window_ok(c, c->zchunk))
            return fail(FD3D_EINVAL, "shot " + std::to_string(s) + ": zchunk too large for a tile sweep");
        const int nr = nrec ? nrec[s] : 0;
        if (nr < 0 || nr > c->opts.max_receivers) return fail(FD3D_EINVAL, "shot " + std::to_string(s) + ": bad nrec");
        if (nr > 0 && (!rec_pos || !rec_pos[s] || !traces || !traces[s]))
            return fail(FD3D_EINVAL, "shot " + std::to_string(s) + ": rec_pos/traces is NULL");
        const int rc = stage_inputs<T>(c, srcs ? &srcs[s] : nullptr, fw[p].src, nr, nr ? rec_pos[s] : nullptr, st);
        if (rc) return fail(rc, "shot " + std::to_string(s) + ": " + g_err);
        fw[p].G = make_grid<T>(c);
        const TileMap tm = shot_tiles(grp, c, fw[p].alt);
        fw[p].tm = tm;
        fw[p].base = tiles;
        tiles += tm.ntx * tm.nty * tm.nzc;
        for (int q = 0; q < 3; ++q) rr[p].v[q] = fw[p].G.f[VX + q];
        rr[p].taps = (const RecTap<T> *)(c->ws + c->L.rec);
        rr[p].traces = nr ? (T *)traces[s] : nullptr;
        rr[p].nrec = nr;
        rr[p].base = recs;
        recs += 3 * nr;
        if (p == grp.s0 + grp.ns - 1) {
            grp.tiles = tiles;
            grp.recs = recs;
            ++gi;
        }
    }
    if (b->staged_pending) {
        HIP_TRY(hipEventSynchronize(b->staged));
        b->staged_pending = false;
    }
    b->fwd_host.assign((const unsigned char *)fw.data(), (const unsigned char *)(fw.data() + b->nshot));
    b->rec_host.assign((const unsigned char *)rr.data(), (const unsigned char *)(rr.data() + b->nshot));
    HIP_TRY(hipMemcpyAsync(b->ws + b->off_fwd, b->fwd_host.data(), b->fwd_host.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(b->ws + b->off_rec, b->rec_host.data(), b->rec_host.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(b->staged, st));
    b->staged_pending = true;

    // persistent grid per group: a multiple of 8 workgroups (one chunk of the list per XCD)
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    // the graph is reused while every launch of the sequence is unchanged
    uint64_t key = 1469598103934665603ull;
    auto mix = [&](long v) { key = (key ^ (uint64_t)v) * 1099511628211ull; };
    mix(flags & FD3D_KEEP_STATE);
    for (BatchGroup &g : b->groups) {
        const int occ = b->fs ? multi_occupancy<T, true>(g) : multi_occupancy<T, false>(g);
        int wgs = b->wgs_req > 0 ? b->wgs_req : cus * occ;
        wgs = std::min(wgs, ((g.tiles + 7) / 8) * 8);
        g.wgs = std::max(8, (wgs + 7) / 8 * 8);
        for (long v : {(long)g.s0, (long)g.ns, (long)g.tiles, (long)g.recs, (long)g.wgs, (long)g.tx, (long)g.ty,
                       (long)g.tx2, (long)g.ty2, (long)g.vac})
            mix(v);
    }
    if (!use_graph) return batch_sequence<T>(b, flags, st);
    if (!b->graph_valid || b->graph_key != (long)key) {
        if (b->graph_valid) {
            (void)hipGraphExecDestroy(b->gexec);
            (void)hipGraphDestroy(b->graph);
            b->graph_valid = false;
        }
        HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
        const int rc = batch_sequence<T>(b, flags, b->cap);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->cap, &g);
        if (rc || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);  // a partial capture is not kept
            if (rc) return rc;
            return fail(FD3D_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        }
        b->graph = g;
        HIP_TRY(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
        b->graph_valid = true;
        b->graph_key = (long)key;
    }
    HIP_TRY(hipGraphLaunch(b->gexec, st));
    return FD3D_OK;
}

int check_gws(const fd3d_ctx *ctx, void *gws, size_t gws_bytes, int k)
{
    if (ctx->opts.free_surface || ctx->opts.vacuum_top)
        return fail(FD3D_EINVAL, "the gradient supports damped boundaries only (no free surface)");
    if (coarse_on(ctx->opts)) return fail(FD3D_EINVAL, "the gradient needs the medium at the simulation nodes");
    if (ctx->nt < 1) return fail(FD3D_EINVAL, "gradient needs nt >= 1");
    if (k < 1 || k > ctx->nt) return fail(FD3D_EINVAL, "ckpt_every must be in [1, nt]");
    if (!gws || ((uintptr_t)gws % kAlign)) return fail(FD3D_EINVAL, "gradient workspace must be 256-byte aligned");
    const size_t need = make_grad_layout(ctx, k).total;
    if (gws_bytes < need) return fail(FD3D_EWS, "gradient workspace too small: need " + std::to_string(need) + " bytes");
    return FD3D_OK;
}

// ---- batched gradient ----------------------------------------------------------
// Batch workspace of fd3d_batch_gradient: descriptor arrays (nshot entries each) of the
// forward pass, of the segment recompute per segment slot m (store pointers of slot m),
// of the adjoint passes (stress-A and velocity-B per slot m, which read the fields
// stored in slot m; velocity-A and stress-B once), of the residual injection, and per
// checkpoint the save and restore copy lists.
struct BatchGradLayout {
    size_t fwd0, fwd_slot, sa_slot, vb_slot, va, sb, inj, save_copy, rest_copy, total;
    size_t fwd_bytes, inj_bytes, copy_bytes;
    int k, nseg;
};

template <typename T> BatchGradLayout make_batch_grad_layout(const fd3d_batch *b, int k)
{
    BatchGradLayout L{};
    L.k = k;
    L.nseg = (b->nt + k - 1) / k;
    L.fwd_bytes = round_up((size_t)b->nshot * sizeof(ShotFwd<T>), kAlign);
    L.inj_bytes = round_up((size_t)b->nshot * sizeof(ShotInject<T>), kAlign);
    L.copy_bytes = round_up((size_t)b->nshot * 9 * sizeof(CopyDesc<T>), kAlign);
    size_t off = 0;
    L.fwd0 = off;
    off += L.fwd_bytes;
    L.fwd_slot = off;
    off += (size_t)k * L.fwd_bytes;
    L.sa_slot = off;
    off += (size_t)k * L.fwd_bytes;
    L.vb_slot = off;
    off += (size_t)k * L.fwd_bytes;
    L.va = off;
    off += L.fwd_bytes;
    L.sb = off;
    off += L.fwd_bytes;
    L.inj = off;
    off += L.inj_bytes;
    L.save_copy = off;
    off += (size_t)L.nseg * L.copy_bytes;
    L.rest_copy = off;
    off += (size_t)L.nseg * L.copy_bytes;
    L.total = off;
    return L;
}

template <typename T>
int batch_gradient_impl(fd3d_batch *b, const fd3d_source *srcs, const int *nrec, const double *const *rec_pos,
                        const void *const *d_obs, void *const *traces, void *const *misfit, void *const *g_lam,
                        void *const *g_mu, void *const *g_rho, void *const *gws, const size_t *gws_bytes, int k,
                        int flags, char *bws, size_t bws_bytes, hipStream_t st)
{
    const int S = b->nshot;
    const BatchGradLayout BL = make_batch_grad_layout<T>(b, k);
    if (!bws || ((uintptr_t)bws % kAlign)) return fail(FD3D_EINVAL, "batch gradient workspace must be 256-byte aligned");
    if (bws_bytes < BL.total) return fail(FD3D_EWS, "batch gradient workspace too small: need " + std::to_string(BL.total));
    std::vector<GradLayout> GL(S);
    std::vector<ShotFwd<T>> fw(S);
    std::vector<ShotRec<T>> rr(S);
    std::vector<ShotInject<T>> ij(S);
    std::vector<AdjGrid<T>> ag(S);
    int tiles = 0, recs = 0, ncol = 0;
    int cbase[kMaxBatchColors] = {0, 0, 0, 0};
    BatchGroup all = whole_batch(b);  // every shot in each launch (lockstep)
    for (int s = 0; s < S; ++s) {
        fd3d_ctx *c = b->ctx[s];
        const std::string tag = "shot " + std::to_string(s) + ": ";
        if (!window_ok(c, c->zchunk)) return fail(FD3D_EINVAL, tag + "zchunk too large for a tile sweep");
        if (!gws || !gws[s]) return fail(FD3D_EINVAL, tag + "gradient workspace is NULL");
        int rc = check_gws(c, gws[s], gws_bytes[s], k);
        if (rc) return fail(rc, tag + g_err);
        const int nr = nrec ? nrec[s] : 0;
        if (nr < 1 || nr > c->opts.max_receivers) return fail(FD3D_EINVAL, tag + "needs 1..max_receivers receivers");
        if (!rec_pos || !rec_pos[s] || !traces || !traces[s] || !d_obs || !d_obs[s] || !g_lam || !g_lam[s] || !g_mu ||
            !g_mu[s] || !g_rho || !g_rho[s])
            return fail(FD3D_EINVAL, tag + "NULL pointer");
        rc = stage_inputs<T>(c, srcs ? &srcs[s] : nullptr, fw[s].src, nr, rec_pos[s], st);
        if (rc) return fail(rc, tag + g_err);
        const int cols = (int)c->color_off.size() - 1;
        if (cols > kMaxBatchColors) return fail(FD3D_EINVAL, tag + "receivers need more than 4 tap-disjoint colours");
        ncol = std::max(ncol, cols);
        GL[s] = make_grad_layout(c, k);
        fw[s].G = make_grid<T>(c);
        std::memset(&fw[s].io, 0, sizeof fw[s].io);
        const TileMap tm = shot_tiles(all, c, fw[s].alt);
        fw[s].tm = tm;
        fw[s].base = tiles;
        tiles += tm.ntx * tm.nty * tm.nzc;
        for (int q = 0; q < 3; ++q) rr[s].v[q] = fw[s].G.f[VX + q];
        rr[s].taps = (const RecTap<T> *)(c->ws + c->L.rec);
        rr[s].traces = (T *)traces[s];
        rr[s].nrec = nr;
        rr[s].base = recs;
        recs += 3 * nr;
        ag[s] = make_adj<T>((char *)gws[s], GL[s]);
        ShotInject<T> &a = ij[s];
        for (int q = 0; q < 3; ++q) a.a[q] = ag[s].a[VX + q];
        a.taps = rr[s].taps;
        a.colors = (const int *)(c->ws + c->L.colors);
        a.res = (const T *)((char *)gws[s] + GL[s].res);
        for (int q = 0; q <= kMaxBatchColors; ++q) a.coff[q] = c->color_off[std::min(q, cols)];
        for (int q = 0; q < kMaxBatchColors; ++q) {
            a.rbase[q] = cbase[q];
            cbase[q] += 3 * (a.coff[q + 1] - a.coff[q]);
        }
    }
    // host images of every descriptor array
    if (b->staged_pending) {
        HIP_TRY(hipEventSynchronize(b->staged));
        b->staged_pending = false;
    }
    b->grad_host.assign(BL.total, 0);
    unsigned char *h = b->grad_host.data();
    const size_t fbytes = S * sizeof(ShotFwd<T>);
    std::memcpy(h + BL.fwd0, fw.data(), fbytes);
    // descriptors of one adjoint pass: the shot's tile map and sources, the pass's grid and outputs
    auto adj_desc = [&](int s, const AdjTiles<T> &P, int p, bool with_src) {
        ShotFwd<T> d = fw[s];
        d.G = P.g[p];
        d.io = P.io[p];
        if (!with_src) {
            std::memset(&d.src, 0, sizeof d.src);
            for (int f = 0; f < NFIELD; ++f) d.src.i0[f] = d.src.j0[f] = d.src.k0[f] = -(1 << 28);
        }
        return d;
    };
    std::vector<ShotFwd<T>> va(S), sb(S);
    for (int m = 0; m < k; ++m) {
        std::vector<ShotFwd<T>> f2 = fw, sa(S), vb(S);
        for (int s = 0; s < S; ++s) {
            char *slot = (char *)gws[s] + GL[s].seg + (size_t)m * GL[s].group;
            for (int f = 0; f < NFIELD; ++f) f2[s].G.save[f] = (T *)(slot + f * GL[s].fstep);
            const AdjTiles<T> P = adj_tiles<T>(fw[s].G, (char *)gws[s], GL[s], slot);
            sa[s] = adj_desc(s, P, 0, false);
            vb[s] = adj_desc(s, P, 2, true);
            if (m == 0) {
                va[s] = adj_desc(s, P, 1, false);
                sb[s] = adj_desc(s, P, 3, false);
            }
        }
        std::memcpy(h + BL.fwd_slot + m * BL.fwd_bytes, f2.data(), fbytes);
        std::memcpy(h + BL.sa_slot + m * BL.fwd_bytes, sa.data(), fbytes);
        std::memcpy(h + BL.vb_slot + m * BL.fwd_bytes, vb.data(), fbytes);
    }
    std::memcpy(h + BL.va, va.data(), fbytes);
    std::memcpy(h + BL.sb, sb.data(), fbytes);
    std::memcpy(h + BL.inj, ij.data(), S * sizeof(ShotInject<T>));
    for (int cidx = 0; cidx < BL.nseg; ++cidx) {
        std::vector<CopyDesc<T>> sv(S * 9), rs(S * 9);
        for (int s = 0; s < S; ++s) {
            char *ck = (char *)gws[s] + GL[s].ckpt + (size_t)cidx * GL[s].group;
            const long n = (long)(b->ctx[s]->L.field_bytes / sizeof(T));
            for (int q = 0; q < NFIELD; ++q) {
                T *live = (T *)state_chunk<T>(b->ctx[s], fw[s].G, q), *kept = (T *)(ck + q * GL[s].chunk);
                sv[s * 9 + q] = CopyDesc<T>{live, kept, n};
                rs[s * 9 + q] = CopyDesc<T>{kept, live, n};
            }
        }
        std::memcpy(h + BL.save_copy + cidx * BL.copy_bytes, sv.data(), sv.size() * sizeof(CopyDesc<T>));
        std::memcpy(h + BL.rest_copy + cidx * BL.copy_bytes, rs.data(), rs.size() * sizeof(CopyDesc<T>));
    }
    b->rec_host.assign((const unsigned char *)rr.data(), (const unsigned char *)(rr.data() + S));
    HIP_TRY(hipMemcpyAsync(bws, h, BL.total, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(b->ws + b->off_rec, b->rec_host.data(), b->rec_host.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(b->staged, st));
    b->staged_pending = true;

    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int occ = multi_occupancy<T, false>(all);
    int wgs = b->wgs_req > 0 ? b->wgs_req : cus * occ;
    all.wgs = std::max(8, (std::min(wgs, ((tiles + 7) / 8) * 8) + 7) / 8 * 8);
    all.tiles = tiles;
    all.recs = recs;

    // forward with checkpoints
    auto desc = [&](size_t off) { return (const ShotFwd<T> *)(bws + off); };
    const ShotRec<T> *rdesc = (const ShotRec<T> *)(b->ws + b->off_rec);
    const ShotInject<T> *idesc = (const ShotInject<T> *)(bws + BL.inj);
    const dim3 cgrid(256, 9 * S);
    if (!(flags & FD3D_KEEP_STATE))
        for (fd3d_ctx *c : b->ctx) zero_fields<T>(c, st);
    auto pass = [&](const ShotFwd<T> *d, int n, int p, const ShotRec<T> *r = nullptr) {
        multi_pass<T, false>(all, d, n, p, st, r, b->nt);
    };
    for (int n = 0; n < b->nt; ++n) {
        if (n % k == 0)
            copy_multi<T><<<cgrid, 256, 0, st>>>((const CopyDesc<T> *)(bws + BL.save_copy + (n / k) * BL.copy_bytes));
        pass(desc(BL.fwd0), n, kPassVel);
        pass(desc(BL.fwd0), n, kPassStress, rdesc);  // also samples the receivers
    }
    // residuals and misfits, zeroed adjoint state, accumulators and segment slots
    for (int s = 0; s < S; ++s) {
        fd3d_ctx *c = b->ctx[s];
        const long nn = (long)nrec[s] * 3 * b->nt;
        double *part = (double *)(c->ws + c->L.part);
        T *res = (T *)((char *)gws[s] + GL[s].res);
        residual_misfit<T><<<kReduceBlocks, 256, 0, st>>>((const T *)traces[s], (const T *)d_obs[s], res, nn, part);
        misfit_final<T><<<1, 64, 0, st>>>(part, kReduceBlocks,
                                          misfit && misfit[s] ? (T *)misfit[s] : (T *)((char *)gws[s] + GL[s].misfit));
        zero_grad_fields<T>((char *)gws[s], GL[s], st);
    }
    // reverse sweep over the segments
    for (int sg = BL.nseg - 1; sg >= 0; --sg) {
        const int n0 = sg * k, n1 = std::min(n0 + k, b->nt);
        copy_multi<T><<<cgrid, 256, 0, st>>>((const CopyDesc<T> *)(bws + BL.rest_copy + sg * BL.copy_bytes));
        for (int n = n0; n < n1; ++n) {
            const ShotFwd<T> *d = desc(BL.fwd_slot + (n - n0) * BL.fwd_bytes);
            pass(d, n, kPassVelSave);
            pass(d, n, kPassStressSave);
        }
        for (int n = n1 - 1; n >= n0; --n) {
            pass(desc(BL.sa_slot + (n - n0) * BL.fwd_bytes), n, kPassStressA);
            pass(desc(BL.va), n, kPassVelA);
            for (int q = 0; q < ncol; ++q)
                if (cbase[q] > 0)
                    inject_residual_multi<T><<<(cbase[q] + 255) / 256, 256, 0, st>>>(idesc, S, q, cbase[q], b->nt, n);
            pass(desc(BL.vb_slot + (n - n0) * BL.fwd_bytes), n, kPassVelB);
            pass(desc(BL.sb), n, kPassStressB);
        }
    }
    // chain rule per shot, in shot order (shots may share the output arrays)
    for (int s = 0; s < S; ++s) {
        fd3d_ctx *c = b->ctx[s];
        const dim3 blk(64, 4, 1), grd((c->n[0] + 63) / 64, (c->n[1] + 3) / 4, c->n[2]);
        grad_finalize<T><<<grd, blk, 0, st>>>(fw[s].G, ag[s], (T *)g_lam[s], (T *)g_mu[s], (T *)g_rho[s]);
        c->grad_ws = (const char *)gws[s];
        c->grad_k = k;
        c->grad_ready = 1;
    }
    HIP_TRY(hipGetLastError());
    return FD3D_OK;
}

// Tangent-linear (Born) forward: the background steps on c and, interleaved, the
// perturbation's steps on dc (same grid and model) fed by the Born source kernels.
template <typename T>
int born_impl(fd3d_ctx *c, fd3d_ctx *dc, const fd3d_source *src, const void *dlam, const void *dmu,
              const void *drho, int nrec, const double *rec_pos, void *traces, void *dtraces, hipStream_t st)
{
    Inject<T> inj, dinj;
    int rc = stage_inputs<T>(c, src, inj, nrec, rec_pos, st);
    if (rc) return rc;
    rc = stage_inputs<T>(dc, nullptr, dinj, nrec, rec_pos, st);
    if (rc) return rc;
    zero_fields<T>(c, st);
    zero_fields<T>(dc, st);
    if (c->L.rows) {  // the perturbation into rows 3-5 of the model block, beside the model
        const void *in[3] = {dlam, dmu, drho};
        T *row[3];
        for (int q = 0; q < 3; ++q) {
            row[q] = (T *)(c->ws + c->L.model + (3 + q) * c->L.fstep);
            copy_field<T>(c, row[q], true, (const T *)in[q], false, -1, st);
        }
        dlam = row[0];
        dmu = row[1];
        drho = row[2];
    }
    const RecTap<T> *taps = (const RecTap<T> *)(c->ws + c->L.rec);
    const RecTap<T> *dtaps = (const RecTap<T> *)(dc->ws + dc->L.rec);
    const dim3 blk(64, 4, 1), grd((c->n[0] + 63) / 64, (c->n[1] + 3) / 4, c->n[2]);
    const Grid<T> G = make_grid<T>(c), D = make_grid<T>(dc);
    BornOut<T> dv, ds;
    for (int q = 0; q < 6; ++q) {
        dv.f[q] = q < 3 ? D.f[VX + q] : nullptr;
        ds.f[q] = D.f[SXX + q];
    }
    // the one-thread-per-cell source kernels for the cell variant
    auto born_source = [&](int n, bool vel) {
        if (vel) born_vel_source<T><<<grd, blk, 0, st>>>(G, dv, (const T *)drho, inj, n);
        else born_stress_source<T><<<grd, blk, 0, st>>>(G, ds, (const T *)dlam, (const T *)dmu);
    };
    const bool tiled = c->variant == FD3D_KERNEL_TILE;
    const TileMap tm = tile_map(c);
    const int nwg = tm.ntx * tm.nty * tm.nzc;
    const RecJob<T> recd = rec_job<T>(D.f[VX], D.f[VY], D.f[VZ], dtaps, nrec, c->nt, (T *)dtraces);
    const RecJob<T> recg = rec_job<T>(G.f[VX], G.f[VY], G.f[VZ], taps, traces ? nrec : 0, c->nt, (T *)traces);
    if (tiled) {
        // each source term in the background's pass that computes its derivatives (the Born
        // modes of the tile bodies), then the perturbation's own pass; the stress launches
        // sample the receivers
        TileIO<T> iovf, iosf;
        std::memset(&iovf, 0, sizeof iovf);
        std::memset(&iosf, 0, sizeof iosf);
        for (int q = 0; q < 3; ++q) iovf.out[q] = D.f[VX + q];
        iovf.acc[0] = (T *)drho;
        for (int q = 0; q < 6; ++q) iosf.out[q] = D.f[SXX + q];
        iosf.acc[0] = (T *)dlam;
        iosf.acc[1] = (T *)dmu;
        const bool ntp = sizeof(T) == 4 && stream_model(c);  // cache policy, as in launch_pass
        for (int n = 0; n < c->nt; ++n) {
            with_tile<T>(c->tile_x, c->tile_y, [&](auto tx, auto ty) {
                constexpr int TX = decltype(tx)::value, TY = decltype(ty)::value;
                if (ntp) vel_tile_adj<T, TX, TY, kBornV, sizeof(T) == 4><<<nwg, TX * TY, 0, st>>>(G, inj, n, tm, iovf);
                else vel_tile_adj<T, TX, TY, kBornV><<<nwg, TX * TY, 0, st>>>(G, inj, n, tm, iovf);
            });
            launch_pass<T, false>(dc, D, dinj, n, kPassVel, st);
            with_tile<T>(c->tile_x, c->tile_y, [&](auto tx, auto ty) {
                constexpr int TX = decltype(tx)::value, TY = decltype(ty)::value;
                const int nb = nwg + rec_blocks(recg, TX * TY);
                if (ntp) stress_tile_born<T, TX, TY, sizeof(T) == 4><<<nb, TX * TY, 0, st>>>(G, inj, n, tm, iosf, recg);
                else stress_tile_born<T, TX, TY><<<nb, TX * TY, 0, st>>>(G, inj, n, tm, iosf, recg);
            });
            launch_pass<T, false>(dc, D, dinj, n, kPassStress, st, TileIO<T>{}, recd);
        }
        HIP_TRY(hipGetLastError());
        return FD3D_OK;
    }
    for (int n = 0; n < c->nt; ++n) {
        born_source(n, true);
        launch_pass<T, false>(dc, D, dinj, n, kPassVel, st);
        launch_pass<T, false>(c, G, inj, n, kPassVel, st);
        born_source(n, false);
        // the stress launches sample the perturbation's and the background's receivers
        launch_pass<T, false>(dc, D, dinj, n, kPassStress, st, TileIO<T>{}, recd);
        launch_pass<T, false>(c, G, inj, n, kPassStress, st, TileIO<T>{}, recg);
    }
    HIP_TRY(hipGetLastError());
    return FD3D_OK;
}

} // namespace

extern "C" {

const char *fd3d_version(void) { return "fd3d 0.1.0 (gfx950)"; }

const char *fd3d_last_error(void) { return g_err.c_str(); }

int fd3d_workspace_bytes(int nx, int ny, int nz, const fd3d_opts *opts, size_t *bytes)
{
    if (!bytes) return fail(FD3D_EINVAL, "bytes is NULL");
    if (nx < 4 || ny < 4 || nz < 4) return fail(FD3D_EINVAL, "grid must have at least 4 nodes per axis");
    if ((double)nx * ny * nz >= 2147483647.0) return fail(FD3D_EINVAL, "grid must hold fewer than 2^31 nodes");
    fd3d_opts o = opts ? *opts : default_opts();
    int rc = check_opts(&o);
    if (rc) return rc;
    const int tsize = o.dtype == FD3D_F64 ? 8 : 4;
    if (o.layout == FD3D_LAYOUT_ROWS && !rows_fit(nx, ny, nz, tsize, std::min(4 + 8, nz)))
        return fail(FD3D_EINVAL, "opts.layout = FD3D_LAYOUT_ROWS: planes too large for interleaved rows "
                                 "(12 planes of 9 nx ny samples must fit 1 GiB)");
    *bytes = layout_of(nx, ny, nz, o).total;
    return FD3D_OK;
}

namespace {

// fd3d_create with the choice of creating the staging event (events = false: the
// context creates no HIP object, for the entry point that allocates nothing).
int create_ctx(fd3d_ctx **out, int nx, int ny, int nz, const void *lam, const void *mu, const void *rho, double dx,
               double dt, int nt, const fd3d_opts *opts, void *workspace, size_t ws_bytes, void *hip_stream,
               bool events)
{
    if (!out) return fail(FD3D_EINVAL, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    int rc = fd3d_workspace_bytes(nx, ny, nz, opts, &need);
    if (rc) return rc;
    if (opts && opts->vacuum_top >= nz) return fail(FD3D_EINVAL, "opts.vacuum_top must be < nz");
    if (opts && opts->vacuum_map) {
        std::vector<int> m((size_t)nx * ny);
        if (hipMemcpy(m.data(), opts->vacuum_map, m.size() * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
            return fail(FD3D_EINVAL, "opts.vacuum_map is not readable device memory");
        for (int v : m)
            if (v < 1 || v >= nz) return fail(FD3D_EINVAL, "opts.vacuum_map entries must lie in [1, nz - 1]");
    }
    if (!lam || !mu || !rho) return fail(FD3D_EINVAL, "model pointer is NULL");
    if (!(dx > 0.0) || !std::isfinite(dx)) return fail(FD3D_EINVAL, "dx must be > 0");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(FD3D_EINVAL, "dt must be > 0");
    if (nt < 0) return fail(FD3D_EINVAL, "nt must be >= 0");
    if (!workspace || ((uintptr_t)workspace % kAlign)) return fail(FD3D_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < need) return fail(FD3D_EWS, "workspace too small: need " + std::to_string(need) + " bytes");
    fd3d_ctx *c = new (std::nothrow) fd3d_ctx();
    if (!c) return fail(FD3D_EINVAL, "out of host memory");
    c->n[0] = nx; c->n[1] = ny; c->n[2] = nz;
    c->nt = nt;
    c->opts = opts ? *opts : default_opts();
    c->opts.max_receivers = max_rec_of(c->opts);
    c->tsize = c->opts.dtype == FD3D_F64 ? 8 : 4;
    c->dx = dx;
    c->dy = c->opts.dy > 0.0 ? c->opts.dy : dx;
    c->dz = c->opts.dz > 0.0 ? c->opts.dz : dx;
    c->dt = dt;
    c->lam = lam; c->mu = mu; c->rho = rho;
    c->ws = (char *)workspace;
    c->ws_bytes = ws_bytes;
    c->L = layout_of(nx, ny, nz, c->opts);
    c->staged_pending = false;
    c->rec_dev_valid = false;
    c->prof_on = 0;
    c->prof_used = 0;
    c->grad_ws = nullptr;
    c->grad_k = 0;
    c->grad_ready = 0;
    // default tile shape by row length (measured on MI355X at 256^3: 256x4 tiles with
    // 64-plane sweeps keep one 1024-thread workgroup per CU and 1 KiB row segments)
    c->variant = FD3D_KERNEL_TILE;
    c->cur = 0;
    if (c->tsize == 4 && nx >= 256) { c->tile_x = 256; c->tile_y = 4; }
    else if (nx >= 128) { c->tile_x = 128; c->tile_y = 4; }
    else { c->tile_x = 64; c->tile_y = 8; }
    c->zchunk = nz >= 128 ? 64 : 32;
    while (!window_ok(c, c->zchunk) && c->zchunk > 4) c->zchunk /= 2;
    if (!window_ok(c, c->zchunk)) c->variant = FD3D_KERNEL_CELL;  // planes too large for a tile sweep
    if (coarse_on(c->opts) && c->variant != FD3D_KERNEL_TILE) {
        delete c;
        return fail(FD3D_EINVAL, "planes too large for the tile kernels, which a coarse medium needs");
    }
    c->staged = nullptr;
    if (events && hipEventCreateWithFlags(&c->staged, hipEventDisableTiming) != hipSuccess) {
        delete c;
        return fail(FD3D_EHIP, "hipEventCreateWithFlags failed");
    }
    hipStream_t st = (hipStream_t)hip_stream;
    if (c->tsize == 8) {
        rc = model_check<double>(c, st);
        if (!rc) rc = upload_profiles<double>(c, st);
        if (!rc) zero_fields<double>(c, st);
        if (!rc) copy_model<double>(c, st);
    } else {
        rc = model_check<float>(c, st);
        if (!rc) rc = upload_profiles<float>(c, st);
        if (!rc) zero_fields<float>(c, st);
        if (!rc) copy_model<float>(c, st);
    }
    if (!rc && hipGetLastError() != hipSuccess) rc = fail(FD3D_EHIP, "launch failed in fd3d_create");
    if (!rc) rc = hipStreamSynchronize(st) == hipSuccess ? FD3D_OK : fail(FD3D_EHIP, "hipStreamSynchronize failed");
    if (rc) {
        if (c->staged) (void)hipEventDestroy(c->staged);
        delete c;
        return rc;
    }
    *out = c;
    return FD3D_OK;
}

} // namespace

int fd3d_create(fd3d_ctx **out, int nx, int ny, int nz, const void *lam, const void *mu, const void *rho, double dx,
                double dt, int nt, const fd3d_opts *opts, void *workspace, size_t ws_bytes, void *hip_stream)
{
    return create_ctx(out, nx, ny, nz, lam, mu, rho, dx, dt, nt, opts, workspace, ws_bytes, hip_stream, true);
}

int fd3d_forward(fd3d_ctx *ctx, const fd3d_source *src, int nrec, const double *rec_pos, void *traces, int flags,
                 void *hip_stream)
{
    if (!ctx) return fail(FD3D_EINVAL, "ctx is NULL");
    if (nrec < 0 || nrec > ctx->opts.max_receivers)
        return fail(FD3D_EINVAL, "nrec must be in [0, max_receivers = " + std::to_string(ctx->opts.max_receivers) + "]");
    if (nrec > 0 && (!rec_pos || (!traces && ctx->nt > 0))) return fail(FD3D_EINVAL, "rec_pos/traces is NULL");
    hipStream_t st = (hipStream_t)hip_stream;
    return ctx->tsize == 8 ? forward_impl<double>(ctx, src, nrec, rec_pos, traces, flags, st)
                           : forward_impl<float>(ctx, src, nrec, rec_pos, traces, flags, st);
}

int fd3d_get_state(fd3d_ctx *ctx, void *const fields[9], void *hip_stream)
{
    if (!ctx || !fields) return fail(FD3D_EINVAL, "ctx/fields is NULL");
    for (int f = 0; f < NFIELD; ++f)
        if (!fields[f]) return fail(FD3D_EINVAL, "field pointer is NULL");
    hipStream_t st = (hipStream_t)hip_stream;
    for (int f = 0; f < NFIELD; ++f) {
        const char *a = ctx->ws + ctx->L.field[ctx->cur][f];
        if (!ctx->L.rows)
            HIP_TRY(hipMemcpyAsync(fields[f], a, ctx->L.field_bytes, hipMemcpyDeviceToDevice, st));
        else if (ctx->tsize == 8)
            copy_field<double>(ctx, (double *)fields[f], false, (const double *)a, true, -1, st);
        else
            copy_field<float>(ctx, (float *)fields[f], false, (const float *)a, true, -1, st);
    }
    HIP_TRY(hipGetLastError());
    return FD3D_OK;
}

namespace {

// Device scratch of the entry point that allocates nothing (fd3d_forward_static): the
// whole forward workspace of one call lives here.  Each GPU the library runs on holds
// its own copy from module load until the process ends.  On the host the array's name
// only stands in for the symbol; kernels and copies get the per-device address that
// hipGetSymbolAddress returns (scratch_address), never the name itself.
static __device__ __align__(256) unsigned char scratch[FD3D_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];  // per device id; null until resolved on that device

// Address of this device's copy of the scratch, resolved once per device with the device
// current (the calling thread's current device).
int scratch_address(void **ptr)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(FD3D_EHIP, "device id out of range for the static scratch");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || ((uintptr_t)p % kAlign)) return fail(FD3D_EHIP, "hipGetSymbolAddress gave no aligned scratch address");
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return FD3D_OK;
}

} // namespace

int fd3d_forward_static(int nx, int ny, int nz, const void *lam, const void *mu, const void *rho, double dx,
                        double dt, int nt, const fd3d_opts *opts, const fd3d_source *src, int nrec,
                        const double *rec_pos, void *traces, void *const final_state[9], void *hip_stream)
{
    size_t need = 0;
    int rc = fd3d_workspace_bytes(nx, ny, nz, opts, &need);
    if (rc) return rc;
    if (need > FD3D_STATIC_SCRATCH_BYTES)
        return fail(FD3D_EWS, "grid " + std::to_string(nx) + "x" + std::to_string(ny) + "x" + std::to_string(nz) +
                                  " needs " + std::to_string(need) + " bytes of workspace; the static scratch holds " +
                                  std::to_string((size_t)FD3D_STATIC_SCRATCH_BYTES));
    if (final_state)
        for (int f = 0; f < NFIELD; ++f)
            if (!final_state[f]) return fail(FD3D_EINVAL, "final_state field pointer is NULL");
    void *ws = nullptr;
    rc = scratch_address(&ws);
    if (rc) return rc;
    fd3d_ctx *c = nullptr;
    rc = create_ctx(&c, nx, ny, nz, lam, mu, rho, dx, dt, nt, opts, ws, FD3D_STATIC_SCRATCH_BYTES, hip_stream, false);
    if (rc) return rc;
    rc = fd3d_forward(c, src, nrec, rec_pos, traces, 0, hip_stream);
    if (!rc && final_state) rc = fd3d_get_state(c, final_state, hip_stream);
    // the context's host staging buffers must outlive the uploads queued from them
    if (hipStreamSynchronize((hipStream_t)hip_stream) != hipSuccess && !rc)
        rc = fail(FD3D_EHIP, "hipStreamSynchronize failed");
    fd3d_destroy(c);
    return rc;
}

int fd3d_set_state(fd3d_ctx *ctx, const void *const fields[9], void *hip_stream)
{
    if (!ctx || !fields) return fail(FD3D_EINVAL, "ctx/fields is NULL");
    for (int f = 0; f < NFIELD; ++f)
        if (!fields[f]) return fail(FD3D_EINVAL, "field pointer is NULL");
    hipStream_t st = (hipStream_t)hip_stream;
    return ctx->tsize == 8 ? set_state_impl<double>(ctx, fields, st) : set_state_impl<float>(ctx, fields, st);
}

int fd3d_model_info(const fd3d_ctx *ctx, double out[4])
{
    if (!ctx || !out) return fail(FD3D_EINVAL, "ctx/out is NULL");
    for (int q = 0; q < 4; ++q) out[q] = ctx->info[q];
    return FD3D_OK;
}

int fd3d_get_layout(const fd3d_ctx *ctx, int *layout)
{
    if (!ctx || !layout) return fail(FD3D_EINVAL, "ctx/layout is NULL");
    *layout = ctx->L.rows ? FD3D_LAYOUT_ROWS : FD3D_LAYOUT_SEPARATE;
    return FD3D_OK;
}

int fd3d_grad_workspace_bytes(const fd3d_ctx *ctx, int ckpt_every, size_t *bytes)
{
    if (!ctx || !bytes) return fail(FD3D_EINVAL, "ctx/bytes is NULL");
    if (ctx->nt < 1) return fail(FD3D_EINVAL, "gradient needs nt >= 1");
    if (ckpt_every < 1 || ckpt_every > ctx->nt) return fail(FD3D_EINVAL, "ckpt_every must be in [1, nt]");
    *bytes = make_grad_layout(ctx, ckpt_every).total;
    return FD3D_OK;
}

int fd3d_forward_ckpt(fd3d_ctx *ctx, const fd3d_source *src, int nrec, const double *rec_pos, void *traces,
                      int flags, void *gws, size_t gws_bytes, int ckpt_every, void *hip_stream)
{
    if (!ctx) return fail(FD3D_EINVAL, "ctx is NULL");
    int rc = check_gws(ctx, gws, gws_bytes, ckpt_every);
    if (rc) return rc;
    if (nrec < 0 || nrec > ctx->opts.max_receivers) return fail(FD3D_EINVAL, "nrec out of range");
    if (nrec > 0 && (!rec_pos || !traces)) return fail(FD3D_EINVAL, "rec_pos/traces is NULL");
    const GradLayout GL = make_grad_layout(ctx, ckpt_every);
    hipStream_t st = (hipStream_t)hip_stream;
    ctx->grad_ready = 0;
    rc = ctx->tsize == 8 ? forward_impl<double>(ctx, src, nrec, rec_pos, traces, flags, st, (char *)gws, &GL)
                         : forward_impl<float>(ctx, src, nrec, rec_pos, traces, flags, st, (char *)gws, &GL);
    if (rc) return rc;
    ctx->grad_ws = (const char *)gws;
    ctx->grad_k = ckpt_every;
    ctx->grad_ready = 1;
    return FD3D_OK;
}

int fd3d_adjoint(fd3d_ctx *ctx, const fd3d_source *src, int nrec, const double *rec_pos, const void *residual,
                 void *g_lam, void *g_mu, void *g_rho, void *gws, size_t gws_bytes, void *hip_stream)
{
    if (!ctx) return fail(FD3D_EINVAL, "ctx is NULL");
    if (!ctx->grad_ready || gws != ctx->grad_ws)
        return fail(FD3D_ESTATE, "fd3d_adjoint needs fd3d_forward_ckpt on the same gradient workspace first");
    int rc = check_gws(ctx, gws, gws_bytes, ctx->grad_k);
    if (rc) return rc;
    if (nrec < 0 || nrec > ctx->opts.max_receivers) return fail(FD3D_EINVAL, "nrec out of range");
    if (nrec > 0 && (!rec_pos || !residual)) return fail(FD3D_EINVAL, "rec_pos/residual is NULL");
    if (!g_lam || !g_mu || !g_rho) return fail(FD3D_EINVAL, "gradient pointer is NULL");
    const GradLayout GL = make_grad_layout(ctx, ctx->grad_k);
    hipStream_t st = (hipStream_t)hip_stream;
    if (ctx->tsize == 8)
        return adjoint_impl<double>(ctx, src, nrec, rec_pos, (const double *)residual, (double *)g_lam,
                                    (double *)g_mu, (double *)g_rho, (char *)gws, GL, st);
    return adjoint_impl<float>(ctx, src, nrec, rec_pos, (const float *)residual, (float *)g_lam, (float *)g_mu,
                               (float *)g_rho, (char *)gws, GL, st);
}

extern "C++" {
template <typename T>
static int gradient_impl(fd3d_ctx *ctx, const fd3d_source *src, int nrec, const double *rec_pos, const void *d_obs,
                         void *traces, void *misfit, void *g_lam, void *g_mu, void *g_rho, void *gws,
                         size_t gws_bytes, int ckpt_every, hipStream_t st)
{
    int rc = fd3d_forward_ckpt(ctx, src, nrec, rec_pos, traces, 0, gws, gws_bytes, ckpt_every, st);
    if (rc) return rc;
    const GradLayout GL = make_grad_layout(ctx, ckpt_every);
    T *res = (T *)((char *)gws + GL.res);
    const long n = (long)nrec * 3 * ctx->nt;
    double *part = (double *)(ctx->ws + ctx->L.part);
    residual_misfit<T><<<kReduceBlocks, 256, 0, st>>>((const T *)traces, (const T *)d_obs, res, n, part);
    misfit_final<T><<<1, 64, 0, st>>>(part, kReduceBlocks, misfit ? (T *)misfit : (T *)((char *)gws + GL.misfit));
    HIP_TRY(hipGetLastError());
    return fd3d_adjoint(ctx, src, nrec, rec_pos, res, g_lam, g_mu, g_rho, gws, gws_bytes, st);
}

} // extern "C++"

int fd3d_born(fd3d_ctx *ctx, fd3d_ctx *dctx, const fd3d_source *src, const void *dlam, const void *dmu,
              const void *drho, int nrec, const double *rec_pos, void *traces, void *dtraces, void *hip_stream)
{
    if (!ctx || !dctx) return fail(FD3D_EINVAL, "ctx/dctx is NULL");
    if (ctx == dctx) return fail(FD3D_EINVAL, "the perturbation needs a context of its own");
    if (!dlam || !dmu || !drho) return fail(FD3D_EINVAL, "model perturbation pointer is NULL");
    if (nrec < 0 || nrec > ctx->opts.max_receivers || nrec > dctx->opts.max_receivers)
        return fail(FD3D_EINVAL, "nrec out of range");
    if (nrec > 0 && (!rec_pos || !dtraces)) return fail(FD3D_EINVAL, "rec_pos/dtraces is NULL");
    for (int a = 0; a < 3; ++a)
        if (ctx->n[a] != dctx->n[a]) return fail(FD3D_EINVAL, "contexts differ in grid size");
    if (ctx->tsize != dctx->tsize || ctx->nt != dctx->nt || ctx->dt != dctx->dt || ctx->dx != dctx->dx ||
        ctx->dy != dctx->dy || ctx->dz != dctx->dz)
        return fail(FD3D_EINVAL, "contexts differ in dtype, nt, dt or spacing");
    if (ctx->lam != dctx->lam || ctx->mu != dctx->mu || ctx->rho != dctx->rho)
        return fail(FD3D_EINVAL, "contexts must share the model arrays");
    if (ctx->L.rows != dctx->L.rows) return fail(FD3D_EINVAL, "contexts differ in field layout");
    for (int f = 0; f < 6; ++f)
        if (ctx->opts.sponge[f] != dctx->opts.sponge[f]) return fail(FD3D_EINVAL, "contexts differ in damping");
    if (ctx->opts.sponge_alpha != dctx->opts.sponge_alpha) return fail(FD3D_EINVAL, "contexts differ in damping");
    if (ctx->opts.free_surface || dctx->opts.free_surface || ctx->opts.vacuum_top || dctx->opts.vacuum_top)
        return fail(FD3D_EINVAL, "the Born forward supports damped boundaries only (no free surface)");
    if (coarse_on(ctx->opts) || coarse_on(dctx->opts))
        return fail(FD3D_EINVAL, "the Born forward needs the medium at the simulation nodes");
    if (ctx->variant == FD3D_KERNEL_FUSED || dctx->variant == FD3D_KERNEL_FUSED)
        return fail(FD3D_EINVAL, "the Born forward runs the tile or cell kernels (set one with fd3d_set_kernel)");
    hipStream_t st = (hipStream_t)hip_stream;
    return ctx->tsize == 8 ? born_impl<double>(ctx, dctx, src, dlam, dmu, drho, nrec, rec_pos, traces, dtraces, st)
                           : born_impl<float>(ctx, dctx, src, dlam, dmu, drho, nrec, rec_pos, traces, dtraces, st);
}

int fd3d_gradient(fd3d_ctx *ctx, const fd3d_source *src, int nrec, const double *rec_pos, const void *d_obs,
                  void *traces, void *misfit, void *g_lam, void *g_mu, void *g_rho, void *gws, size_t gws_bytes,
                  int ckpt_every, void *hip_stream)
{
    if (!ctx) return fail(FD3D_EINVAL, "ctx is NULL");
    if (nrec < 1 || !d_obs || !traces) return fail(FD3D_EINVAL, "fd3d_gradient needs receivers, d_obs and traces");
    hipStream_t st = (hipStream_t)hip_stream;
    return ctx->tsize == 8 ? gradient_impl<double>(ctx, src, nrec, rec_pos, d_obs, traces, misfit, g_lam, g_mu, g_rho,
                                                   gws, gws_bytes, ckpt_every, st)
                           : gradient_impl<float>(ctx, src, nrec, rec_pos, d_obs, traces, misfit, g_lam, g_mu, g_rho,
                                                  gws, gws_bytes, ckpt_every, st);
}

int fd3d_get_adjoint_state(fd3d_ctx *ctx, const void *gws, void *const fields[9], void *hip_stream)
{
    if (!ctx || !gws || !fields) return fail(FD3D_EINVAL, "ctx/gws/fields is NULL");
    if (!ctx->grad_ready || gws != ctx->grad_ws) return fail(FD3D_ESTATE, "no adjoint state in this workspace");
    for (int f = 0; f < NFIELD; ++f)
        if (!fields[f]) return fail(FD3D_EINVAL, "field pointer is NULL");
    const GradLayout GL = make_grad_layout(ctx, ctx->grad_k);
    hipStream_t st = (hipStream_t)hip_stream;
    const dim3 blk(64, 4, 1), grd((ctx->n[0] + 63) / 64, (ctx->n[1] + 3) / 4, ctx->n[2]);
    for (int f = 0; f < NFIELD; ++f) {
        const char *a = (const char *)gws + GL.adj + f * GL.fstep;
        if (f <= VZ) {
            if (ctx->tsize == 8)
                scale_velocity<double><<<grd, blk, 0, st>>>(make_grid<double>(ctx), (const double *)a, f, (double *)fields[f]);
            else
                scale_velocity<float><<<grd, blk, 0, st>>>(make_grid<float>(ctx), (const float *)a, f, (float *)fields[f]);
        } else if (!ctx->L.rows) {
            HIP_TRY(hipMemcpyAsync(fields[f], a, ctx->L.field_bytes, hipMemcpyDeviceToDevice, st));
        } else if (ctx->tsize == 8) {
            copy_field<double>(ctx, (double *)fields[f], false, (const double *)a, true, -1, st);
        } else {
            copy_field<float>(ctx, (float *)fields[f], false, (const float *)a, true, -1, st);
        }
    }
    HIP_TRY(hipGetLastError());
    return FD3D_OK;
}

int fd3d_set_kernel(fd3d_ctx *ctx, const fd3d_kernel *k)
{
    if (!ctx || !k) return fail(FD3D_EINVAL, "ctx/k is NULL");
    if (k->variant != FD3D_KERNEL_CELL && k->variant != FD3D_KERNEL_TILE && k->variant != FD3D_KERNEL_FUSED)
        return fail(FD3D_EINVAL, "unknown kernel variant");
    if (k->variant == FD3D_KERNEL_TILE && !tile_supported(ctx->tsize, k->tile_x, k->tile_y))
        return fail(FD3D_EINVAL, "unsupported tile shape " + std::to_string(k->tile_x) + "x" + std::to_string(k->tile_y));
    if (k->variant == FD3D_KERNEL_FUSED && !fused_supported(ctx, k->tile_x, k->tile_y))
        return fail(FD3D_EINVAL, "unsupported fused tile shape " + std::to_string(k->tile_x) + "x" +
                                     std::to_string(k->tile_y));
    if (k->zchunk < 4) return fail(FD3D_EINVAL, "zchunk must be >= 4");
    if (coarse_on(ctx->opts) && k->variant != FD3D_KERNEL_TILE)
        return fail(FD3D_EINVAL, "a coarse medium runs on the tile kernels only");
    if (k->variant != FD3D_KERNEL_CELL && !window_ok(ctx, k->zchunk))
        return fail(FD3D_EINVAL, "zchunk too large: (zchunk + 8) planes must fit in 1 GiB");
    ctx->variant = k->variant;
    if (k->variant != FD3D_KERNEL_CELL) {
        ctx->tile_x = k->tile_x;
        ctx->tile_y = k->tile_y;
    }
    ctx->zchunk = k->zchunk;
    return FD3D_OK;
}

int fd3d_get_kernel(const fd3d_ctx *ctx, fd3d_kernel *k)
{
    if (!ctx || !k) return fail(FD3D_EINVAL, "ctx/k is NULL");
    k->variant = ctx->variant;
    k->tile_x = ctx->tile_x;
    k->tile_y = ctx->tile_y;
    k->zchunk = ctx->zchunk;
    return FD3D_OK;
}

int fd3d_batch_workspace_bytes(int nshot, fd3d_ctx *const *ctxs, size_t *bytes)
{
    if (nshot < 1 || nshot > kMaxShots || !ctxs || !bytes)
        return fail(FD3D_EINVAL, "nshot must be in [1, " + std::to_string(kMaxShots) + "]");
    if (!ctxs[0]) return fail(FD3D_EINVAL, "context 0 is NULL");
    *bytes = batch_desc_bytes(nshot, ctxs[0]->tsize);
    return FD3D_OK;
}

int fd3d_batch_create(fd3d_batch **out, int nshot, fd3d_ctx *const *ctxs, void *workspace, size_t ws_bytes)
{
    if (!out) return fail(FD3D_EINVAL, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    int rc = fd3d_batch_workspace_bytes(nshot, ctxs, &need);
    if (rc) return rc;
    for (int s = 0; s < nshot; ++s) {
        if (!ctxs[s]) return fail(FD3D_EINVAL, "context " + std::to_string(s) + " is NULL");
        if (ctxs[s]->tsize != ctxs[0]->tsize) return fail(FD3D_EINVAL, "all shots must share one dtype");
        if (ctxs[s]->nt != ctxs[0]->nt) return fail(FD3D_EINVAL, "all shots must share nt");
        if (ctxs[s]->opts.free_surface != ctxs[0]->opts.free_surface)
            return fail(FD3D_EINVAL, "all shots must share the free-surface option");
        if (coarse_on(ctxs[s]->opts))
            return fail(FD3D_EINVAL, "context " + std::to_string(s) + ": a batch needs media at the simulation nodes");
        if (!window_ok(ctxs[s], ctxs[s]->zchunk))
            return fail(FD3D_EINVAL, "context " + std::to_string(s) + ": zchunk too large for a tile sweep");
        for (int q = 0; q < s; ++q)
            if (ctxs[q] == ctxs[s]) return fail(FD3D_EINVAL, "a context appears twice in the batch");
    }
    if (!workspace || ((uintptr_t)workspace % kAlign)) return fail(FD3D_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < need) return fail(FD3D_EWS, "batch workspace too small: need " + std::to_string(need) + " bytes");
    fd3d_batch *b = new (std::nothrow) fd3d_batch();
    if (!b) return fail(FD3D_EINVAL, "out of host memory");
    b->nshot = nshot;
    b->ctx.assign(ctxs, ctxs + nshot);
    b->tsize = ctxs[0]->tsize;
    b->nt = ctxs[0]->nt;
    b->fs = ctxs[0]->opts.free_surface;
    b->ws = (char *)workspace;
    b->ws_bytes = ws_bytes;
    b->off_fwd = 0;
    b->off_rec = round_up((size_t)nshot * (b->tsize == 8 ? sizeof(ShotFwd<double>) : sizeof(ShotFwd<float>)), kAlign);
    // tile shape of the batch: the widest default among the shots that every shot supports
    int minx = ctxs[0]->n[0];
    for (int s = 1; s < nshot; ++s) minx = std::min(minx, ctxs[s]->n[0]);
    if (b->tsize == 4 && minx >= 256) { b->tile_x = 256; b->tile_y = 4; }
    else if (minx >= 128) { b->tile_x = 128; b->tile_y = 4; }
    else { b->tile_x = 64; b->tile_y = 8; }
    b->wgs_req = 0;
    b->tile2_x = b->tile2_y = 0;
    b->staged_pending = false;
    b->graph_valid = false;
    b->graph_key = 0;
    b->group_bytes = 0;
    if (hipEventCreateWithFlags(&b->staged, hipEventDisableTiming) != hipSuccess) {
        delete b;
        return fail(FD3D_EHIP, "hipEventCreateWithFlags failed");
    }
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
        (void)hipEventDestroy(b->staged);
        delete b;
        return fail(FD3D_EHIP, "hipStreamCreateWithFlags failed");
    }
    *out = b;
    return FD3D_OK;
}

int fd3d_batch_set_kernel(fd3d_batch *b, int tile_x, int tile_y, int workgroups)
{
    return fd3d_batch_set_tiles(b, tile_x, tile_y, 0, 0, workgroups);
}

int fd3d_batch_set_tiles(fd3d_batch *b, int tile_x, int tile_y, int tile2_x, int tile2_y, int workgroups)
{
    if (!b) return fail(FD3D_EINVAL, "batch is NULL");
    if (!tile_supported(b->tsize, tile_x, tile_y))
        return fail(FD3D_EINVAL, "unsupported tile shape " + std::to_string(tile_x) + "x" + std::to_string(tile_y));
    if ((tile2_x || tile2_y) && !pair_supported(b->tsize, tile_x, tile_y, tile2_x, tile2_y))
        return fail(FD3D_EINVAL, "unsupported pair of tile shapes");
    if (workgroups < 0) return fail(FD3D_EINVAL, "workgroups must be >= 0");
    b->tile_x = tile_x;
    b->tile_y = tile_y;
    b->tile2_x = tile2_x;
    b->tile2_y = tile2_y;
    b->wgs_req = workgroups;
    return FD3D_OK;
}

int fd3d_batch_set_schedule(fd3d_batch *b, size_t group_bytes)
{
    if (!b) return fail(FD3D_EINVAL, "batch is NULL");
    b->group_bytes = group_bytes;
    return FD3D_OK;
}

int fd3d_batch_autotune(fd3d_batch *b, int steps, int best[6], double *best_ms, void *hip_stream)
{
    if (!b) return fail(FD3D_EINVAL, "batch is NULL");
    if (steps < 1) return fail(FD3D_EINVAL, "steps must be >= 1");
    hipStream_t st = (hipStream_t)hip_stream;
    // single shapes, then pairs (primary, second)
    static const int shapes[][4] = {{64, 4, 0, 0},    {64, 8, 0, 0},   {64, 16, 0, 0},   {128, 4, 0, 0},
                                    {128, 8, 0, 0},   {256, 4, 0, 0},  {256, 4, 64, 16}, {128, 8, 64, 16},
                                    {256, 4, 128, 8}, {128, 4, 64, 8}};
    // cache-blocked group budgets tried after the shapes (MiB; 0: lockstep)
    static const int budgets[] = {96, 128, 192, 256, 384};
    const int nt_save = b->nt;
    const size_t keep_group = b->group_bytes;
    const int keep[5] = {b->tile_x, b->tile_y, b->tile2_x, b->tile2_y, b->wgs_req};
    int win[5] = {keep[0], keep[1], keep[2], keep[3], keep[4]};
    int win_mib = 0;
    double win_ms = 1e300;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(FD3D_EHIP, "hipEventCreate failed");
    b->nt = steps;
    b->group_bytes = 0;
    int rc = FD3D_OK;
    // times `steps` steps of the current settings (after one untimed run)
    auto time_it = [&](float &ms) {
        for (int rep = 0; rep < 2 && !rc; ++rep) {
            if (rep == 1 && hipEventRecord(e0, st) != hipSuccess) rc = fail(FD3D_EHIP, "hipEventRecord");
            if (!rc)
                rc = b->tsize == 8 ? batch_forward_impl<double>(b, nullptr, nullptr, nullptr, nullptr, FD3D_KEEP_STATE, 0, st)
                                   : batch_forward_impl<float>(b, nullptr, nullptr, nullptr, nullptr, FD3D_KEEP_STATE, 0, st);
        }
        if (rc) return;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            rc = fail(FD3D_EHIP, "timing events failed");
            return;
        }
        ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
    };
    for (const auto &sh : shapes) {
        if (!tile_supported(b->tsize, sh[0], sh[1])) continue;
        if (sh[2] && !pair_supported(b->tsize, sh[0], sh[1], sh[2], sh[3])) continue;
        // persistent grid (CUs x occupancy) or one workgroup per tile
        for (int mode = 0; mode < 2 && !rc; ++mode) {
            b->tile_x = sh[0];
            b->tile_y = sh[1];
            b->tile2_x = sh[2];
            b->tile2_y = sh[3];
            b->wgs_req = 0;
            if (mode == 1) {
                long tiles = 0;
                const BatchGroup all = whole_batch(b);
                for (const fd3d_ctx *c : b->ctx) {
                    int alt = 0;
                    const TileMap tm = shot_tiles(all, c, alt);
                    tiles += (long)tm.ntx * tm.nty * tm.nzc;
                }
                b->wgs_req = (int)std::min<long>((tiles + 7) / 8 * 8, 1L << 30);
            }
            float ms = 0.0f;
            time_it(ms);
            if (rc) break;
            if (ms < win_ms) {
                win_ms = ms;
                win[0] = b->tile_x;
                win[1] = b->tile_y;
                win[2] = b->tile2_x;
                win[3] = b->tile2_y;
                win[4] = b->wgs_req;
            }
        }
        if (rc) break;
    }
    // the schedule, with the winning shapes for the launches that use the batch's shapes
    if (!rc) {
        b->tile_x = win[0];
        b->tile_y = win[1];
        b->tile2_x = win[2];
        b->tile2_y = win[3];
        b->wgs_req = win[4];
        for (int mib : budgets) {
            b->group_bytes = (size_t)mib << 20;
            float ms = 0.0f;
            time_it(ms);
            if (rc) break;
            if (ms < win_ms) {
                win_ms = ms;
                win_mib = mib;
            }
        }
    }
    b->nt = nt_save;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const int *use = rc ? keep : win;
    b->tile_x = use[0];
    b->tile_y = use[1];
    b->tile2_x = use[2];
    b->tile2_y = use[3];
    b->wgs_req = use[4];
    b->group_bytes = rc ? keep_group : (size_t)win_mib << 20;
    if (rc) return rc;
    for (fd3d_ctx *c : b->ctx) zero_fields_any(c, st);
    if (best) {
        for (int q = 0; q < 5; ++q) best[q] = win[q];
        best[5] = win_mib;
    }
    if (best_ms) *best_ms = win_ms / steps;
    return FD3D_OK;
}

int fd3d_batch_forward(fd3d_batch *b, const fd3d_source *srcs, const int *nrec, const double *const *rec_pos,
                       void *const *traces, int flags, int use_graph, void *hip_stream)
{
    if (!b) return fail(FD3D_EINVAL, "batch is NULL");
    hipStream_t st = (hipStream_t)hip_stream;
    return b->tsize == 8 ? batch_forward_impl<double>(b, srcs, nrec, rec_pos, traces, flags, use_graph, st)
                         : batch_forward_impl<float>(b, srcs, nrec, rec_pos, traces, flags, use_graph, st);
}

int fd3d_batch_grad_workspace_bytes(const fd3d_batch *b, int ckpt_every, size_t *bytes)
{
    if (!b || !bytes) return fail(FD3D_EINVAL, "batch/bytes is NULL");
    if (ckpt_every < 1 || ckpt_every > b->nt) return fail(FD3D_EINVAL, "ckpt_every must be in [1, nt]");
    *bytes = b->tsize == 8 ? make_batch_grad_layout<double>(b, ckpt_every).total
                           : make_batch_grad_layout<float>(b, ckpt_every).total;
    return FD3D_OK;
}

int fd3d_batch_gradient(fd3d_batch *b, const fd3d_source *srcs, const int *nrec, const double *const *rec_pos,
                        const void *const *d_obs, void *const *traces, void *const *misfit, void *const *g_lam,
                        void *const *g_mu, void *const *g_rho, void *const *gws, const size_t *gws_bytes,
                        int ckpt_every, int flags, void *bws, size_t bws_bytes, void *hip_stream)
{
    if (!b || !gws_bytes) return fail(FD3D_EINVAL, "batch/gws_bytes is NULL");
    if (b->fs) return fail(FD3D_EINVAL, "the gradient supports damped boundaries only (no free surface)");
    if (ckpt_every < 1 || ckpt_every > b->nt) return fail(FD3D_EINVAL, "ckpt_every must be in [1, nt]");
    hipStream_t st = (hipStream_t)hip_stream;
    return b->tsize == 8
               ? batch_gradient_impl<double>(b, srcs, nrec, rec_pos, d_obs, traces, misfit, g_lam, g_mu, g_rho, gws,
                                             gws_bytes, ckpt_every, flags, (char *)bws, bws_bytes, st)
               : batch_gradient_impl<float>(b, srcs, nrec, rec_pos, d_obs, traces, misfit, g_lam, g_mu, g_rho, gws,
                                            gws_bytes, ckpt_every, flags, (char *)bws, bws_bytes, st);
}

void fd3d_batch_destroy(fd3d_batch *b)
{
    if (!b) return;
    if (b->staged_pending) (void)hipEventSynchronize(b->staged);
    if (b->graph_valid) {
        (void)hipGraphExecDestroy(b->gexec);
        (void)hipGraphDestroy(b->graph);
    }
    (void)hipStreamDestroy(b->cap);
    (void)hipEventDestroy(b->staged);
    delete b;
}

int fd3d_autotune(fd3d_ctx *ctx, int steps, fd3d_kernel *best, double *best_ms, void *hip_stream)
{
    if (!ctx) return fail(FD3D_EINVAL, "ctx is NULL");
    if (steps < 1) return fail(FD3D_EINVAL, "steps must be >= 1");
    hipStream_t st = (hipStream_t)hip_stream;
    // the one-thread-per-cell kernel (no z sweep) can win on small grids, where a sweep's
    // planes cost a memory round trip each
    static const int shapes[][3] = {{FD3D_KERNEL_CELL, 64, 4},   {FD3D_KERNEL_TILE, 64, 4},   {FD3D_KERNEL_TILE, 64, 8},
                                    {FD3D_KERNEL_TILE, 64, 16},  {FD3D_KERNEL_TILE, 128, 4},  {FD3D_KERNEL_TILE, 128, 8},
                                    {FD3D_KERNEL_TILE, 256, 4},  {FD3D_KERNEL_FUSED, 64, 4},  {FD3D_KERNEL_FUSED, 64, 8}};
    // z chunks: powers of two, and the depths that cut the grid into m equal sweeps
    // (m = 1 .. 8), so that the workgroup count can match whole rounds of the CUs (on a
    // 512 x 512 x 256 grid, 256 x 4 tiles sweeping all 256 planes are one workgroup per CU)
    std::vector<int> chunks = {4, 8, 16, 32, 64, 128};
    for (int m = 1; m <= 8; ++m) {
        const int zc = (ctx->n[2] + m - 1) / m;
        if (zc >= 4 && std::find(chunks.begin(), chunks.end(), zc) == chunks.end()) chunks.push_back(zc);
    }
    std::sort(chunks.begin(), chunks.end());
    const int nt_save = ctx->nt;
    const fd3d_kernel keep = {ctx->variant, ctx->tile_x, ctx->tile_y, ctx->zchunk};
    fd3d_kernel win = keep;
    double win_ms = 1e300;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(FD3D_EHIP, "hipEventCreate failed");
    ctx->nt = steps;
    int rc = FD3D_OK;
    for (const auto &sh : shapes) {
        if (sh[0] == FD3D_KERNEL_TILE && !tile_supported(ctx->tsize, sh[1], sh[2])) continue;
        if (coarse_on(ctx->opts) && sh[0] != FD3D_KERNEL_TILE) continue;
        if (sh[0] == FD3D_KERNEL_FUSED && !fused_supported(ctx, sh[1], sh[2])) continue;
        if (sh[1] > 64 && ctx->n[0] < sh[1] / 2) continue;  // mostly idle lanes
        for (int zc : chunks) {
            if (sh[0] == FD3D_KERNEL_CELL && zc != chunks[0]) break;  // no z chunks
            if (sh[0] == FD3D_KERNEL_FUSED && zc < 8) continue;
            if (zc > ctx->n[2] && zc != chunks[0]) continue;
            if (!window_ok(ctx, zc)) continue;
            ctx->variant = sh[0];
            ctx->tile_x = sh[1];
            ctx->tile_y = sh[2];
            ctx->zchunk = zc;
            // one warm-up run and two timed runs (the faster counts), all from the current
            // (clobbered) state
            float ms = 3.0e38f;
            for (int rep = 0; rep < 3 && !rc; ++rep) {
                if (rep >= 1 && hipEventRecord(e0, st) != hipSuccess) rc = fail(FD3D_EHIP, "hipEventRecord");
                if (!rc) rc = ctx->tsize == 8 ? forward_impl<double>(ctx, nullptr, 0, nullptr, nullptr, FD3D_KEEP_STATE, st)
                                             : forward_impl<float>(ctx, nullptr, 0, nullptr, nullptr, FD3D_KEEP_STATE, st);
                if (!rc && rep >= 1) {
                    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                        rc = fail(FD3D_EHIP, "timing events failed");
                        break;
                    }
                    float t = 0.0f;
                    (void)hipEventElapsedTime(&t, e0, e1);
                    ms = std::min(ms, t);
                }
            }
            if (rc) break;
            if (ms < win_ms) {
                win_ms = ms;
                win = fd3d_kernel{sh[0], sh[1], sh[2], zc};
            }
        }
        if (rc) break;
    }
    ctx->nt = nt_save;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const fd3d_kernel &use = rc ? keep : win;
    ctx->variant = use.variant;
    ctx->tile_x = use.tile_x;
    ctx->tile_y = use.tile_y;
    ctx->zchunk = use.zchunk;
    if (rc) return rc;
    zero_fields_any(ctx, st);
    if (best) *best = win;
    if (best_ms) *best_ms = win_ms / steps;
    return FD3D_OK;
}

int fd3d_profile(fd3d_ctx *ctx, int enable)
{
    if (!ctx) return fail(FD3D_EINVAL, "ctx is NULL");
    ctx->prof_on = enable ? 1 : 0;
    return FD3D_OK;
}

int fd3d_upsample(const void *coarse, int mx, int my, int mz, void *fine, int nx, int ny, int nz, int dtype,
                  void *hip_stream)
{
    if (!coarse || !fine) return fail(FD3D_EINVAL, "coarse/fine is NULL");
    if (mx < 1 || my < 1 || mz < 1 || nx < 1 || ny < 1 || nz < 1)
        return fail(FD3D_EINVAL, "grid sizes must be >= 1");
    if (dtype != FD3D_F32 && dtype != FD3D_F64) return fail(FD3D_EINVAL, "dtype must be FD3D_F32 or FD3D_F64");
    const double nf = (double)nx * ny * nz, nc = (double)mx * my * mz;
    if (nf >= 9.2e18 || nc >= 9.2e18) return fail(FD3D_EINVAL, "grid too large");
    const int ts = dtype == FD3D_F64 ? 8 : 4;
    const char *c0 = (const char *)coarse, *c1 = c0 + (size_t)nc * ts;
    const char *f0 = (const char *)fine, *f1 = f0 + (size_t)nf * ts;
    if (c0 < f1 && f0 < c1) return fail(FD3D_EINVAL, "coarse and fine overlap");
    hipStream_t st = (hipStream_t)hip_stream;
    const int blocks = (int)std::min<double>(8192.0, std::ceil(nf / 256.0));
    if (dtype == FD3D_F64)
        upsample_trilinear<double><<<blocks, 256, 0, st>>>((const double *)coarse, mx, my, mz, (double *)fine, nx, ny, nz);
    else
        upsample_trilinear<float><<<blocks, 256, 0, st>>>((const float *)coarse, mx, my, mz, (float *)fine, nx, ny, nz);
    HIP_TRY(hipGetLastError());
    return FD3D_OK;
}

int fd3d_profile_read(fd3d_ctx *ctx, double ms[4], int launches[4])
{
    if (!ctx || !ms || !launches) return fail(FD3D_EINVAL, "ctx/ms/launches is NULL");
    for (int p = 0; p < 4; ++p) { ms[p] = 0.0; launches[p] = 0; }
    if (ctx->prof_used == 0) return FD3D_OK;
    HIP_TRY(hipEventSynchronize(ctx->prof_ev[2 * ctx->prof_used - 1]));
    for (int q = 0; q < ctx->prof_used; ++q) {
        float t = 0.0f;
        HIP_TRY(hipEventElapsedTime(&t, ctx->prof_ev[2 * q], ctx->prof_ev[2 * q + 1]));
        const int p = ctx->prof_pass[q];
        if (p >= 0 && p < 4) { ms[p] += t; launches[p] += 1; }
    }
    return FD3D_OK;
}

void fd3d_destroy(fd3d_ctx *ctx)
{
    if (!ctx) return;
    if (ctx->staged_pending) (void)hipEventSynchronize(ctx->staged);
    if (ctx->staged) (void)hipEventDestroy(ctx->staged);
    for (hipEvent_t e : ctx->prof_ev) {
        (void)hipEventSynchronize(e);
        (void)hipEventDestroy(e);
    }
    delete ctx;
}

} // extern "C"
