// Contexts (Sec. 2.2): options, workspace layout, the model check and stability bound,
// Cerjan damping profiles, source and receiver staging (Sec. 2.3, 2.4), state access,
// and the forward entry point that allocates nothing.
#include "host.h"

#include <mutex>
#include <new>
#include <unordered_set>

using namespace fd3d;

namespace fd3d {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

} // namespace fd3d

namespace {

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

} // namespace

namespace fd3d {

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

Layout layout_of(int nx, int ny, int nz, const fd3d_opts &o)
{
    const int tsize = o.dtype == FD3D_F64 ? 8 : 4;
    const bool rows = rows_layout(nx, ny, nz, tsize, o);
    return make_layout(nx, ny, nz, tsize, max_rec_of(o), rows, rows && !coarse_on(o));
}

} // namespace fd3d

namespace {


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

template <typename T> int set_state_impl(fd3d_ctx *c, const void *const fields[9], hipStream_t st)
{
    const Grid<T> G = make_grid<T>(c);
    for (int f = 0; f < NFIELD; ++f) copy_field<T>(c, G.f[f], true, (const T *)fields[f], false, f, st);
    HIP_TRY(hipGetLastError());
    return FD3D_OK;
}

} // namespace

namespace fd3d {

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

template int stage_inputs<float>(fd3d_ctx *, const fd3d_source *, Inject<float> &, int, const double *, hipStream_t);
template int stage_inputs<double>(fd3d_ctx *, const fd3d_source *, Inject<double> &, int, const double *, hipStream_t);

void zero_fields_any(fd3d_ctx *c, hipStream_t st)
{
    if (c->tsize == 8) zero_fields<double>(c, st);
    else zero_fields<float>(c, st);
}

} // namespace fd3d

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
    c->adj_done = 0;
    c->grad_y = 0;
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
        // uploads queued from the context's host buffers before the failure finish first
        (void)hipStreamSynchronize(st);
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
