// The forward step loop (Sec. 2.2 update order: velocity pass, receiver sampling, stress
// pass) on the caller's stream, the kernel variants it can run (cell, tile, fused) and
// the tuner that picks one.
#include "host.h"

#include "fwd_fused.h"

using namespace fd3d;

namespace {

// rec: receiver sampling carried by a forward stress launch (extra workgroups).
// NTP: cache policy of the model loads and the gradient's stored data (see stream_model).
template <typename T, int TX, int TY, bool FS, bool NTP>
void launch_tiles(const Grid<T> &G, const Inject<T> &inj, int n, const TileMap &tm, int pass, hipStream_t st,
                  const RecJob<T> &rec)
{
    const int nwg = tm.ntx * tm.nty * tm.nzc;
    constexpr int NT = TX * TY;
    const int nws = nwg + rec_blocks(rec, NT);
    if (G.save[VX] != nullptr && pass == kPassVel) pass = kPassVelSave;
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
    case kPassVelSave: vel_tile<T, TX, TY, FS, kFwdSave, false, NTP><<<nwg, NT, 0, st>>>(G, inj, n, tm); break;
    default: stress_tile<T, TX, TY, FS, kFwd, false, NTP><<<nws, NT, 0, st>>>(G, inj, n, tm, rec); break;
    }
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

} // namespace

namespace fd3d {

template <typename T, bool FS>
void launch_pass(const fd3d_ctx *c, const Grid<T> &G, const Inject<T> &inj, int n, int pass, hipStream_t st,
                 const TileIO<T> &, const RecJob<T> &rec)
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
            launch_tiles<T, TX, TY, FS, sizeof(T) == 4>(G, inj, n, tm, pass, st, rec);
        else
            launch_tiles<T, TX, TY, FS, false>(G, inj, n, tm, pass, st, rec);
    });
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

template <typename T>
int forward_impl(fd3d_ctx *c, const fd3d_source *src, int nrec, const double *rec_pos, void *traces, int flags,
                 hipStream_t st, char *gws, const GradLayout *GL)
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

#define FD3D_FORWARD_INSTANCES(T, FS)                                                                        \
    template void launch_pass<T, FS>(const fd3d_ctx *, const Grid<T> &, const Inject<T> &, int, int, hipStream_t, \
                                     const TileIO<T> &, const RecJob<T> &);                                  \
    template void step<T, FS>(fd3d_ctx *, const Grid<T> &, const Inject<T> &, int, int, const RecTap<T> *, T *,  \
                              hipStream_t, Timer &);
FD3D_FORWARD_INSTANCES(float, false)
FD3D_FORWARD_INSTANCES(float, true)
FD3D_FORWARD_INSTANCES(double, false)
FD3D_FORWARD_INSTANCES(double, true)
#undef FD3D_FORWARD_INSTANCES
template int forward_impl<float>(fd3d_ctx *, const fd3d_source *, int, const double *, void *, int, hipStream_t,
                                 char *, const GradLayout *);
template int forward_impl<double>(fd3d_ctx *, const fd3d_source *, int, const double *, void *, int, hipStream_t,
                                  char *, const GradLayout *);

} // namespace fd3d

extern "C" {

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
        return fail(FD3D_EINVAL, "zchunk too large: a sweep's window (zchunk + 8 planes, at most nz) must fit in 1 GiB");
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
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        return fail(FD3D_EHIP, "hipEventCreate failed");
    }
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

} // extern "C"
