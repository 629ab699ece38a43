// FWI gradient by the discrete adjoint (the exact transpose of the forward steps) with
// snapshot checkpointing: the checkpointed forward, the reverse sweep over the segments
// (recompute, then the adjoint passes of each step backwards) and the misfit.
#include "host.h"

using namespace fd3d;

namespace {

// One adjoint pass of a tiled step (stress-A, stress-M, velocity-A, stress-B) on the
// context's tile shape and cache policy (the streaming policy also covers the stored
// velocities).
template <typename T>
void launch_adj_pass(const fd3d_ctx *c, const Grid<T> &G, const Inject<T> &inj, int n, int pass, hipStream_t st,
                     const TileIO<T> &io)
{
    const TileMap tm = tile_map(c);
    const int nwg = tm.ntx * tm.nty * tm.nzc;
    with_tile<T>(c->tile_x, c->tile_y, [&](auto tx, auto ty) {
        constexpr int TX = decltype(tx)::value, TY = decltype(ty)::value, NT = TX * TY;
        constexpr bool F32 = sizeof(T) == 4;
        const bool ntp = F32 && stream_model(c);
        switch (pass) {
        case kPassStressA:
            if (ntp) stress_tile_adj<T, TX, TY, kAdjA, F32><<<nwg, NT, 0, st>>>(G, inj, tm, io);
            else stress_tile_adj<T, TX, TY, kAdjA, false><<<nwg, NT, 0, st>>>(G, inj, tm, io);
            break;
        case kPassStressM:
            if (ntp) stress_tile_adj<T, TX, TY, kAdjM, F32><<<nwg, NT, 0, st>>>(G, inj, tm, io);
            else stress_tile_adj<T, TX, TY, kAdjM, false><<<nwg, NT, 0, st>>>(G, inj, tm, io);
            break;
        case kPassVelA:
            if (ntp) vel_tile_adj<T, TX, TY, kAdjA, F32><<<nwg, NT, 0, st>>>(G, inj, n, tm, io);
            else vel_tile_adj<T, TX, TY, kAdjA, false><<<nwg, NT, 0, st>>>(G, inj, n, tm, io);
            break;
        default:
            if (ntp) stress_tile_adj<T, TX, TY, kAdjB, F32><<<nwg, NT, 0, st>>>(G, inj, tm, io);
            else stress_tile_adj<T, TX, TY, kAdjB, false><<<nwg, NT, 0, st>>>(G, inj, tm, io);
            break;
        }
    });
}

// Reverse sweep over the checkpointed segments: recompute each segment (storing
// v^{n+1/2} per step), then run the adjoint steps backwards; finally map the
// staggered-point gradients to the node arrays (accumulated into g_*).
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
    // residual injection per tap-disjoint colour: into A_v (cell adjoint), or into Y and g_b
    // (tiled adjoint, segment step m)
    auto inject = [&](int n, int m) {
        const TapAdjoint<T> ta = tiled ? tap_adjoint<T>(G, gws, GL, m) : TapAdjoint<T>{};
        for (size_t col = 0; col + 1 < c->color_off.size(); ++col) {
            const int cnt = c->color_off[col + 1] - c->color_off[col];
            const int *list = colors + c->color_off[col];
            if (tiled)
                inject_residual_tiled<T><<<(24 * cnt + 255) / 256, 256, 0, st>>>(ta, taps, list, cnt, residual, c->nt, n);
            else
                inject_residual<T><<<(3 * cnt + 255) / 256, 256, 0, st>>>(A.a[VX], A.a[VY], A.a[VZ], taps, list, cnt,
                                                                         residual, c->nt, n);
        }
    };
    c->grad_y = tiled;
    for (int sgi = GL.nseg - 1; sgi >= 0; --sgi) {
        const int n0 = sgi * GL.k, n1 = std::min(n0 + GL.k, c->nt);
        const char *ck = gws + GL.ckpt + (size_t)sgi * GL.group;
        for (int q = 0; q < NFIELD; ++q)
            HIP_TRY(hipMemcpyAsync(state_chunk<T>(c, G, q), ck + q * GL.chunk, c->L.field_bytes,
                                   hipMemcpyDeviceToDevice, st));
        if (!tiled)  // the cell adjoint's v^{n-1/2} of the segment's first step
            HIP_TRY(hipMemcpyAsync(gws + GL.prev, ck, prev_copy_bytes(c, GL), hipMemcpyDeviceToDevice, st));
        for (int n = n0; n < n1; ++n) {
            const int m = n - n0;
            char *slot = seg_slot(gws, GL, m);
            if (tiled) {  // velocities out of place: slot m-1 (the live state for m = 0) -> slot m
                Grid<T> Gv = G, Gs = G;
                for (int q = 0; q < 3; ++q) {
                    Gv.save[VX + q] = Gs.f[VX + q] = (T *)(slot + q * GL.fstep);
                    if (m > 0) Gv.f[VX + q] = (T *)(seg_slot(gws, GL, m - 1) + q * GL.fstep);
                }
                tm.begin(0);
                launch_pass<T, false>(c, Gv, inj, n, kPassVel, st);
                tm.end();
                tm.begin(2);
                launch_pass<T, false>(c, Gs, inj, n, kPassStress, st);
                tm.end();
            } else {  // in place, also storing v^{n+1/2} in slot m
                Grid<T> Gs = G;
                for (int q = 0; q < 3; ++q) Gs.save[VX + q] = (T *)(slot + q * GL.fstep);
                step<T, false>(c, Gs, inj, n, 0, taps, nullptr, st, tm);
            }
        }
        for (int n = n1 - 1; n >= n0; --n) {
            const int m = n - n0;
            if (tiled) {  // stress-B of step n + 1 and stress-A of step n in one pass
                const AdjTiles<T> P = adj_tiles<T>(G, gws, GL, m);
                launch_adj_pass<T>(c, P.g[0], none, n, kPassStressM, st, P.io[0]);
                launch_adj_pass<T>(c, P.g[1], none, n, kPassVelA, st, P.io[1]);
                inject(n, m);
            } else {
                set_stored_velocity(A, gws, GL, m);
                adj_stress_cell<T><<<grd, blk, 0, st>>>(G, A);
                inject(n, m);
                adj_vel_cell<T><<<grd, blk, 0, st>>>(G, A);
            }
        }
    }
    if (tiled) {  // stress-B of step 0, then the initial velocity's term of the b gradient
        const AdjTiles<T> P = adj_tiles<T>(G, gws, GL, 0);
        launch_adj_pass<T>(c, P.g[2], none, 0, kPassStressB, st, P.io[2]);
        launch_gb_initial<T>(G, A, gws, GL, st);
    }
    grad_finalize<T><<<grd, blk, 0, st>>>(G, A, g_lam, g_mu, g_rho);
    HIP_TRY(hipGetLastError());
    return FD3D_OK;
}


} // namespace

namespace fd3d {

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
    off += (size_t)((k + 2) / 3) * g.group;
    g.prev = off;
    off += g.group;
    g.res = off;
    off += round_up((size_t)c->opts.max_receivers * 3 * (size_t)(c->nt > 0 ? c->nt : 1) * c->tsize, kAlign);
    g.misfit = off;
    off += kAlign;
    g.total = off;
    return g;
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

} // namespace fd3d

extern "C" {

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
    ctx->adj_done = 0;
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
        rc = adjoint_impl<double>(ctx, src, nrec, rec_pos, (const double *)residual, (double *)g_lam,
                                  (double *)g_mu, (double *)g_rho, (char *)gws, GL, st);
    else
        rc = adjoint_impl<float>(ctx, src, nrec, rec_pos, (const float *)residual, (float *)g_lam, (float *)g_mu,
                                 (float *)g_rho, (char *)gws, GL, st);
    ctx->adj_done = rc == FD3D_OK;
    return rc;
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
    if (!ctx->grad_ready || !ctx->adj_done || gws != ctx->grad_ws)
        return fail(FD3D_ESTATE, "no adjoint state in this workspace (fd3d_adjoint has not run on it)");
    for (int f = 0; f < NFIELD; ++f)
        if (!fields[f]) return fail(FD3D_EINVAL, "field pointer is NULL");
    const GradLayout GL = make_grad_layout(ctx, ctx->grad_k);
    hipStream_t st = (hipStream_t)hip_stream;
    const dim3 blk(64, 4, 1), grd((ctx->n[0] + 63) / 64, (ctx->n[1] + 3) / 4, ctx->n[2]);
    for (int f = 0; f < NFIELD; ++f) {
        const char *a = (const char *)gws + GL.adj + f * GL.fstep;
        if (f <= VZ && ctx->grad_y) {  // tiled adjoint: from Y (intermediate fields 6-8)
            const char *y = (const char *)gws + GL.scr + (6 + f) * GL.fstep;
            if (ctx->tsize == 8)
                velocity_from_y<double><<<grd, blk, 0, st>>>(make_grid<double>(ctx), (const double *)y, f, (double *)fields[f]);
            else
                velocity_from_y<float><<<grd, blk, 0, st>>>(make_grid<float>(ctx), (const float *)y, f, (float *)fields[f]);
        } else if (f <= VZ) {
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


} // extern "C"
