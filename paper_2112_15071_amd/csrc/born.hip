// Tangent-linear (Born) forward: the background and the perturbation stepped together,
// the perturbation driven by the model perturbation's source terms.
#include "host.h"

#include "born_cell.h"

using namespace fd3d;

namespace {

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
    const Grid<T> G = make_grid<T>(c);
    Grid<T> D = make_grid<T>(dc);
    if (c->L.model && dc->L.model) {  // the same model (checked): the perturbation reads c's copy
        D.lam = G.lam;
        D.mu = G.mu;
        D.rho = G.rho;
    }
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
        // the background and the perturbation in one velocity sweep and one stress sweep
        // (the Born modes of the tile bodies); the stress sweep samples both receiver sets
        TileIO<T> iov, ios;
        std::memset(&iov, 0, sizeof iov);
        std::memset(&ios, 0, sizeof ios);
        for (int q = 0; q < 3; ++q) {
            iov.out[q] = D.f[VX + q];
            ios.pin[q] = D.f[VX + q];
        }
        for (int q = 0; q < 6; ++q) {
            iov.pin[q] = D.f[SXX + q];
            ios.out[q] = D.f[SXX + q];
        }
        iov.acc[0] = (T *)drho;
        ios.acc[0] = (T *)dlam;
        ios.acc[1] = (T *)dmu;
        const bool ntp = sizeof(T) == 4 && stream_model(c);  // cache policy, as in launch_pass
        for (int n = 0; n < c->nt; ++n) {
            with_tile<T>(c->tile_x, c->tile_y, [&](auto tx, auto ty) {
                constexpr int TX = decltype(tx)::value, TY = decltype(ty)::value, NT = TX * TY;
                const int nb = nwg + (recg.nq + recd.nq + NT - 1) / NT;
                if (ntp) {
                    vel_tile_adj<T, TX, TY, kBornV, sizeof(T) == 4><<<nwg, NT, 0, st>>>(G, inj, n, tm, iov);
                    stress_tile_born<T, TX, TY, sizeof(T) == 4><<<nb, NT, 0, st>>>(G, inj, n, tm, ios, recg, recd);
                } else {
                    vel_tile_adj<T, TX, TY, kBornV><<<nwg, NT, 0, st>>>(G, inj, n, tm, iov);
                    stress_tile_born<T, TX, TY><<<nb, NT, 0, st>>>(G, inj, n, tm, ios, recg, recd);
                }
            });
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
    if (ctx->variant != dctx->variant ||
        (ctx->variant == FD3D_KERNEL_TILE && (ctx->tile_x != dctx->tile_x || ctx->tile_y != dctx->tile_y ||
                                              ctx->zchunk != dctx->zchunk)))
        return fail(FD3D_EINVAL, "the Born forward steps both contexts with one kernel configuration");
    hipStream_t st = (hipStream_t)hip_stream;
    return ctx->tsize == 8 ? born_impl<double>(ctx, dctx, src, dlam, dmu, drho, nrec, rec_pos, traces, dtraces, st)
                           : born_impl<float>(ctx, dctx, src, dlam, dmu, drho, nrec, rec_pos, traces, dtraces, st);
}

} // extern "C"
