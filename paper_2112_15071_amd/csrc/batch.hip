// Batches: many contexts (uneven grids, own models, sources and receivers) stepped
// together, one persistent launch per pass for all shots, optionally captured once as a
// hipGraph holding the whole nt-step sequence; the batch tuner and the batched gradient.
//
// Schedules.  Lockstep: every launch covers every shot, and the shots advance one step
// at a time together.  Cache-blocked groups: the shots, taken from the smallest working
// set (nine fields and three model arrays) to the largest, are cut into runs whose
// working sets add up to at most a given number of bytes; one group runs all its nt
// steps (one launch per pass over the group's shots) before the next group starts.
// Sized to the last-level (Infinity) cache, a group's fields stay resident from one step
// to the next.  Shots are independent, so both schedules give every shot the same result
// bit for bit.
#include "host.h"

#include <new>

using namespace fd3d;

// Shots at positions [s0, s0 + ns) of the batch's schedule order, stepped by one launch
// per pass: their work items and receiver components (counted from the group's first),
// the persistent grid size and the tile shapes of the launch (tx2 = 0: one shape).
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

// Two contexts whose batched passes read the same model arrays: the caller's, in place,
// or one copy in interleaved rows (see share_model).
bool shares_model(const fd3d_ctx *a, const fd3d_ctx *b)
{
    return a->L.rows == b->L.rows && (a->lam == b->lam || a->mu == b->mu || a->rho == b->rho);
}

// A context with interleaved rows reads its own copy of the model.  In a batch, the shots
// whose contexts were created over the same caller arrays with the same grid and type hold
// identical copies in the same layout, and all read the copy of the first such shot: one
// launch then streams the shared model once, as shots over separate arrays do.
template <typename T> void share_model(Grid<T> &G, const fd3d_ctx *c, fd3d_ctx *const *ctx, int nshot)
{
    if (!c->L.model) return;
    for (int r = 0; r < nshot; ++r) {
        const fd3d_ctx *o = ctx[r];
        if (o == c) return;
        if (o->L.model && o->lam == c->lam && o->mu == c->mu && o->rho == c->rho && o->tsize == c->tsize &&
            o->n[0] == c->n[0] && o->n[1] == c->n[1] && o->n[2] == c->n[2]) {
            G.lam = (const T *)(o->ws + o->L.model);
            G.mu = (const T *)(o->ws + o->L.model + o->L.fstep);
            G.rho = (const T *)(o->ws + o->L.model + 2 * o->L.fstep);
            return;
        }
    }
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
    // the gradient's passes stream its per-shot data (stored velocities, accumulators) and
    // keep the model, which the shots share, under the plain policy
    constexpr int NTD = sizeof(T) == 4 ? 2 : 0;
    switch (pass) {
    case kPassVel: vel_tile_multi<T, TX, TY, TX2, TY2, FS><<<g, NT, 0, st>>>(d, S, W, n); break;
    case kPassStress: stress_tile_multi<T, TX, TY, TX2, TY2, FS><<<gs, NT, 0, st>>>(d, S, W, n, rec); break;
    case kPassVelSave: vel_tile_multi<T, TX, TY, TX2, TY2, FS, kFwdSave, false, NTD><<<g, NT, 0, st>>>(d, S, W, n); break;
    case kPassStressA:
        stress_tile_multi<T, TX, TY, TX2, TY2, false, kAdjA, false, NTD><<<g, NT, 0, st>>>(d, S, W, n, none);
        break;
    case kPassStressM:  // one tile shape only: two shapes' LDS planes of this pass exceed a CU's LDS
        if constexpr (TX2 == 0) stress_tile_multi<T, TX, TY, 0, 0, false, kAdjM, false, NTD><<<g, NT, 0, st>>>(d, S, W, n, none);
        else return fail(FD3D_EINVAL, "stress-M batches take one tile shape");
        break;
    case kPassVelA: vel_tile_multi<T, TX, TY, TX2, TY2, false, kAdjA, false, NTD><<<g, NT, 0, st>>>(d, S, W, n); break;
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
        share_model<T>(fw[p].G, c, b->ctx.data(), b->nshot);
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
        const hipError_t ie = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
            (void)hipGraphDestroy(g);
            return fail(FD3D_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
        }
        b->graph = g;
        b->graph_valid = true;
        b->graph_key = (long)key;
    }
    HIP_TRY(hipGraphLaunch(b->gexec, st));
    return FD3D_OK;
}

// ---- batched gradient ----------------------------------------------------------
// Batch workspace of fd3d_batch_gradient: descriptor arrays (nshot entries each) of the
// forward pass, of the segment recompute per segment slot m (velocity: v^{n-1/2} from
// slot m-1, or the live state for m = 0, v^{n+1/2} into slot m; stress: v^{n+1/2} of slot m),
// of the adjoint passes (stress-M and velocity-A per slot m, which read the velocity
// stored for segment step m; the closing stress-B), of the residual injection per slot m,
// and per checkpoint the save and restore copy lists.
struct BatchGradLayout {
    size_t fwd0, fwd_slot, fst_slot, sa_slot, va_slot, sb, inj_slot, save_copy, rest_copy, total;
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
    L.fst_slot = off;
    off += (size_t)k * L.fwd_bytes;
    L.sa_slot = off;
    off += (size_t)k * L.fwd_bytes;
    L.va_slot = off;
    off += (size_t)k * L.fwd_bytes;
    L.sb = off;
    off += L.fwd_bytes;
    L.inj_slot = off;
    off += (size_t)k * L.inj_bytes;
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
        share_model<T>(fw[s].G, c, b->ctx.data(), b->nshot);
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
        ShotInject<T> &a = ij[s];  // .t per segment slot below
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
    // descriptors of one adjoint pass: the shot's tile map, the pass's grid and outputs, no source
    auto adj_desc = [&](int s, const AdjTiles<T> &P, int p) {
        ShotFwd<T> d = fw[s];
        d.G = P.g[p];
        d.io = P.io[p];
        std::memset(&d.src, 0, sizeof d.src);
        for (int f = 0; f < NFIELD; ++f) d.src.i0[f] = d.src.j0[f] = d.src.k0[f] = -(1 << 28);
        return d;
    };
    std::vector<ShotFwd<T>> sb(S);
    for (int m = 0; m < k; ++m) {
        std::vector<ShotFwd<T>> f2 = fw, f3 = fw, sa(S), va(S);
        std::vector<ShotInject<T>> ijm = ij;
        for (int s = 0; s < S; ++s) {
            char *w = (char *)gws[s];
            char *slot = seg_slot(w, GL[s], m);
            for (int q = 0; q < 3; ++q) {
                f2[s].G.save[VX + q] = f3[s].G.f[VX + q] = (T *)(slot + q * GL[s].fstep);
                if (m > 0) f2[s].G.f[VX + q] = (T *)(seg_slot(w, GL[s], m - 1) + q * GL[s].fstep);
            }
            const AdjTiles<T> P = adj_tiles<T>(fw[s].G, w, GL[s], m);
            sa[s] = adj_desc(s, P, 0);
            va[s] = adj_desc(s, P, 1);
            if (m == 0) sb[s] = adj_desc(s, P, 2);
            ijm[s].t = tap_adjoint<T>(fw[s].G, w, GL[s], m);
        }
        std::memcpy(h + BL.fwd_slot + m * BL.fwd_bytes, f2.data(), fbytes);
        std::memcpy(h + BL.fst_slot + m * BL.fwd_bytes, f3.data(), fbytes);
        std::memcpy(h + BL.sa_slot + m * BL.fwd_bytes, sa.data(), fbytes);
        std::memcpy(h + BL.va_slot + m * BL.fwd_bytes, va.data(), fbytes);
        std::memcpy(h + BL.inj_slot + m * BL.inj_bytes, ijm.data(), S * sizeof(ShotInject<T>));
    }
    std::memcpy(h + BL.sb, sb.data(), fbytes);
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

    const bool merged = all.tx2 == 0;  // stress-M (one tile shape)
    // forward with checkpoints
    auto desc = [&](size_t off) { return (const ShotFwd<T> *)(bws + off); };
    const ShotRec<T> *rdesc = (const ShotRec<T> *)(b->ws + b->off_rec);
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
            pass(desc(BL.fwd_slot + (n - n0) * BL.fwd_bytes), n, kPassVelSave);
            pass(desc(BL.fst_slot + (n - n0) * BL.fwd_bytes), n, kPassStress);
        }
        for (int n = n1 - 1; n >= n0; --n) {
            const int m = n - n0;
            // stress-B of step n + 1 and stress-A of step n in one pass (with two tile shapes,
            // whose LDS planes of that pass do not fit one CU, as two passes)
            if (merged) {
                pass(desc(BL.sa_slot + m * BL.fwd_bytes), n, kPassStressM);
            } else {
                if (n + 1 < b->nt) pass(desc(BL.sb), n + 1, kPassStressB);
                pass(desc(BL.sa_slot + m * BL.fwd_bytes), n, kPassStressA);
            }
            pass(desc(BL.va_slot + m * BL.fwd_bytes), n, kPassVelA);
            const ShotInject<T> *idesc = (const ShotInject<T> *)(bws + BL.inj_slot + m * BL.inj_bytes);
            for (int q = 0; q < ncol; ++q)
                if (cbase[q] > 0)
                    inject_residual_multi<T><<<(8 * cbase[q] + 255) / 256, 256, 0, st>>>(idesc, S, q, cbase[q], b->nt, n);
        }
    }
    pass(desc(BL.sb), 0, kPassStressB);  // stress-B of step 0
    // chain rule per shot, in shot order (shots may share the output arrays)
    for (int s = 0; s < S; ++s) {
        fd3d_ctx *c = b->ctx[s];
        const dim3 blk(64, 4, 1), grd((c->n[0] + 63) / 64, (c->n[1] + 3) / 4, c->n[2]);
        launch_gb_initial<T>(fw[s].G, ag[s], (char *)gws[s], GL[s], st);
        grad_finalize<T><<<grd, blk, 0, st>>>(fw[s].G, ag[s], (T *)g_lam[s], (T *)g_mu[s], (T *)g_rho[s]);
        c->grad_ws = (const char *)gws[s];
        c->grad_k = k;
        c->grad_ready = 1;
        c->adj_done = 1;
        c->grad_y = 1;
    }
    HIP_TRY(hipGetLastError());
    return FD3D_OK;
}

} // namespace

extern "C" {

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
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        return fail(FD3D_EHIP, "hipEventCreate failed");
    }
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

} // extern "C"
