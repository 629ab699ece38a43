/*
 * fd3d.h -- C ABI of the MI355X (gfx950) time-stepped 3D elastic velocity-stress
 * staggered-grid finite-difference library (arXiv 2112.15071).
 *
 * The operation (all entry points share it):
 *   Sec. 2.1, Eq.(1)-(3)  rho dv/dt = div(sigma) + f ;  dsigma/dt = C(lambda, mu) : strain rate
 *   Sec. 2.1.1            Graves staggering: sxx,syy,szz at (x,y,z); sxy at (x+1/2,y+1/2,z);
 *                         sxz at (x+1/2,y,z+1/2); syz at (x,y+1/2,z+1/2); vx at (x+1/2,y,z);
 *                         vy at (x,y+1/2,z); vz at (x,y,z+1/2)
 *   Sec. 2.1.2, Eq.(4)    fourth-order staggered derivative, weights 9/8 and -1/24, divided by dx
 *   Sec. 2.2              one copy of each field, updated in place: velocity pass, then stress pass
 *   Sec. 2.2.1            rho, lambda, mu at staggered points = means of the neighbouring nodes
 *   Sec. 2.4              receivers: trilinear sampling of v every step, kept on the device
 *   Sec. 2.5              edge damping (Cerjan profile) and a free top surface (stress imaging,
 *                         second-order z difference next to the surface)
 *
 * Conventions.
 *   - Arrays are x-fastest: idx = i + nx*(j + ny*k), k = 0 is the top (z down).
 *   - A component staggered along an axis has n-1 active samples there; the last slot
 *     stays zero.  Samples outside the grid read as zero.
 *   - T is float (FD3D_F32) or double (FD3D_F64), chosen once per context.
 *   - Positions are in grid units (node spacing 1), order (x, y, z).
 *   - Step n (0-based): velocity pass v^{n-1/2} -> v^{n+1/2} (force source uses wavelet[n]);
 *     receivers record v^{n+1/2} into traces[r][c][n]; stress pass sigma^n -> sigma^{n+1}
 *     (moment source uses wavelet[n]).  Inside a pass the source is added before the
 *     damping factor multiplies the field.
 *
 * Ownership.  The caller owns every device buffer (model, wavelet, traces, residual,
 * gradients, workspaces) and keeps it alive until the work enqueued on the stream has
 * finished.  The library never allocates device memory; it lays its state out inside
 * the caller's workspace.  A context is host memory freed by fd3d_destroy.
 *
 * Streams.  Every call enqueues on the caller's hipStream_t (NULL = default stream) and
 * returns without waiting, except fd3d_create (reads back model statistics) and calls
 * with check_finite set (read back one flag).
 *
 * Errors.  Functions return FD3D_OK (0) or a negative code; fd3d_last_error() gives a
 * message for the calling thread.  No C++ exception crosses the ABI.
 */
#ifndef FD3D_H
#define FD3D_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FD3D_OK 0
#define FD3D_EINVAL (-1)     /* bad shape, pointer, dtype, alignment or option */
#define FD3D_ECFL (-2)       /* dt above the O(2,4) bound 6/(7 sqrt 3) dx / vp_max (Eq.(5)) */
#define FD3D_EMODEL (-3)     /* rho <= 0, mu < 0, lambda + 2 mu <= 0 or a non-finite value */
#define FD3D_ERANGE (-4)     /* a source or receiver tap falls outside a component's active samples */
#define FD3D_EWS (-5)        /* workspace too small */
#define FD3D_EHIP (-6)       /* a HIP call or kernel launch failed */
#define FD3D_ENONFINITE (-7) /* check_finite found a non-finite field value */
#define FD3D_ESTATE (-8)     /* call out of order (e.g. adjoint without checkpoints) */

#define FD3D_F32 0
#define FD3D_F64 1

/* kernel variants of the step loop (fd3d_set_kernel) */
#define FD3D_KERNEL_CELL 0 /* one thread per cell, neighbours from global memory */
#define FD3D_KERNEL_TILE 1 /* LDS-staged x/y halo planes + register z sweep (default) */
#define FD3D_KERNEL_FUSED 2 /* velocity and stress of a step in one z sweep over a double-buffered
                               state; tiles 64x4 and 64x8 (FP32), 64x4 (FP64) */

/* field storage in the workspace (fd3d_opts.layout); every layout gives the same results */
#define FD3D_LAYOUT_AUTO 0     /* interleaved rows when a tile sweep over the whole depth fits one
                                  buffer window (9 nx ny nz samples in 1 GiB), separate arrays
                                  otherwise */
#define FD3D_LAYOUT_SEPARATE 1 /* one array per field; the model arrays are read in place */
#define FD3D_LAYOUT_ROWS 2     /* interleaved rows: [nz][ny][9][nx], field q in row q, so that a
                                  tile's rows of the nine fields lie side by side; the model is
                                  copied once, at create, into a block of the same shape.  Needs
                                  min(12, nz) planes of 9 nx ny samples within 1 GiB and
                                  9 nx ny nz < 2^31 (else FD3D_EINVAL) */

/* fd3d_forward flags */
#define FD3D_KEEP_STATE 1 /* start from the current state instead of zeros */

typedef struct fd3d_opts {
    int dtype;           /* FD3D_F32 or FD3D_F64 */
    int sponge[6];       /* damping width in cells per face: x-, x+, y-, y+, z- (top), z+ */
    double sponge_alpha; /* Cerjan coefficient; <= 0 selects 0.3 / width per face */
    int free_surface;    /* 1: stress-imaging free surface at k = 0 (top width ignored) */
    int check_finite;    /* 1: forward returns FD3D_ENONFINITE if the final state blew up */
    int max_receivers;   /* receiver capacity of the workspace; <= 0 selects 4096 */
    double dy, dz;       /* spacing along y and z (m); 0 selects dx (cubic cells).  Table 5
                          * runs cells of different size per axis: each Eq.(4) derivative
                          * divides by its own axis' spacing, point sources inject per
                          * cell volume dx dy dz, and the stability bound becomes
                          * dt <= (6/7) / (vp_max sqrt(1/dx^2 + 1/dy^2 + 1/dz^2)). */
    int vacuum_top;      /* > 0: vacuum free surface (Sec. 2.5): the model holds low values
                          * above the first solid node plane k = vacuum_top (typically
                          * lam = mu = 0 and a small density, which the model check then
                          * accepts), and every z derivative whose result lies within one
                          * cell of that plane takes the second-order difference.  The
                          * effective surface is half a cell above the plane.  The vacuum
                          * density must keep the interface stable (a few per cent of the
                          * solid's in the tests).  Excludes free_surface; forward only (no
                          * gradient, no Born), tile and cell kernels.  0: off. */
    const void *vacuum_map; /* with vacuum_top > 0, optional topography: device int32
                          * [ny][nx], the first solid node plane of each column (1 .. nz-1,
                          * checked at create, which copies it once to the host; the array
                          * must stay alive and unchanged while the context is used).  A
                          * sample between columns (half position in x or y) takes the
                          * deepest plane beside it.  NULL: vacuum_top everywhere. */
    int coarse[3];       /* all >= 2: coarse medium (Sec. 2.2.1: medium textures smaller than
                          * the simulation grid, every read a trilinear sample).  lam, mu, rho
                          * given to fd3d_create are then node arrays of (mx, my, mz) =
                          * coarse[0..2] nodes spanning the same box as the simulation grid
                          * (simulation coordinate x sits at coarse coordinate
                          * x (m - 1) / (n - 1)), and the step kernels read every medium value
                          * as the trilinear sample at its own position: rho at the three
                          * velocity samples, lambda and mu at the nodes, mu at the three shear
                          * samples (instead of means of node values).  Forward only (no
                          * gradient, Born or batch), tile kernels only, not with vacuum_top.
                          * fd3d_upsample followed by node arrays is the other reading of a
                          * coarse medium: it differs where a mean straddles a coarse node.
                          * All 0: lam, mu, rho are node arrays of the simulation grid. */
    int layout;          /* FD3D_LAYOUT_AUTO (0), FD3D_LAYOUT_SEPARATE or FD3D_LAYOUT_ROWS */
} fd3d_opts;

typedef struct fd3d_source {
    double pos[3];       /* grid units */
    double moment[6];    /* Mxx Myy Mzz Mxy Mxz Myz (N m): sigma_ij -= dt w M_ij s[n] / (dx dy dz) */
    double force[3];     /* Fx Fy Fz (N): v_i += dt b w F_i s[n] / (dx dy dz) */
    const void *wavelet; /* device T[nt]: s[n] (moment rate, 1/s, for moment sources) */
} fd3d_source;

typedef struct fd3d_ctx fd3d_ctx;

/* Library version string (static storage). */
const char *fd3d_version(void);

/* Message of the last failed call on this thread ("" if none). */
const char *fd3d_last_error(void);

/* Bytes of forward workspace for a grid (nine fields, damping profiles, receiver
 * descriptors, reduction scratch).  opts may be NULL (FP32, no damping, 4096 receivers). */
int fd3d_workspace_bytes(int nx, int ny, int nz, const fd3d_opts *opts, size_t *bytes);

/* Create a context over caller-owned device node arrays lam, mu, rho (T[nz][ny][nx],
 * Sec. 2.2 / 2.2.1) with spacing dx (m; dy, dz in opts), step dt (s) and nt steps.
 * Validates the model on the device (FD3D_EMODEL), checks dt against
 * (6/7) / (vp_max sqrt(1/dx^2 + 1/dy^2 + 1/dz^2)), i.e. 6/(7 sqrt 3) dx / vp_max for cubic
 * cells (FD3D_ECFL; Eq.(5) prints the rounded 0.495), builds the damping profiles on the host in double
 * and uploads them.  workspace: device, >= fd3d_workspace_bytes, 256-byte aligned.
 * With interleaved rows (fd3d_opts.layout) the model is copied into the workspace here
 * and the passes read that copy; the caller's arrays must still stay alive and unchanged
 * (batches and the Born forward recognise a shared model by their addresses).
 * Synchronises the stream once (model statistics). */
int fd3d_create(fd3d_ctx **out, int nx, int ny, int nz, const void *lam, const void *mu,
                const void *rho, double dx, double dt, int nt, const fd3d_opts *opts,
                void *workspace, size_t ws_bytes, void *hip_stream);

/* Run nt steps (Sec. 2.2 update order) from zero state (or the current state with
 * FD3D_KEEP_STATE).  src may be NULL (no source); its wavelet is device T[nt].
 * rec_pos: host double[nrec][3]; traces: device T[nrec][3][nt] (written).
 * FD3D_ERANGE if a tap of the source or a receiver is not an active sample. */
int fd3d_forward(fd3d_ctx *ctx, const fd3d_source *src, int nrec, const double *rec_pos,
                 void *traces, int flags, void *hip_stream);

/* For callers that cannot allocate device memory (tight serving loops, harnesses that
 * forbid allocation): fd3d_create + fd3d_forward (flags 0) + fd3d_get_state in one call,
 * with the whole forward workspace in the library's static device scratch instead of a
 * caller workspace.  The scratch holds FD3D_STATIC_SCRATCH_BYTES (64 MiB) per GPU, taken
 * when the library's code object is loaded on that GPU and held until the process ends;
 * grids whose fd3d_workspace_bytes exceed it are rejected with FD3D_EWS (with the default
 * options -- 4096 receivers, the automatic field layout, which is interleaved rows with a
 * model copy for grids this small -- FP32 grids up to 84^3 cells, FP64 up to 67^3).
 * Arguments as fd3d_create and fd3d_forward: model arrays, src (its wavelet), rec_pos and
 * traces are the caller's; final_state (9 device T[nz][ny][nx], order as fd3d_get_state)
 * receives the final state, or is NULL.  The call allocates no device memory and creates
 * no HIP object (no event, stream or graph); it synchronises the stream before it
 * returns.  Every call on one GPU shares that GPU's scratch, which keeps the last call's
 * state: the call zeroes what must start at zero, and calls that overlap on one GPU (from
 * several host threads) race. */
#define FD3D_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int fd3d_forward_static(int nx, int ny, int nz, const void *lam, const void *mu, const void *rho,
                        double dx, double dt, int nt, const fd3d_opts *opts, const fd3d_source *src,
                        int nrec, const double *rec_pos, void *traces, void *const final_state[9],
                        void *hip_stream);

/* Copy the state out of / into the context: fields[9] are device T[nz][ny][nx] in the
 * order vx vy vz sxx syy szz sxy sxz syz (v^{n-1/2}, sigma^n).  set_state zeroes the
 * pinned slots of the staggered components. */
int fd3d_get_state(fd3d_ctx *ctx, void *const fields[9], void *hip_stream);
int fd3d_set_state(fd3d_ctx *ctx, const void *const fields[9], void *hip_stream);

/* Model statistics read back at create: out[0] = vp_max, out[1] = vs_min over mu > 0
 * (0 if none), out[2] = rho_min, out[3] = largest stable dt (m/s, m/s, kg/m^3, s). */
int fd3d_model_info(const fd3d_ctx *ctx, double out[4]);

/* Field storage the context chose: FD3D_LAYOUT_SEPARATE or FD3D_LAYOUT_ROWS (never AUTO). */
int fd3d_get_layout(const fd3d_ctx *ctx, int *layout);

/* ---- FWI gradient: discrete adjoint with snapshot checkpointing -------------------
 *
 * J = 1/2 sum_{r,c,n} (d - d_obs)^2 over the traces of one shot; residual = dJ/dd.
 * The gradient is the exact transpose of the forward steps (velocity pass, sampling,
 * stress pass) taken in reverse order, with respect to the node arrays lambda, mu, rho
 * given to fd3d_create (chain rule through the Sec. 2.2.1 means).  The forward state is
 * checkpointed every ckpt_every steps; the reverse sweep restores a checkpoint,
 * recomputes its segment while storing v^{n+1/2} per step, then runs the adjoint steps
 * of the segment backwards.  The buoyancy gradient of the one-thread-per-cell kernels
 * takes each step's increment from the stored v^{n+1/2} and v^{n-1/2}; the tile kernels
 * sum the same terms by parts over the steps, from v^{n+1/2} alone, plus one term of the
 * initial velocity after step 0 (equal up to rounding).  Damped boundaries only
 * (FD3D_EINVAL with the free surface).  The gradient workspace gws is caller-owned
 * device memory, 256-byte aligned: groups of nine fields in the context's field layout
 * (adjoint state, gradient accumulators, intermediate fields, one per checkpoint --
 * ceil(nt / ckpt_every) --, the velocities of a segment, three steps per group --
 * ceil(ckpt_every / 3) --, and a copy of the segment's checkpoint, which only the
 * one-thread-per-cell kernels read) plus a residual buffer.
 */

/* Bytes of gradient workspace for checkpoints every ckpt_every steps (1 <= k <= nt). */
int fd3d_grad_workspace_bytes(const fd3d_ctx *ctx, int ckpt_every, size_t *bytes);

/* fd3d_forward that also writes the checkpoints into gws (flags as in fd3d_forward).
 * Must precede fd3d_adjoint on the same gws. */
int fd3d_forward_ckpt(fd3d_ctx *ctx, const fd3d_source *src, int nrec, const double *rec_pos,
                      void *traces, int flags, void *gws, size_t gws_bytes, int ckpt_every,
                      void *hip_stream);

/* Reverse sweep.  residual: device T[nrec][3][nt] (dJ/dd); src and receivers must be those
 * of the fd3d_forward_ckpt call.  Accumulates (+=) into g_lam, g_mu, g_rho (device
 * T[nz][ny][nx]).  Leaves the adjoint of the initial state in gws (see below).  Uses and
 * overwrites the context's forward state.  FD3D_ESTATE without a preceding checkpointed
 * forward on this gws. */
int fd3d_adjoint(fd3d_ctx *ctx, const fd3d_source *src, int nrec, const double *rec_pos,
                 const void *residual, void *g_lam, void *g_mu, void *g_rho, void *gws,
                 size_t gws_bytes, void *hip_stream);

/* One shot of the L2 misfit: fd3d_forward_ckpt (traces written), residual = traces - d_obs,
 * misfit[0] = J (device T, or NULL), then fd3d_adjoint (gradients accumulated). */
int fd3d_gradient(fd3d_ctx *ctx, const fd3d_source *src, int nrec, const double *rec_pos,
                  const void *d_obs, void *traces, void *misfit, void *g_lam, void *g_mu,
                  void *g_rho, void *gws, size_t gws_bytes, int ckpt_every, void *hip_stream);

/* Tangent-linear (Born) forward: the derivative of the traces along a model perturbation
 * (dlam, dmu, drho: device node arrays T[nz][ny][nx]).  Each step differentiates the
 * forward step (Sec. 2.1 Eq.(1)-(3) with Eq.(4)): the perturbation state takes the same
 * velocity and stress passes as the background, fed before each pass by the
 * perturbation's first-order effect on the background -- dt db (D_S sigma + force term)
 * with db = -b^2 drho_eff, then dt dC E(v) with dC built from dlam, dmu (means as for C).
 * With the tile kernels one velocity sweep and one stress sweep step both states.
 * ctx runs the background (src, traces: device T[nrec][3][nt] or NULL); dctx is a second
 * context over the same model arrays, grid, dtype, nt, dt, spacing, damping, field layout
 * and kernel configuration (fd3d_set_kernel), whose state holds the perturbation
 * (dtraces: device T[nrec][3][nt]).  Both states start at zero and are overwritten.
 * Damped boundaries only; tile or cell kernels (not fused).  FD3D_EINVAL when the
 * contexts do not match. */
int fd3d_born(fd3d_ctx *ctx, fd3d_ctx *dctx, const fd3d_source *src, const void *dlam,
              const void *dmu, const void *drho, int nrec, const double *rec_pos, void *traces,
              void *dtraces, void *hip_stream);

/* After fd3d_adjoint: the adjoint of the initial state (v^{-1/2}, sigma^0) into fields[9]
 * (device T[nz][ny][nx], order as fd3d_get_state) -- the dot-product test quantity.
 * FD3D_ESTATE unless an adjoint (fd3d_adjoint, fd3d_gradient or a batched gradient) has
 * run on gws since its checkpointed forward. */
int fd3d_get_adjoint_state(fd3d_ctx *ctx, const void *gws, void *const fields[9],
                           void *hip_stream);

/* ---- Batches: many shots stepped together ------------------------------------------
 *
 * A batch groups contexts (each with its own grid size, model, workspace, source and
 * receivers; one dtype, one nt and one free-surface option for all).  Each pass of each
 * step runs as ONE persistent launch over the flat list of every shot's tiles (the list
 * is split into 8 contiguous chunks, one per XCD); with use_graph the whole nt-step
 * sequence is captured once into a hipGraph and replayed by one hipGraphLaunch on the
 * caller's stream (recaptured when the tiling or receiver counts change).  Per-shot
 * results are identical to fd3d_forward on each context with the same tile shape.
 * fd3d_batch_set_schedule switches the forward from this lockstep order to
 * cache-blocked groups (the gradient always runs lockstep).
 * The batch workspace holds the per-shot descriptors (caller-owned device memory).
 * The contexts must outlive the batch. */
typedef struct fd3d_batch fd3d_batch;

int fd3d_batch_workspace_bytes(int nshot, fd3d_ctx *const *ctxs, size_t *bytes);
int fd3d_batch_create(fd3d_batch **out, int nshot, fd3d_ctx *const *ctxs, void *workspace,
                      size_t ws_bytes);

/* Tile shape for every shot of the batch (fd3d_kernel shapes) and the number of
 * persistent workgroups (0: CUs x occupancy, rounded to a multiple of 8). */
int fd3d_batch_set_kernel(fd3d_batch *b, int tile_x, int tile_y, int workgroups);

/* A second tile shape with the same workgroup size for the shots whose rows it covers
 * with fewer idle columns (tile2_x = tile2_y = 0: none).  Supported pairs: FP32 256x4 +
 * 64x16, 128x8 + 64x16, 256x4 + 128x8, 128x4 + 64x8; FP64 128x4 + 64x8.  FD3D_EINVAL
 * otherwise.  fd3d_batch_set_kernel sets one shape. */
int fd3d_batch_set_tiles(fd3d_batch *b, int tile_x, int tile_y, int tile2_x, int tile2_y, int workgroups);

/* Order of the batched forward.  group_bytes = 0 (default): lockstep, every launch covers
 * every shot and all shots advance one step at a time.  group_bytes > 0: cache-blocked
 * groups -- runs of consecutive shots (in batch order) whose working sets (9 fields and
 * 3 model arrays each, 12 x cells x sizeof(T) bytes per shot) add up to at most
 * group_bytes (a group holds at least one shot); each group runs all nt steps, one launch
 * per pass over its shots, before the next group starts, so that a group sized to the
 * last-level cache (256 MB Infinity Cache on MI355X) keeps its fields resident between
 * steps.  A group whose shots all use the tile kernel with one shape of their own
 * (fd3d_set_kernel / fd3d_autotune on each context) launches with that shape; other
 * groups use the batch's shapes.  Results per shot are the same in both orders. */
int fd3d_batch_set_schedule(fd3d_batch *b, size_t group_bytes);

/* Times `steps` batched steps (sources and receivers off, one warm-up run each) for
 * every supported tile shape and pair of shapes in lockstep, with the persistent grid
 * and with one workgroup per tile, then the cache-blocked schedule with group budgets of
 * 96, 128, 192, 256 and 384 MiB; keeps the fastest for later batch calls and writes it to best =
 * {tile_x, tile_y, tile2_x, tile2_y, workgroups (0 = persistent), group MiB (0 =
 * lockstep)} and its ms per step to *best_ms (each when non-NULL).  Every shot's forward
 * state is zeroed afterwards.  Synchronises the stream. */
int fd3d_batch_autotune(fd3d_batch *b, int steps, int best[6], double *best_ms, void *hip_stream);

/* srcs[nshot] (or NULL), nrec[nshot], rec_pos[nshot] (host double[nrec][3] each),
 * traces[nshot] (device T[nrec][3][nt] each); flags as fd3d_forward. */
int fd3d_batch_forward(fd3d_batch *b, const fd3d_source *srcs, const int *nrec,
                       const double *const *rec_pos, void *const *traces, int flags, int use_graph,
                       void *hip_stream);

/* Batched L2-misfit gradient: fd3d_gradient for every shot of the batch, stepped
 * together (forward with checkpoints, then per segment a batched recompute and batched
 * adjoint steps; residual injection per tap-disjoint colour, at most 4 colours per shot).
 * Per shot s: d_obs[s], traces[s] (written), misfit[s] (device T or NULL), g_*[s]
 * (accumulated; shots may share output arrays, they are added in shot order), gws[s]
 * (a gradient workspace of fd3d_grad_workspace_bytes(ctx_s, ckpt_every) bytes).  bws is a
 * batch gradient workspace of fd3d_batch_grad_workspace_bytes bytes.  flags: 0 or
 * FD3D_KEEP_STATE (start every shot from its context's current state).  Results per shot
 * equal fd3d_gradient's. */
int fd3d_batch_grad_workspace_bytes(const fd3d_batch *b, int ckpt_every, size_t *bytes);
int fd3d_batch_gradient(fd3d_batch *b, const fd3d_source *srcs, const int *nrec,
                        const double *const *rec_pos, const void *const *d_obs, void *const *traces,
                        void *const *misfit, void *const *g_lam, void *const *g_mu,
                        void *const *g_rho, void *const *gws, const size_t *gws_bytes,
                        int ckpt_every, int flags, void *bws, size_t bws_bytes, void *hip_stream);

void fd3d_batch_destroy(fd3d_batch *b);

/* Kernel selection for the step loop of later calls on this context.  All variants
 * compute the same update with the same operation order per sample. */
typedef struct fd3d_kernel {
    int variant;  /* FD3D_KERNEL_CELL, FD3D_KERNEL_TILE or FD3D_KERNEL_FUSED */
    int tile_x;   /* tile columns: 64, 128 or 256 */
    int tile_y;   /* tile rows: FP32 64x{4,8,16}, 128x{4,8}, 256x4; FP64 64x{4,8}, 128x4;
                     fused: FP32 64x{4,8}, FP64 64x4 */
    int zchunk;   /* z planes swept by one workgroup, >= 4 */
} fd3d_kernel;

/* Default at create: FD3D_KERNEL_TILE with 256x4 tiles (FP32, nx >= 256), 128x4
 * (nx >= 128) or 64x8, and 64-plane sweeps (nz >= 128) or 32.  FD3D_EINVAL for an
 * unsupported shape.  The fused variant keeps two copies of the state and swaps them
 * every step; the state accessors always address the current copy, and the gradient's
 * segment recompute and adjoint passes use the tile kernels of the same tile shape. */
int fd3d_set_kernel(fd3d_ctx *ctx, const fd3d_kernel *k);
int fd3d_get_kernel(const fd3d_ctx *ctx, fd3d_kernel *k);

/* Autotuner: times the cell kernel and every supported tile and fused shape with z chunks
 * of 4, 8, 16, 32, 64 and 128 planes and of ceil(nz / m) planes for m = 1 .. 8 (the whole
 * depth and its even splits; fused from 8 planes; the chunks that fit the grid) for
 * `steps` steps on this context (a warm-up and two timed runs each, the faster counting;
 * no source; on the caller's stream; waits for each timing), keeps the fastest for later
 * calls and writes it to *best (and its ms per step to *best_ms) when non-NULL.  The
 * forward state is zeroed afterwards. */
int fd3d_autotune(fd3d_ctx *ctx, int steps, fd3d_kernel *best, double *best_ms, void *hip_stream);

/* Per-kernel timing of the step loop.  With enable = 1, later forward calls record a
 * HIP event pair on the caller's stream around every kernel launch of the loop (the
 * kernels themselves are unchanged).  fd3d_profile_read waits for the last recorded
 * event and returns, per pass (0 = velocity, 1 = receiver sampling, 2 = stress,
 * 3 = fused step), the summed kernel time in ms and the number of launches of the last
 * profiled call.  The stress launch of the tile and cell kernels also samples the
 * receivers, so pass 1 is launched on its own only after a fused step. */
int fd3d_profile(fd3d_ctx *ctx, int enable);
int fd3d_profile_read(fd3d_ctx *ctx, double ms[4], int launches[4]);

/* Coarse medium grid (Sec. 2.2.1: the medium textures may be smaller than the simulation
 * grid, every read being a trilinear sample).  Samples coarse (device T[mz][my][mx]) at
 * every node of the simulation grid, fine (device T[nz][ny][nx]): both grids span the same
 * box corner node to corner node, so fine node i sits at coarse coordinate
 * i (m - 1) / (n - 1) per axis (m = 1: constant along that axis).  Weights and sums in
 * double.  Use it for lam, mu and rho before fd3d_create.  Caller-owned, non-overlapping
 * buffers; enqueued on the stream.  FD3D_EINVAL for NULL, sizes < 1, a bad dtype or
 * overlapping buffers. */
int fd3d_upsample(const void *coarse, int mx, int my, int mz, void *fine, int nx, int ny,
                  int nz, int dtype, void *hip_stream);

void fd3d_destroy(fd3d_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* FD3D_H */
