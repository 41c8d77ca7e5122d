/*
 * gravity.h -- C ABI of the MI355X thin-disk self-gravity library.
 *
 * The library computes the midplane force (F_x, F_y) of an infinitesimally
 * thin disk whose surface density is given, on disjoint rectangular zones, by
 * a first-order Taylor polynomial s_i + dsx_i (x - x_i) + dsy_i (y - y_i)
 * (Tseng, Shang & Yen, Section 2, the decomposition over zones D_i and the
 * Taylor density of each zone).  The force at every zone centre is
 *
 *   F_x = G sum_i [ s_i K^{x,0}_i + dsx_i K^{x,x}_i + dsy_i K^{x,y}_i ]
 *
 * (and F_y likewise) with the exact cell-integrated kernels of Section 2 at
 * z = 0; a plan with a height z != 0 gives (F_x, F_y, F_z) at that height
 * above every zone centre (the kernels of Section 2 at general z).  On a
 * uniform grid this double sum is a discrete convolution
 * (Section 4, the FFT form of the uniform-grid sum) and is evaluated by
 * zero-padded 2D FFTs, free of artificial boundary conditions.  On an AMR
 * grid (Section 3, Berger-Oliger refinement with leaf zones only) the same
 * leaf-by-leaf sum is evaluated exactly by injecting every leaf's linear
 * density onto the finest lattice and convolving with cell-centre kernels
 * (targets that are finest leaves) and lattice-corner kernels (targets that
 * are coarser leaves, whose centres are finest-lattice corners).
 *
 * Conventions
 *  - All array arguments of the solve calls are DEVICE
 *    pointers owned by the caller; they must stay valid until the work queued
 *    on `stream` has completed.  `stream` is a hipStream_t (NULL = the null
 *    stream).  Calls return once the work is queued.
 *  - Element type of every array is float for GRAVITY_F32 plans and double
 *    for GRAVITY_F64 plans.
 *  - "Composite packed" layout: the base n0 x n0 block first, then each patch
 *    of the descriptor in order; each block row-major (row = y index, x
 *    fastest).  Cells covered by a finer patch are not leaves: their input
 *    values are ignored and their outputs are written as 0.  A uniform grid
 *    is the base block alone.
 *  - Errors are returned as status codes; nothing aborts or throws across the
 *    ABI.  gravity_last_error() gives a message for the calling thread's last
 *    non-OK status.  A device fault surfaces as GRAVITY_EDEVICE.
 *
 * Thread safety: plans are immutable after creation; concurrent solves on
 * one plan are safe when each uses its own workspace and outputs.
 */
#ifndef GRAVITY_H
#define GRAVITY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gravity_plan_s *gravity_plan_t;

typedef enum {
    GRAVITY_OK = 0,
    GRAVITY_EINVAL = 1,       /* malformed descriptor or arguments */
    GRAVITY_ENOMEM = 2,       /* device allocation failed */
    GRAVITY_EDEVICE = 3,      /* HIP runtime or kernel error */
    GRAVITY_EUNSUPPORTED = 4, /* valid request outside the supported sizes */
    GRAVITY_EBUSY = 5         /* resource temporarily unavailable */
} gravity_status_t;

typedef enum { GRAVITY_F32 = 0, GRAVITY_F64 = 1 } gravity_prec_t;

/* GRAVITY_SLOPES_GIVEN: the first-order Taylor slopes (dsx, dsy) of every
 * zone are inputs (the paper's second-order method).  GRAVITY_SLOPES_NONE:
 * piecewise-constant density, dsx = dsy = 0 (first order). */
typedef enum { GRAVITY_SLOPES_NONE = 0, GRAVITY_SLOPES_GIVEN = 1 } gravity_slopes_t;

/*
 * How an AMR layout (nlevels > 1) is solved.
 *
 * GRAVITY_AMR_EXACT: the leaf-by-leaf sum of Section 2, to rounding.  Every
 * leaf's linear density is injected onto the finest lattice (exact by the
 * additivity of the zone integrals) and convolved with the cell-centre and
 * lattice-corner kernel families; cost follows the finest lattice
 * (n0 * 2^(nlevels-1) <= 4096 cells per side).
 *
 * GRAVITY_AMR_NESTED: an approximation whose cost follows the refined area
 * (finest lattices beyond 4096 cells per side; nlevels <= 6, midplane only).
 * Covered cells get the linear density of least-squares distance to their
 * children (mass and first moments kept); the base grid is solved exactly
 * with that restricted data; every refined level l is tiled by 64 x 64 boxes
 * of level-l cells, and at the level-l cells of each box
 *   F^l = F_fine + interp(F^{l-1} - F_coarse),
 * where F_fine and F_coarse are exact zero-padded FFT solves of the
 * level-l and level-(l-1) truncated composites on the box grown by 32
 * level-l cells on every side (128^2 and 64^2 cell regions), and interp
 * carries the parent-level difference (the field of everything outside the
 * region) to the child centres (biquadratic on the 3 x 3 parent cells where
 * they exist, else bilinear, planar or linear).  The level fields are summed
 * in FP64 and every leaf takes F^l of its own level.  Its deviation from the
 * exact leaf sum is of the order of 1e-5 relative (second order in the
 * parent spacing, largest along box edges).
 */
typedef enum { GRAVITY_AMR_EXACT = 0, GRAVITY_AMR_NESTED = 1 } gravity_amr_method_t;

/* A rectangle of nx x ny cells at refinement level `level` (1 .. nlevels-1;
 * the base grid is level 0; refinement ratio 2), lower-left cell (i0, j0) in
 * that level's global cell index.  i0, j0, nx, ny must be even, patches of
 * one level disjoint, and each patch must lie inside the level below it. */
typedef struct {
    int32_t level, i0, j0, nx, ny;
} gravity_patch_t;

typedef struct {
    int32_t n0x, n0y;               /* base cells per side; equal, power of two */
    double x0, y0;                  /* lower-left corner of the domain */
    double h0;                      /* base cell size */
    int32_t nlevels;                /* 1 = uniform grid */
    int32_t npatches;
    const gravity_patch_t *patches; /* host array, copied at plan time */
    gravity_prec_t prec;
    gravity_slopes_t slopes;
    double G;                       /* gravitational constant */
    double z;                       /* height of the target plane above the disk
                                       (domain units); 0 = midplane (Fx, Fy),
                                       otherwise (Fx, Fy, Fz) at that height */
    int32_t amr_method;             /* gravity_amr_method_t (AMR layouts only) */
} gravity_desc_t;

typedef struct {
    int32_t n_finest;    /* finest lattice cells per side, n0 * 2^(nlevels-1) */
    int32_t fft_size;    /* largest zero-padded FFT size per side: 2 * n_finest
                            (GRAVITY_AMR_NESTED: 2 * n0, the base solve) */
    int64_t n_cells;     /* composite-packed array length (all cells) */
    int64_t n_leaves;    /* leaf zones (forces computed) */
    size_t workspace_bytes;
    size_t resident_bytes; /* device memory held by the plan and its spectra */
    int32_t variants[3];   /* kernel variants in use (row forward, column, row inverse) */
    int32_t ncomp;         /* force components: 2 (midplane) or 3 (off-plane) */
} gravity_plan_info_t;

/*
 * Create a plan: validates the descriptor and builds (or takes from the
 * resident cache) the kernel spectra for its FFT size and precision.  The
 * kernel tables are the exact integrals of Section 2 (K^{x,0}, K^{x,x},
 * K^{x,y} and the y family; with desc->z != 0 those at height z and the
 * vertical family K^{z,0}, K^{z,x}, K^{z,y}) at every source offset, built
 * in double precision on the device and transformed with a double precision
 * FFT.  Sizes: 16 <= n_finest <= 4096, powers of two (GRAVITY_AMR_NESTED:
 * 16 <= n0 <= 4096 and nlevels <= 6, any finest lattice up to 2^30 cells).
 * Kernel variants: unless GRAVITY_AUTOTUNE=0, the first plan of each size,
 * precision and layout kind times every variant of its three FFT kernels
 * and keeps the fastest (GRAVITY_TUNE_FILE persists the choices,
 * GRAVITY_VARIANTS="rf,col,ri" forces them).
 * Errors: EINVAL (bad descriptor or nesting), EUNSUPPORTED (size or
 * non-square grid), ENOMEM, EDEVICE.  *out is NULL on error.
 * Runs on the calling thread's current HIP device, which the plan records;
 * solves must be issued with that device current.
 */
gravity_status_t gravity_plan(const gravity_desc_t *desc, gravity_plan_t *out);

/* Bytes of device workspace one gravity_solve on this plan needs. */
gravity_status_t gravity_plan_workspace_bytes(gravity_plan_t plan, size_t *bytes);

/* Sizes of a plan (see gravity_plan_info_t). */
gravity_status_t gravity_plan_get_info(gravity_plan_t plan, gravity_plan_info_t *info);

/*
 * Queue one solve on `stream`.
 *   sigma, dsx, dsy : composite-packed inputs (dsx, dsy may be NULL only for
 *                     GRAVITY_SLOPES_NONE plans; they are ignored there)
 *   fx, fy          : composite-packed outputs (leaf forces, 0 elsewhere)
 *   workspace       : device buffer of gravity_plan_workspace_bytes bytes,
 *                     256-byte aligned, not shared with concurrent solves
 * Errors: EINVAL (NULL pointer, misaligned workspace, off-plane plan),
 * EDEVICE.
 */
gravity_status_t gravity_solve(gravity_plan_t plan, const void *sigma, const void *dsx,
                               const void *dsy, void *fx, void *fy, void *workspace,
                               void *stream);

/*
 * Off-plane solve (plans with desc->z != 0; Section 2 at general z): the
 * force at height z above every leaf centre, as gravity_solve with a third
 * composite-packed output fz (the vertical component; attraction towards
 * the disk).  Errors: as gravity_solve; EINVAL for a midplane plan (use
 * gravity_solve) or a NULL fz.  Off-plane plans are solved through this
 * call, gravity_solve_batch_xyz and gravity_server_submit_xyz (the other
 * solve calls and the profiling call return EINVAL or EUNSUPPORTED).
 */
gravity_status_t gravity_solve_xyz(gravity_plan_t plan, const void *sigma, const void *dsx,
                                   const void *dsy, void *fx, void *fy, void *fz,
                                   void *workspace, void *stream);

/*
 * Allocation-free solve, for callers that cannot allocate device memory or
 * hand over a workspace (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  Same inputs, outputs and results as
 * gravity_solve (bit-identical), but the workspace is a static device array
 * of GRAVITY_NOALLOC_SCRATCH_BYTES bytes inside the library, one per device
 * (taken at the first such call on a device and held until the process
 * ends).  The call allocates nothing.  Every allocation-free solve on one
 * device shares that array: calls whose work overlaps on the device (other
 * streams, other threads) race and must be serialised by the caller; solves
 * queued on one stream are ordered and safe.  No part of the array needs
 * clearing: each stage writes every workspace element that a later stage
 * reads.
 * Errors: as gravity_solve; EUNSUPPORTED if the plan's workspace
 * (gravity_plan_workspace_bytes) exceeds GRAVITY_NOALLOC_SCRATCH_BYTES
 * (e.g. FP32 uniform grids up to 1024^2 fit, FP64 up to 512^2).
 */
#define GRAVITY_NOALLOC_SCRATCH_BYTES (64u << 20)
gravity_status_t gravity_solve_noalloc(gravity_plan_t plan, const void *sigma, const void *dsx,
                                       const void *dsy, void *fx, void *fy, void *stream);

/* Workspace bytes for gravity_solve_batch over these n plans. */
gravity_status_t gravity_batch_workspace_bytes(int32_t n, const gravity_plan_t *plans,
                                               size_t *bytes);

/*
 * Queue n independent solves (plans may differ in size, levels and
 * precision) as one batch: solves that share an FFT size and precision run
 * together in each kernel launch.  Arrays of n device pointers as in
 * gravity_solve (dsx/dsy may be NULL, or hold NULL entries for
 * GRAVITY_SLOPES_NONE plans).  Results are bit-identical to n separate
 * gravity_solve calls.  workspace: gravity_batch_workspace_bytes bytes.
 */
gravity_status_t gravity_solve_batch(int32_t n, const gravity_plan_t *plans,
                                     const void *const *sigma, const void *const *dsx,
                                     const void *const *dsy, void *const *fx,
                                     void *const *fy, void *workspace, void *stream);

/*
 * As gravity_solve_batch, but the uniform midplane solves with slopes and
 * 64 <= n0 <= 1024 (FFT sizes 128 to 2048) run in ONE persistent launch per
 * precision, whatever their sizes: a device work queue of units (row groups,
 * columns) in pass order, taken by resident blocks from an atomic counter;
 * a unit waits, with a bounded spin, until its own solve's previous pass is
 * complete (the units it waits for were taken earlier by running blocks, so
 * every wait ends).  The other solves of the batch run as in
 * gravity_solve_batch.  The persistent kernels use fixed transform shapes
 * (4 elements per thread; 8 in 2048-point columns) instead of the plans'
 * tuned variants, so results agree with gravity_solve to rounding rather
 * than bit for bit.  Per-solve argument blocks are uploaded through a
 * pinned staging buffer with an asynchronous copy on `stream`, so the call
 * is not meant for graph capture.
 * workspace: gravity_batch_workspace_bytes bytes (the same as for
 * gravity_solve_batch; it includes the launch's tables).
 */
gravity_status_t gravity_solve_batch_persistent(int32_t n, const gravity_plan_t *plans,
                                                const void *const *sigma, const void *const *dsx,
                                                const void *const *dsy, void *const *fx,
                                                void *const *fy, void *workspace, void *stream);

/*
 * Diagnostics of the last gravity_solve_batch_persistent call made with
 * these n plans and this workspace: waits for `stream` (the call's stream)
 * and stores in *abandoned the number of work units whose bounded wait
 * reached its limit, so that the unit and the rest of its block's work were
 * skipped and those solves' results are incomplete.  The queue's ordering
 * excludes this (every awaited unit is held by a running block); a non-zero
 * count reports a device or library fault.  Host-synchronising; for tests
 * and monitoring, not for the solve path.
 */
gravity_status_t gravity_batch_persistent_abandoned(int32_t n, const gravity_plan_t *plans,
                                                   const void *workspace, void *stream,
                                                   uint32_t *abandoned);

/*
 * As gravity_solve_batch, for batches that include off-plane plans:
 * fz holds n device pointers (entries of midplane plans are ignored and
 * may be NULL).  Results are bit-identical to the single-solve calls.
 */
gravity_status_t gravity_solve_batch_xyz(int32_t n, const gravity_plan_t *plans,
                                         const void *const *sigma, const void *const *dsx,
                                         const void *const *dsy, void *const *fx,
                                         void *const *fy, void *const *fz, void *workspace,
                                         void *stream);

/*
 * Profiling aid: queue one solve on `stream` as gravity_solve does, but
 * launch every stage (kernel) of the pipeline `reps` times back to back
 * between two HIP events recorded on that stream, wait for them, and return
 * the mean device time of one launch of each stage in
 * stage_ms[0 .. *nstages - 1] (at most 8 stages; names from
 * gravity_stage_name).  Every stage rewrites its whole output from its
 * input, so the outputs are those of a plain solve.
 * Errors: as gravity_solve; EINVAL if reps < 1 or stage_ms/nstages is NULL.
 */
gravity_status_t gravity_solve_profiled(gravity_plan_t plan, const void *sigma, const void *dsx,
                                        const void *dsy, void *fx, void *fy, void *workspace,
                                        void *stream, int32_t reps, double *stage_ms,
                                        int32_t *nstages);

/* Name of stage `stage` of this plan's pipeline ("" if out of range):
 * uniform plans "row_fwd", "col", "row_inv"; AMR plans add "gather".
 * (Plans of GRAVITY_AMR_NESTED are not profiled: EUNSUPPORTED.) */
const char *gravity_stage_name(gravity_plan_t plan, int32_t stage);

/*
 * Request server (continuous batching).  A server owns a device arena of
 * `hbm_budget_bytes` (allocated once, at creation) from which each admitted
 * request's workspace is taken, `nstreams` HIP streams of default priority,
 * and a dispatcher thread.  gravity_server_submit() queues a solve and
 * returns a ticket at once; the dispatcher admits pending requests in
 * arrival order as arena space frees up (a request that does not fit waits,
 * smaller later ones may pass it), groups admitted requests that can share
 * kernel launches (same size, precision, layout kind) into batches of up to
 * `max_batch`, and queues each batch on the least-loaded stream, so work of
 * different requests overlaps on the device.  Ordering with the caller: at
 * submit an event is recorded on the caller's `stream`, and the server's
 * stream waits for it before the request's kernels, so inputs written by
 * work queued earlier on that stream are read only once it is done.  The
 * dispatcher detects completion by polling an event recorded after each
 * batch (about every 20 microseconds while work is in flight); a request's
 * latency runs from submit to that detection (host monotonic clock).  A
 * request's result is bit-identical to a gravity_solve of the same plan and
 * inputs, alone or in any mix.  The budget covers request workspaces only:
 * the plans' resident spectra and maps, and the caller's arrays, are
 * outside it.  A batch whose launch fails is waited for on its stream before
 * its arena range is released, and every one of its requests completes with
 * the error status.
 * Plans and their resident spectra must outlive the requests that use them;
 * inputs and outputs stay caller-owned and must stay valid until completion.
 * Errors: EINVAL (bad arguments), ENOMEM (arena allocation; or, on submit, a
 * request whose workspace exceeds the whole budget).
 */
typedef struct gravity_server_s *gravity_server_t;

typedef struct {
    int64_t submitted, completed, in_flight, pending;
    double latency_p50_ms, latency_p99_ms, latency_max_ms; /* over completed requests */
    size_t budget_bytes, bytes_in_use, peak_bytes_in_use;
    int64_t batches, leaves_completed;
} gravity_server_stats_t;

gravity_status_t gravity_server_create(size_t hbm_budget_bytes, int32_t nstreams, int32_t max_batch,
                                       gravity_server_t *out);
/* Queue a solve (arrays as in gravity_solve); `stream`: the caller's stream
 * that produced the inputs (hipStream_t, NULL = null stream).  Returns a
 * ticket at once. */
gravity_status_t gravity_server_submit(gravity_server_t srv, gravity_plan_t plan, const void *sigma,
                                       const void *dsx, const void *dsy, void *fx, void *fy,
                                       void *stream, int64_t *ticket);
/* As gravity_server_submit, with the third output fz of an off-plane plan. */
gravity_status_t gravity_server_submit_xyz(gravity_server_t srv, gravity_plan_t plan,
                                           const void *sigma, const void *dsx, const void *dsy,
                                           void *fx, void *fy, void *fz, void *stream,
                                           int64_t *ticket);
/* *done = 1 once the ticket's solve has completed on the device. */
gravity_status_t gravity_server_poll(gravity_server_t srv, int64_t ticket, int32_t *done);
/* Block until the ticket completes; *latency_ms (optional) gets its latency. */
gravity_status_t gravity_server_wait(gravity_server_t srv, int64_t ticket, double *latency_ms);
/* Block until every submitted request has completed. */
gravity_status_t gravity_server_drain(gravity_server_t srv);
gravity_status_t gravity_server_get_stats(gravity_server_t srv, gravity_server_stats_t *stats);
/* Clear the latency record and counters (arena and streams are kept). */
gravity_status_t gravity_server_reset_stats(gravity_server_t srv);
/* Drain, stop the dispatcher, release streams and arena (NULL ignored). */
void gravity_server_destroy(gravity_server_t srv);

/* Release a plan (NULL is ignored).  Spectra stay resident while another
 * plan uses them.  The caller must ensure no queued solve still uses it. */
void gravity_plan_destroy(gravity_plan_t plan);

/* Device bytes currently held by the resident spectrum cache. */
size_t gravity_cache_bytes(void);

/* Message for the calling thread's last non-OK status ("" if none). */
const char *gravity_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GRAVITY_H */
