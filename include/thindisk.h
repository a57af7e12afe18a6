/*
 * thindisk.h -- C ABI of the MI355X (gfx950) thin-disk self-gravity solver.
 *
 * The library computes the mid-plane gravitational force of an
 * infinitesimally thin disk whose surface density lives on a hierarchy of
 * nested uniform grids (Wang, Taam & Yen, "Self-Gravitational Force
 * Calculation of Infinitesimally Thin Gaseous Disks on Nested Grids"):
 *
 *   F_x(t) = sum over every active source cell c on every level of
 *            integral_c (xbar - x_t) / |rbar - r_t|^3 sigma(xbar, ybar),
 *
 * G = 1, with sigma linear in each cell about the cell centre
 * (Section 2.1, eq. eqnSigma):  sigma = s + dsdx (x - x_c) + dsdy (y - y_c).
 * The cell integrals are closed-form four-corner differences (eqs. eqnCalK,
 * eqnbnot0, eqnbeq0, with the slope antiderivatives v ln(u+r) and -r); the
 * sums are evaluated as zero-padded 2-D FFT generalized convolutions, with
 * the polyphase splits of Cases 2' and 3' (Section 2.2, eqs. eqnbmnn,
 * eqnbnmn) for pairs of levels of different resolution.  F_y follows by
 * exchanging x and y.
 *
 * A plan can compute the potential instead (td_plan_create_quantity with
 * TD_POTENTIAL): Phi(t) = - sum over active c of integral_c sigma / |rbar -
 * r_t| (eq. eqnPhixy0, Green's function -1/rho, G = 1), whose cell
 * integrals are the four-corner differences of u ln(v+r) + v ln(u+r),
 * v r/2 + (u^2/2) ln(v+r) and its exchange, through the same convolutions.
 *
 * Conventions
 *   - Level l holds one or more patches of n x n cells of width
 *     h_l = h0 / ratio^l and height aspect * h_l (ratio 2, 3 or 4; the same
 *     refinement ratio in x and y); level 0 is a single patch.  A patch's
 *     lower-left corner is (x0 + ox h_l, y0 + oy aspect h_l): ox, oy are
 *     integer offsets in level-l cells from the level-0 origin.  Every patch of
 *     level l+1 lies inside one patch of level l with its edges on level-l
 *     nodes (Section 2.1: integer ratio between nested levels).
 *   - A cell covered by a patch of level l+1 is not part of level l's
 *     domain: its sigma / slopes are ignored, and its force outputs are
 *     written as 0.
 *   - Every field is row-major [j][i] (x fastest), n * n elements per patch
 *     of the plan's dtype (float for TD_F32, double for TD_F64).
 *   - Forces have the units of sigma (G = 1): F = -grad Phi, attractive;
 *     the potential has the units of sigma times length.
 *
 * Ownership and errors
 *   - Field pointers are DEVICE pointers owned by the caller; the library
 *     reads / writes them only inside the stream work it enqueues.
 *   - The context owns twiddle tables and the resident kernel spectra; a
 *     plan owns its workspace and job lists.  Destroy plans before their
 *     context.
 *   - Every entry point returns td_status; on any error nothing has been
 *     enqueued and no output has been written.  td_last_error() returns a
 *     thread-local message describing the last failure.
 *   - Solves are asynchronous on the given HIP stream (NULL = the null
 *     stream); the caller synchronises before reading outputs.  Two solves
 *     of the SAME plan must not run concurrently (they share workspace).
 */
#ifndef THINDISK_H
#define THINDISK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TD_OK = 0,
    TD_EINVAL = 1,       /* bad argument (NULL, size, count, dtype)          */
    TD_EALIGN = 2,       /* a child patch edge is not on its parent lattice  */
    TD_ENEST = 3,        /* a child patch is not inside its parent           */
    TD_ENOMEM = 4,       /* device allocation failed or HBM budget exceeded  */
    TD_EDEVICE = 5,      /* HIP runtime error                                */
    TD_EBUSY = 6,        /* server admission refused (no room, no queueing)  */
    TD_EUNSUPPORTED = 7  /* valid but not supported by this build            */
} td_status;

typedef enum { TD_F32 = 0, TD_F64 = 1 } td_dtype;

/* One patch of n x n cells of the hierarchy (a grid Omega^l_k of Section
 * 2.1; physically square when the hierarchy's aspect is 1). */
typedef struct {
    int32_t level; /* refinement level, 0 = base                          */
    int32_t n;     /* cells per side                                      */
    int32_t ox;    /* lower-left offset in this level's cells, from the   */
    int32_t oy;    /* level-0 origin                                      */
} td_patch;

/* A nested-grid hierarchy: exactly one level-0 patch (at offset 0, 0), and
 * on every level l >= 1 one or more non-overlapping patches, each inside a
 * patch of level l-1 with its edges on level-(l-1) nodes (Section 2.1:
 * integer refinement ratio).  Patches are listed grouped by level, level 0
 * first; every per-patch array of a request follows this order. */
typedef struct {
    double x0, y0;           /* lower-left corner of level 0              */
    double h0;               /* level-0 cell width (x side)               */
    int32_t ratio;           /* refinement ratio between levels: 2, 3, 4  */
    int32_t npatches;        /* 1 .. TD_MAX_PATCHES                       */
    const td_patch* patches; /* [npatches], grouped by level              */
    double aspect;           /* cell height / width, every level (Section
                                2.1 allows different x and y spacings);
                                0 = square cells, else in [1/64, 64]      */
} td_hierarchy;

#define TD_MAX_LEVELS 8
#define TD_MAX_PATCHES 8   /* over all levels                             */
#define TD_MAX_N 2048      /* cells per side of a level's bounding square */

typedef struct td_context td_context;
typedef struct td_plan td_plan;
typedef struct td_batch td_batch;
typedef struct td_server td_server;

/* Where the in-cell slopes of the linear reconstruction (Section 2.1, eq.
 * eqnSigma) come from.  The paper fixes the slopes only as constants of each
 * cell.  TD_SLOPES_ESTIMATE derives them from sigma on the device, inside
 * the solve: the centred difference (s[i+1] - s[i-1]) / 2h of the cell
 * values, the one-sided difference towards the interior in a patch's first
 * and last column (row), and 0 along an axis where the patch is one cell
 * wide.  Each patch uses only its own values, covered cells included (their
 * stored value enters their neighbours' slopes; as sources they are still
 * excluded).  With these slopes the solver reproduces the error tables of
 * Section 3 (Tables 1-5). */
#define TD_SLOPES_GIVEN 0     /* dsdx / dsdy as passed (NULL = zero)      */
#define TD_SLOPES_ESTIMATE 1  /* from sigma, as above; dsdx, dsdy NULL    */

/* One force solve.  Arrays are indexed by patch (hierarchy order); patch k
 * holds n_k x n_k values, row-major [y][x].  All pointers are device
 * pointers of the plan's dtype, aligned to its element size (TD_EINVAL
 * otherwise).  With TD_SLOPES_GIVEN, dsdx / dsdy may be NULL (all slopes
 * zero) and an individual entry may also be NULL.  A zero-initialised
 * slopes field means TD_SLOPES_GIVEN. */
typedef struct {
    td_plan* plan;
    const void* const* sigma;   /* [npatches] sigma at cell centres         */
    const void* const* dsdx;    /* [npatches] or NULL: x-slope in each cell */
    const void* const* dsdy;    /* [npatches] or NULL                       */
    void* const* fx;            /* [npatches] outputs                       */
    void* const* fy;            /* [npatches] outputs                       */
    int32_t slopes;             /* TD_SLOPES_GIVEN or TD_SLOPES_ESTIMATE    */
} td_request;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `hip_device`.  `hbm_budget_bytes` caps the
 * device memory the context may hold (resident spectra + plan workspace);
 * 0 = no cap.  */
td_status td_context_create(int hip_device, size_t hbm_budget_bytes, td_context** out);
td_status td_context_destroy(td_context* ctx);
/* Bytes currently held by the context and its plans. */
td_status td_context_usage(const td_context* ctx, size_t* bytes_in_use, size_t* spectra_bytes);

/* Debug mode (flags 0 = off).  With TD_DEBUG_NONFINITE every solve of the
 * context -- td_solve, td_solve_noalloc, batches, served requests -- also
 * counts the NaN / Inf values it wrote to its outputs, on the solve's
 * stream after its passes (one small launch per output array; none under
 * graph capture, where a batch replay is counted after the replay).  The
 * counter is allocated when the mode is first enabled. */
#define TD_DEBUG_NONFINITE 1
td_status td_context_set_debug(td_context* ctx, int32_t flags);
/* Wait for the device, return the number of non-finite outputs counted
 * since the previous call (0 if debug mode was never enabled), clear it. */
td_status td_debug_nonfinite(td_context* ctx, uint64_t* count);

/* ---------------------------------------------------------------- geometry */

/* Validate a hierarchy (ratio, sizes, alignment, nesting, overlap, aspect).
 * TD_OK if it can be planned.  Levels may differ in resolution by at most
 * 16x (ratio^(levels-1) <= 16), and each level's patches must span at most
 * TD_MAX_N cells (TD_EUNSUPPORTED otherwise); an aspect outside 0 or
 * [1/64, 64] is TD_EINVAL. */
td_status td_hierarchy_check(const td_hierarchy* h);

/* For a hierarchy of one patch per level (patches[l] on level l, sizes
 * given): fill patches[1..].ox/oy so that each child patch is centred as
 * near as its parent lattice allows to (cx[l-1], cy[l-1]) -- lower-left
 * rounded to the nearest parent node and clamped inside the parent
 * (requested centres need not lie on any lattice).  patches[0] gets offset
 * (0, 0); inout->patches is set to `patches`. */
td_status td_hierarchy_snap(td_hierarchy* inout, td_patch* patches, const double* cx,
                            const double* cy);

/* ---------------------------------------------------------------- plans */

/* What a plan's solves compute. */
#define TD_FORCE 0       /* Fx into fx, Fy into fy (Section 2.1)              */
#define TD_POTENTIAL 1   /* Phi into fx (eq. eqnPhixy0); fy may be NULL, else
                            it receives 0 */

/* Validate the hierarchy, build (or find resident) the kernel spectra for
 * every level pair, and allocate the plan's workspace.  The kernel tables
 * (cell integrals of every offset and polyphase phase) are generated on the
 * GPU in FP64 and transformed in FP64; TD_F32 plans use them rounded to
 * FP32.  Synchronous.  td_plan_create makes a TD_FORCE plan. */
td_status td_plan_create(td_context* ctx, const td_hierarchy* h, td_dtype dtype,
                         td_plan** out);
/* As td_plan_create, for quantity TD_FORCE or TD_POTENTIAL (TD_EINVAL
 * otherwise).  A potential plan has its own resident spectra (the three
 * potential tables; the second component's tables are zero, so a potential
 * solve costs what a force solve does); its solves write Phi, in units of
 * sigma times length, into the fx outputs.  Force and potential plans may
 * share a batch or a server. */
td_status td_plan_create_quantity(td_context* ctx, const td_hierarchy* h, td_dtype dtype,
                                  int32_t quantity, td_plan** out);
/* Host-only planning: validate the hierarchy, build every job list of the
 * plan that td_plan_create would build (default launch shapes) and prove
 * on the host that each job's reads and writes stay inside its workspace,
 * fields and kernel spectra and that every workspace row a pass reads was
 * written by the pass before.  Needs no device.  workspace_bytes (may be
 * NULL) receives the plan's workspace size. */
td_status td_plan_check(const td_hierarchy* h, td_dtype dtype, size_t* workspace_bytes);
/* Workspace and (shared, resident) spectrum bytes this plan uses. */
td_status td_plan_footprint(const td_plan* plan, size_t* workspace_bytes,
                            size_t* spectra_bytes);
td_status td_plan_destroy(td_plan* plan);

/* Enqueue one solve on `hip_stream` (a hipStream_t, or NULL).  The field
 * pointers travel in the kernel arguments: nothing is copied to the device
 * per solve, and a solve captured into a graph replays on the captured
 * pointers. */
td_status td_solve(const td_request* req, void* hip_stream);

/* td_solve for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  It
 * runs the same kernels and jobs as td_solve (identical results) but takes
 * its workspace from a fixed device array of TD_NOALLOC_SCRATCH_BYTES
 * (32 MiB) per GPU, part of the library's code object and held until the
 * process ends, instead of the plan's own workspace; it calls no hipMalloc,
 * hipFree or other allocating routine.  A plan whose workspace exceeds the
 * array (td_plan_footprint minus the job tables; e.g. more than two
 * 256^2 FP64 levels) is refused with TD_ENOMEM, nothing enqueued.  Every
 * call on a GPU shares that GPU's array, which keeps the last call's
 * contents (no solve reads workspace it has not written first): calls that
 * overlap on one GPU -- on different streams, or with another thread's call
 * -- race and must be ordered by the caller.  Plans, inputs and outputs as
 * for td_solve. */
#define TD_NOALLOC_SCRATCH_BYTES (32u << 20)
td_status td_solve_noalloc(const td_request* req, void* hip_stream);

/* ---------------------------------------------------------------- batches */

/* A batch plan fuses `count` plans (same dtype, same context) into one set
 * of launches: each FFT pass runs for every hierarchy of the batch in one
 * kernel launch per transform length.  The batch owns its own workspace. */
td_status td_batch_create(td_context* ctx, int32_t count, td_plan* const* plans,
                          td_batch** out);
/* Enqueue the solves (reqs[k].plan must be the k-th plan given at creation).
 * With use_graph != 0, the launches are captured once into a HIP graph and
 * replayed; before each replay the current field pointers are copied to the
 * batch's device pointer table on the stream, outside the graph, so a
 * replay always reads the request's pointers. */
td_status td_batch_solve(td_batch* batch, const td_request* reqs, int use_graph,
                         void* hip_stream);
td_status td_batch_footprint(const td_batch* batch, size_t* workspace_bytes);
/* How the batch launches its column pass (the fused column FFTs and
 * spectral products; the row passes always run one workgroup per job).
 * TD_LAUNCH_DIRECT (the default): one workgroup per job, dispatched by the
 * hardware.  TD_LAUNCH_PERSISTENT: each column launch has a grid of about
 * as many workgroups as the device holds at once, and each workgroup takes
 * jobs from work lists built at creation, one per XCD (the jobs of one
 * spectral column together, longest first); a workgroup whose list is
 * drained takes jobs from the others.  The lists' counters live in the
 * batch and are zeroed by a kernel ahead of each solve (also inside a
 * captured graph), so two solves of one batch must not run concurrently,
 * as for its workspace.  Results are identical; on the 64-disk batch the
 * persistent launches measured 5% slower than direct ones in FP32 and
 * FP64.  Changing the mode drops a captured graph (after waiting for the
 * device). */
#define TD_LAUNCH_DIRECT 0
#define TD_LAUNCH_PERSISTENT 1
td_status td_batch_set_launch(td_batch* batch, int32_t mode);
td_status td_batch_destroy(td_batch* batch);

/* ---------------------------------------------------------------- autotune */

/* Time the candidate launch shapes (FFTs per workgroup, LDS budget) of every
 * pass for transform lengths up to max_M in `dtype`, keep the fastest, and
 * use them for plans created afterwards.  With db_path != NULL, results are
 * read from / appended to that JSON file (keyed by pass, M, dtype, arch). */
td_status td_autotune(td_context* ctx, td_dtype dtype, int32_t max_M, const char* db_path);

/* ---------------------------------------------------------------- serving */

/* A server owns a worker thread that takes submitted solves, admits them by
 * HBM footprint (plan workspace against the context budget), groups the
 * admitted ones into batches as they arrive (continuous batching: requests
 * that arrive while others run join the next launch) and runs up to
 * max_inflight batches concurrently on its own streams. */
td_status td_server_create(td_context* ctx, int32_t max_inflight, int32_t max_batch,
                           td_server** out);
/* Requests waiting for admission at most (default 65536); submissions
 * beyond it are refused (see td_server_submit). */
td_status td_server_set_queue_limit(td_server* s, int32_t max_queued);
/* Submit a solve.  The request's plan must stay alive until the ticket is
 * done.  Ordering: the call records an event on `hip_stream` (a hipStream_t
 * of the caller, NULL = the null stream), and the solve starts only after
 * the work enqueued there before the call -- the writes of sigma and the
 * slopes, and any earlier use of the output buffers -- has completed.  The
 * caller must not write the inputs or touch the outputs again until the
 * ticket is done.  If the server has no room (queue at its limit) and
 * queue_if_full is 0, returns TD_EBUSY (counted as refused).  Arrival time
 * = time of the call. */
td_status td_server_submit(td_server* s, const td_request* req, int32_t queue_if_full,
                           void* hip_stream, uint64_t* ticket);
/* Submit a solve of a hierarchy for which the caller holds no plan
 * (req->plan must be NULL; the other fields of req as for td_solve, with
 * npatches of `h`).  The server plans the hierarchy on a thread of its own
 * -- spectra and job tables are built on the context's stream while
 * flights keep running -- keeps the plan for later requests of the same
 * hierarchy (until the server is destroyed), and then admits the request as
 * td_server_submit does.  Validation errors are returned at once; planning
 * failures (e.g. TD_ENOMEM) are reported by td_server_poll.  Ordering and
 * refusal as td_server_submit. */
td_status td_server_submit_hierarchy(td_server* s, const td_hierarchy* h, td_dtype dtype,
                                     int32_t quantity, const td_request* req,
                                     int32_t queue_if_full, void* hip_stream, uint64_t* ticket);
/* done = 1 once the outputs of `ticket` are complete on the device.
 * latency_s = completion - submission (seconds), valid when done.  A ticket
 * reported done (or failed) is forgotten: polling it again is TD_EINVAL.  A
 * request that failed returns its error status (e.g. TD_ENOMEM when its
 * workspace can never fit in the budget) instead of TD_OK. */
td_status td_server_poll(td_server* s, uint64_t ticket, int32_t* done, double* latency_s);
/* Block until every submitted request is done. */
td_status td_server_drain(td_server* s);
/* Cancel a request that has not started (queued or waiting for its plan);
 * TD_EINVAL if unknown or started.  The ticket is forgotten. */
td_status td_server_cancel(td_server* s, uint64_t ticket);
/* Counters: completed, cancelled, refused, deferred (admission waited for
 * memory), batches launched, peak queue depth. */
td_status td_server_stats(const td_server* s, uint64_t* completed, uint64_t* cancelled,
                          uint64_t* refused, uint64_t* deferred, uint64_t* batches,
                          uint64_t* peak_queue);
/* Hierarchies planned by the server (td_server_submit_hierarchy) and
 * requests that failed. */
td_status td_server_stats2(const td_server* s, uint64_t* planned, uint64_t* failed);
/* Stop accepting work, finish every submitted request, free the server's
 * streams, workspace pool and the plans it made. */
td_status td_server_destroy(td_server* s);

/* ---------------------------------------------------------------- diagnostics */

/* Write the FP64 kernel table of one level pair kind into host memory:
 * out[6][M][M], entry [ny][nx] is the cell integral for a lattice offset
 * (output - input) of (nx or nx-M, ny or ny-M), in units of the finer cell
 * width (the cell height is aspect widths; 0 = square); kind = 1 (same
 * level), 2 (finer source, ratio m), 3 (coarser source, ratio m); (kx, ky)
 * the polyphase phase.  TD_FORCE: I0, Ixx, Ixy,
 * J0, Jyy, Jyx, Case-3 slope entries with the factor 1/m that converts the
 * coarse source's slope scaling.  TD_POTENTIAL: P0 = int 1/r, Px = int
 * (u-uc)/r, Py = int (v-vc)/r and three zero planes, Case-3 entries with
 * 1/m (slopes 1/m^2).  Synchronous; for tests. */
td_status td_kernel_table(td_context* ctx, int32_t quantity, double aspect, int32_t M,
                          int32_t kind, int32_t m, int32_t kx, int32_t ky, double* out_host);

/* The timed launch kinds of a solve, in launch order. */
#define TD_NPASS 4   /* row_fwd, col, row_inv, row_inv_accumulate */

/* Per-pass timing.  `pass_mask` selects the launch kinds to time (bit p =
 * kind p in TD_NPASS order; TD_TIMING_ALL for every kind, 0 to stop).
 * While enabled, every solve enqueued outside graph capture records a HIP
 * event pair around each selected kind on the solve's stream.
 * td_timing_read waits for the recorded events, writes the summed
 * milliseconds and the number of timed launches per kind (arrays of
 * TD_NPASS, either may be NULL) since the previous read, and clears them. */
#define TD_TIMING_ALL ((1 << TD_NPASS) - 1)
td_status td_timing_enable(td_context* ctx, int pass_mask);
td_status td_timing_read(td_context* ctx, double* ms, int64_t* launches);

/* Algorithmic HBM bytes one solve of the plan moves in each pass (array of
 * TD_NPASS), for requests with the given slopes mode: row_fwd reads every
 * source value in range (sigma only with TD_SLOPES_ESTIMATE, whose slope
 * jobs re-read sigma) and writes its row spectra; col reads every
 * row-spectrum plane and every stored kernel plane once and writes every
 * column output once; row_inv reads its column outputs once per target row
 * that uses them and writes (or reads and writes, when accumulating) every
 * force value.  TD_EINVAL for an unknown slopes mode. */
td_status td_plan_traffic(const td_plan* plan, int32_t slopes, double* bytes);

const char* td_status_string(td_status s);
const char* td_last_error(void);
/* Library version string. */
const char* td_version(void);

#ifdef __cplusplus
}
#endif
#endif /* THINDISK_H */
