/*
 * hemamg.h -- C ABI of the MI355X (gfx950) aggregation-AMG solver library.
 *
 * The library solves A u = f (Section 2 of Ganesan & Shah, "SParSH-AMG: A
 * library for hybrid CPU-GPU algebraic multigrid and preconditioned iterative
 * methods") for a square CSR matrix A held in GPU memory, with algebraic
 * multigrid built by node-based heavy edge matching (Section 2.1.1,
 * Algorithm 2) used as a preconditioner of CG (Algorithm 4) or BiCGStab
 * (Algorithm 5).  Every step runs as HIP kernels on one GPU.
 *
 * Conventions for every entry point:
 *  - Indices are int32 and 0-based.  CSR rows store their diagonal, columns
 *    are strictly ascending, and the pattern is structurally symmetric
 *    ((i,j) stored iff (j,i) stored; values may differ).
 *  - Pointers marked [device] are GPU memory; [host] pointers are CPU memory.
 *  - All GPU work is enqueued on the given stream (hipStream_t passed as a
 *    void*; NULL is the default stream).  Calls that return data to the host
 *    synchronise that stream before returning.
 *  - Every function returns an amg_status and never aborts; on failure
 *    amg_last_error() holds a message for the calling thread.
 *  - A handle may be used by one thread at a time.
 */
#ifndef HEMAMG_H
#define HEMAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AMG_OK = 0,
    AMG_EINVAL = 1,        /* invalid argument or matrix                        */
    AMG_ENOMEM = 2,        /* GPU allocation failed                             */
    AMG_ENOTCONV = 3,      /* iteration limit reached (info and x still valid)  */
    AMG_EBREAKDOWN = 4,    /* Krylov breakdown: zero or non-finite denominator  */
    AMG_ENOTFINITE = 5,    /* NaN or Inf in the input                           */
    AMG_ESTALL = 6,        /* coarsening stalled above max_dense_rows           */
    AMG_ESINGULAR = 7,     /* coarsest matrix is singular                       */
    AMG_EHIP = 8           /* HIP runtime error                                 */
} amg_status;

typedef struct amg_hier amg_hier; /* opaque hierarchy handle, owned by the library */

/* CSR matrix.  [device] arrays; borrowed: they must stay valid and unchanged
 * for the lifetime of any handle built from them. */
typedef struct {
    int32_t n;              /* rows = columns, > 0                  */
    int64_t nnz;            /* row_ptr[n], < 2^31                    */
    const int32_t* row_ptr; /* [device] int32[n+1], row_ptr[0] = 0   */
    const int32_t* col_idx; /* [device] int32[nnz]                   */
    const double* val;      /* [device] float64[nnz]                 */
} amg_csr;

/* Hierarchy and cycle parameters (Section 3 setup phase; Algorithm 1). */
typedef struct {
    int32_t passes_per_level; /* matching passes composed per level: 1 or 2 (2)   */
    int32_t max_coarse_rows;  /* coarsen until n <= this, 1..4096 (64)            */
    int32_t max_levels;       /* levels including the coarsest, 1..64 (32)        */
    int32_t max_dense_rows;   /* largest coarsest level accepted when coarsening  *
                               * stalls or hits max_levels, 1..4096 (4096); the   *
                               * coarsest level is factored densely (LU) and      *
                               * applied as an explicit inverse                   */
    double omega;             /* damped-Jacobi weight (2/3)                       */
    int32_t pre, post;        /* smoothing sweeps before/after the coarse
                               * correction, 0..8 (1, 1)                          */
    int32_t true_res_period;  /* recompute b - A x every this many iterations,   *
                               * 0 = only when the recursive residual converges   *
                               * (50)                                             */
    int32_t precond_fp32;     /* 1: the V-cycle runs in float (level values,
                               * vectors and sums), the Krylov method and the
                               * coarsest solve stay in double; needs pre = post
                               * = 1.  The hierarchy itself is built in double
                               * either way, so aggregates and coarse operators
                               * do not change.  0: double throughout (0)         */
    double stall_ratio;       /* a level of n <= max_dense_rows rows becomes the
                               * coarsest when coarsening it would keep
                               * n_c >= stall_ratio * n rows; in (0, 1]; 1 stops
                               * only when no row is merged (0.9)                 */
    int32_t hem;              /* matching: 0 node-based (Algorithm 2), 1 edge-
                               * based (Algorithm 3: edges by weight descending,
                               * ties by smaller then larger endpoint) (0)         */
    int32_t alternate;        /* 1: node-based passes alternate direction (Section
                               * 2.1.1): the setup's passes, counted from 0 across
                               * levels, start from the first index when even and
                               * from the last when odd (vertices and row entries
                               * scanned downward, ties to the highest index);
                               * coarse ids follow each aggregate's smallest fine
                               * index either way.  Needs hem = 0.  0: every pass
                               * from the first index (0)                          */
} amg_params;

/* Result of a Krylov solve.  [host] */
typedef struct {
    int32_t iters;       /* number of solution updates performed               */
    double rel_res;      /* recursive ||r|| / ||b|| at the stop                */
    double true_rel_res; /* ||b - A x|| / ||b|| at the stop (last recomputed) */
    double setup_ms;     /* host wall time of the setup call that built the
                          * hierarchy (amg_setup, or amg_batch_setup for the
                          * whole batch; 0 for a batch made by
                          * amg_batch_create)                                  */
    double solve_ms;     /* host wall time of the call                         */
    int32_t levels;      /* levels of the hierarchy, the coarsest included     */
    int32_t status;      /* same as the return value                           */
} amg_info;

/* Device-memory allocator (the setup phase of Section 3 builds every coarse
 * level in GPU memory; Section 3.1 makes that memory the scarce resource, so
 * the caller may own it).  Every device buffer a handle or batch owns, and
 * every temporary of its setup, is drawn through it in a few large chunks:
 *  - alloc(bytes, ctx, stream) returns `bytes` (a multiple of 256) of device
 *    memory on the current device, 256-byte aligned, usable by work enqueued
 *    on `stream` (a hipStream_t, possibly NULL), or NULL on failure (the
 *    entry point then returns AMG_ENOMEM after freeing what it drew);
 *  - free(ptr, ctx, stream) returns a block alloc gave.  Work enqueued on
 *    `stream` may still use the block: the allocator must reuse it only for
 *    work ordered after that (stream-ordered release, as hipFreeAsync and
 *    PyTorch's caching allocator do).
 * Both are called on the thread of the entry point (for a server, on its
 * worker threads).  The allocator must outlive every handle, batch and
 * server it was given to.  Passing NULL (or a struct whose alloc is NULL)
 * uses the library's own stream-ordered pool. */
typedef struct {
    void* (*alloc)(size_t bytes, void* ctx, void* stream);
    void (*free)(void* ptr, void* ctx, void* stream);
    void* ctx;
} amg_allocator;

/* Device memory the library's own pool keeps for reuse on the current device
 * (the chunks of destroyed handles, batches and servers, held so that later
 * setups do not go back to the driver; at most a quarter of the device's
 * memory and 64 GiB).  amg_cached_bytes stores the kept bytes in *bytes
 * (AMG_EINVAL for NULL).  amg_release_cached waits for the work that last
 * used each kept chunk, frees the chunks and returns the pool's unused
 * memory to the driver, as a caller sharing the device with another
 * allocator may want to do; live handles, batches and servers are not
 * touched.  Memory drawn through a caller's amg_allocator is never kept.
 * Errors: AMG_EHIP.  [host] */
amg_status amg_cached_bytes(uint64_t* bytes);
amg_status amg_release_cached(void);

/* Fills *p with the defaults shown above.  [host] */
amg_status amg_params_default(amg_params* p);

/* Setup phase (Section 3; Algorithm 2 per pass; coarse operator P^T A P of
 * Section 2.1.1; LU of the coarsest matrix, Section 2).  Validates A (sorted
 * in-range columns, non-zero finite diagonal, finite values, structural
 * symmetry), builds every level on the GPU and returns a handle in *out
 * (*out = NULL on error).  Blocks the host until the stream has finished.
 * Coarse levels, D^{-1}, aggregate maps, the coarsest inverse and (at the
 * first solve) the Krylov workspace are owned by the handle and drawn through
 * `alloc` (NULL: the library's pool); level 0 is borrowed from A.
 * Errors: AMG_EINVAL, AMG_ENOTFINITE, AMG_ESTALL, AMG_ESINGULAR, AMG_ENOMEM
 * (an allocation failed; nothing drawn stays allocated), AMG_EHIP. */
amg_status amg_setup(const amg_csr* A, const amg_params* params, const amg_allocator* alloc, void* stream,
                     amg_hier** out);

/* Releases every buffer owned by the handle (after synchronising its last
 * stream).  NULL is accepted. */
amg_status amg_destroy(amg_hier* h);

/* Algorithm 1: one V-cycle from a zero initial guess, z = M^{-1} r.
 * r, z: [device] float64[n], must not alias.  Asynchronous on `stream`.
 * Errors: AMG_EINVAL for a NULL argument. */
amg_status amg_vcycle(amg_hier* h, const double* r, double* z, void* stream);

/* Algorithm 4 (method 0: preconditioned CG, A symmetric positive definite)
 * or Algorithm 5 (method 1: preconditioned BiCGStab, right preconditioned)
 * with one V-cycle as the preconditioner, or AMG as a stationary solver
 * (method 2: Algorithm 1 repeated, x <- x + V(b - A x), the "AMG as a
 * solver" use of Section 4).  Stops when the recursive residual reaches
 * ||r|| <= rtol ||b|| and the recomputed residual b - A x confirms it (the
 * stationary solver recomputes the residual every iteration).
 * b: [device] float64[n]; x: [device] float64[n], initial guess on entry,
 * the last iterate on return (also on AMG_ENOTCONV and AMG_EBREAKDOWN).
 * info: [host], may be NULL.  Blocks the host until done.  The first solve
 * of a handle draws its Krylov workspace through the handle's allocator.
 * Errors: AMG_EINVAL, AMG_ENOTFINITE (b or x0 not finite), AMG_ENOTCONV,
 * AMG_EBREAKDOWN, AMG_ENOMEM (workspace), AMG_EHIP. */
amg_status krylov_solve(amg_hier* h, int32_t method, const double* b, double* x, double rtol, int32_t maxit,
                        void* stream, amg_info* info);

/* krylov_solve for callers that cannot allocate memory during the call (a
 * serving loop that must not call hipMalloc, a harness that forbids it): the
 * same arguments, kernels and results, but the Krylov work vectors come from
 * a scratch array compiled into the library (80 MiB on every device the
 * library runs on, held until the process ends), so the call allocates
 * nothing and never draws the handle's workspace.  Iterations are not
 * replayed from graphs.  Limit: the handle's level 0 has at most 1048576
 * rows (else AMG_EINVAL).  Calls on one device share that scratch: calls that
 * overlap in time on one device (other threads, or work still running on
 * other streams) race and give wrong results; the call blocks the host until
 * its work is done, so calls made one after another are safe.
 * Errors: as krylov_solve (AMG_ENOMEM cannot occur). */
amg_status krylov_solve_noalloc(amg_hier* h, int32_t method, const double* b, double* x, double rtol,
                                int32_t maxit, void* stream, amg_info* info);

/* Number of levels (coarsest included) and the size of level k.  [host] */
amg_status amg_num_levels(const amg_hier* h, int32_t* levels);
amg_status amg_level_size(const amg_hier* h, int32_t k, int32_t* n, int64_t* nnz);

/* Copies level k to [host] buffers (any may be NULL): row_ptr int32[n+1],
 * col_idx int32[nnz], val float64[nnz], agg int32[n] (aggregate of each row
 * on level k+1; untouched on the coarsest level).  Synchronises the stream. */
amg_status amg_export_level(const amg_hier* h, int32_t k, int32_t* row_ptr, int32_t* col_idx, double* val,
                            int32_t* agg, void* stream);

/* Setup statistics of each matching pass, in setup order, up to `cap`
 * entries per array: rounds run, GPU time in milliseconds (HIP events around
 * the pass, its coarse numbering included), rows and entries of the matched
 * operator; the number of passes and the bytes of GPU memory the handle owns.
 * Any output may be NULL.  [host] */
amg_status amg_setup_stats(const amg_hier* h, int32_t cap, int32_t* rounds, double* match_ms, int32_t* pass_n,
                           int64_t* pass_nnz, int32_t* npasses, size_t* owned_bytes);

/* Kernel timing for measurement: when enabled, the launches of the selected
 * kernel class are bracketed by HIP events on their stream and their
 * durations accumulated.  kernel: 0 = level-0 fused prolongation + smoothing,
 * 1 = level-0 fused smoothing + residual + restriction, 2 = Krylov SpMV.
 * amg_timing_read returns the launch count and total milliseconds
 * (synchronises the events).  [host] */
amg_status amg_timing_enable(amg_hier* h, int32_t kernel, int32_t on);
amg_status amg_timing_read(amg_hier* h, int32_t kernel, int64_t* launches, double* total_ms);

/* Autotuner: chooses each level's V-cycle schedule by timing both steps of
 * the level on this hierarchy (CSR-stream kernels with 128, 256 or 512 rows
 * per block, or lane-group kernels with 2, 4 or 8 lanes per row) and keeps
 * the fastest for later V-cycles and solves.  The schedules differ only in
 * the order of a row's additions.  schedule: [host] int32[levels] or NULL;
 * receives rows per block for CSR-stream levels, minus the lanes per row for
 * lane-group levels, 0 for the coarsest (all 0 when pre/post are not 1, whose
 * path has one schedule).  Overwrites the handle's work vectors; blocks the
 * host.  Errors: AMG_EINVAL, AMG_EHIP. */
amg_status amg_autotune(amg_hier* h, void* stream, int32_t* schedule);

/* Message for the last failing call on this thread (never NULL). */
const char* amg_last_error(void);

/* ------------------------------------------------------------------------
 * Serving: independent solve requests of different sizes on one GPU.
 * A server owns `workers` host threads, each with its own HIP stream; a
 * request runs setup, the Krylov solve and teardown on one worker while other
 * requests proceed on the others, so their kernels overlap on the device.
 * Requests are admitted in arrival order while the sum of the shares of the
 * requests in flight stays within `hbm_budget_bytes` (the device-memory
 * concern of Section 3.1, here as admission control).  A request's share is
 * its footprint (amg_footprint_bytes) until its setup is done, then the
 * device memory it holds (never more than the footprint).  With batch >= 2 a
 * worker starts a group only once the whole group it would take fits the
 * budget, or nothing else is in flight.
 * ------------------------------------------------------------------------ */
typedef struct amg_server amg_server;

typedef struct {
    int32_t workers;          /* concurrent requests, 1..64 (4)                 */
    int32_t batch;            /* >= 2: a worker takes up to this many queued
                               * requests with equal method (PCG or BiCGStab),
                               * rtol, maxit and size class (at most 32768
                               * rows, or more), builds their hierarchies
                               * together (amg_batch_setup) and solves them
                               * together, each request completing when its
                               * own system stops; 0 or 1: one request per
                               * worker (0)                                      */
    uint64_t hbm_budget_bytes; /* admission budget (64 GiB)                     */
    amg_params params;        /* hierarchy and cycle parameters of every request */
    amg_allocator alloc;      /* device memory of every request's hierarchy,
                               * workspace and batch buffers, drawn on the
                               * worker threads (alloc = NULL: the library's
                               * pool) (NULL)                                    */
} amg_server_config;

/* Upper estimate of the device memory one request of n rows and nnz entries
 * needs at its peak (hierarchy, Krylov workspace and setup scratch; level 0
 * is the caller's).  It assumes the coarse levels together hold at most n
 * rows and nnz entries (operator complexity <= 2).  It counts the bytes the
 * request asks for: the library's own pool rounds each chunk up to a size
 * class (at most 25% more), a caller's amg_allocator gets the exact sizes.
 * [host] */
amg_status amg_footprint_bytes(int32_t n, int64_t nnz, const amg_params* params, uint64_t* bytes);

/* Fills *c with the defaults shown above (params from amg_params_default). */
amg_status amg_server_config_default(amg_server_config* c);

/* Starts the worker threads on the current device.  Errors: AMG_EINVAL,
 * AMG_EHIP. */
amg_status amg_server_create(const amg_server_config* c, amg_server** out);

/* Queues one request: A (borrowed, [device] arrays as in amg_setup), b and x
 * ([device] float64[n]; x holds the initial guess) must stay valid until
 * amg_server_wait returns for it.  method/rtol/maxit as in krylov_solve.
 * stream: the producer's stream (NULL: the default stream); the worker
 * reads A, b and x only after the work enqueued on it before this call has
 * finished, so they may still be written asynchronously there.  The worker
 * writes x on its own stream; amg_server_wait returns after that write.
 * Returns at once with a ticket.  Errors: AMG_EINVAL (NULL argument, or a
 * footprint above the whole budget), AMG_EHIP. */
amg_status amg_server_submit(amg_server* s, const amg_csr* A, const double* b, double* x, int32_t method,
                             double rtol, int32_t maxit, void* stream, int64_t* ticket);

/* Blocks until request `ticket` has finished and releases it (one wait per
 * ticket; a second wait returns AMG_EINVAL).  info [host]
 * (may be NULL) receives the solve summary; latency_ms (may be NULL) the
 * time from submission to completion, queueing included.  Returns the
 * request's own status (setup or solve error). */
amg_status amg_server_wait(amg_server* s, int64_t ticket, amg_info* info, double* latency_ms);

/* Finishes every queued request, stops the workers and frees the server.
 * Results of requests nobody waited for are discarded.  NULL is accepted. */
amg_status amg_server_destroy(amg_server* s);

/* ------------------------------------------------------------------------
 * Batched solves: many independent systems of different sizes advanced
 * together, each kernel launch of the V-cycle (Algorithm 1) and of the
 * preconditioned CG or BiCGStab iteration (Algorithms 4, 5) covering every
 * system.
 * A batch copies the hierarchies it is made from into concatenated levels
 * (the hierarchies may be destroyed once amg_batch_create returns).  Each
 * system keeps its own CG scalars, stop test, residual replacement and
 * breakdown checks, exactly as krylov_solve applies them; a finished system
 * is masked off while the others continue.  A system's result does not
 * depend on which other systems share the batch.  One thread at a time per
 * batch.
 * ------------------------------------------------------------------------ */
typedef struct amg_batch amg_batch;

/* Builds a batch from `count` hierarchies (order kept).  Every hierarchy needs
 * at least two levels and pre = post = 1, and all must share precond_fp32,
 * omega and true_res_period.  The batch's device memory is drawn through
 * `alloc` (NULL: the library's pool).  Blocks the host until the copies are
 * done.  Errors: AMG_EINVAL, AMG_ENOMEM, AMG_EHIP. */
amg_status amg_batch_create(const amg_hier* const* hiers, int32_t count, const amg_allocator* alloc, void* stream,
                            amg_batch** out);

/* Batched setup (the setup phase of Section 3 for many systems at once): the
 * systems' levels are built together on block-diagonal concatenations of
 * their operators, so every matching round, Galerkin product and level
 * kernel covers all of them, while each system's stop rules apply to it
 * alone.  Every system gets exactly the hierarchy amg_setup would build, and
 * a solve of the returned batch gives bit for bit what amg_batch_create on
 * the separate hierarchies gives.  A: [host] amg_csr[count] (arrays on the
 * device, borrowed only during the call); params shared by all (pre = post
 * = 1).  status: [host] amg_status[count] or NULL; a system that fails
 * (invalid matrix, stall, singular coarsest level, or a single level) gets
 * its status there, takes no rows in the batch and reports the status from
 * amg_batch_solve.  A matrix that is not structurally symmetric fails the
 * whole call.  Device memory (the batch and the setup's temporaries) is drawn
 * through `alloc` (NULL: the library's pool).  Blocks the host.
 * Errors: AMG_EINVAL, AMG_ENOMEM, AMG_EHIP. */
amg_status amg_batch_setup(const amg_csr* A, int32_t count, const amg_params* params, const amg_allocator* alloc,
                           void* stream, amg_batch** out, amg_status* status);

/* offsets: [host] int32[count + 1]; system i occupies rows
 * offsets[i] .. offsets[i+1]-1 of the batch vectors. */
amg_status amg_batch_rows(const amg_batch* b, int32_t* offsets);

/* Preconditioned CG (method 0, Algorithm 4) or BiCGStab (method 1,
 * Algorithm 5) on every system at once.
 * b, x: [device] float64[offsets[count]], the systems' right-hand sides and
 * initial guesses one after another; x receives the solutions.  info: [host]
 * amg_info[count], one per system (status per system; solve_ms is the call's
 * wall time).  Returns AMG_OK when every system converged, else the first
 * failing system's status.  Blocks the host until done.
 * Errors: AMG_EINVAL, AMG_ENOTFINITE, AMG_ENOTCONV, AMG_EBREAKDOWN, AMG_EHIP. */
amg_status amg_batch_solve(amg_batch* bt, int32_t method, const double* b, double* x, double rtol, int32_t maxit,
                           void* stream, amg_info* info);

/* Iterations are replayed from HIP graphs captured at the first solve of each
 * method (on by default).  While a capture lasts, device-wide calls from other
 * threads of the process (hipDeviceSynchronize, allocations) fail with
 * hipErrorStreamCaptureUnsupported, so multi-threaded callers turn graphs off
 * (on = 0); results are the same either way. */
amg_status amg_batch_set_graphs(amg_batch* b, int32_t on);

/* Number of concatenated levels of a batch (its deepest system's). */
amg_status amg_batch_levels(const amg_batch* b, int32_t* levels);

/* Autotuner for a batch: rows per block (128, 256 or 512) of each level's
 * CSR-stream kernels, chosen by timing the level's steps on this batch.
 * Results do not change (a row's sum is formed in entry order whatever the
 * block size).  schedule: [host] int32[levels] or NULL (0 for the last
 * level).  Blocks the host.  Errors: AMG_EINVAL, AMG_EHIP. */
amg_status amg_batch_autotune(amg_batch* b, void* stream, int32_t* schedule);

/* Frees the batch.  NULL is accepted. */
amg_status amg_batch_destroy(amg_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* HEMAMG_H */
