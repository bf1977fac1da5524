/*
 * mesh_sdd.h -- C-ABI of the MI355X interface-node Monte-Carlo solver for
 * stochastic domain decomposition of the parabolic mesh generator
 * (Bihlo, Haynes & Walsh, arXiv:1504.00084).
 *
 * Problem solved per call (paper section 3.4-3.6): given the mesh density
 * rho frozen at t^n (section 3.2, MP linearisation), the mesh (x^n, y^n) and
 * the boundary data at t^n and t^{n+1}, estimate (x, y) at t^{n+1} at every
 * artificial subdomain-interface node of the computational grid, by N
 * independent Euler-Maruyama paths of K substeps of the SDE
 *     dPhi = (grad rho / rho) dt + sqrt(2) dW          (eq. ...SolutionB)
 * started at the node and run over one mesh step tau.  A path that leaves a
 * Dirichlet side (endpoint outside, or Brownian-bridge crossing inside a
 * substep) takes the boundary value there (eq. ...SolutionA, second term);
 * a survivor takes the bicubic interpolant of the mesh at t^n at its final
 * position (first term; periodic problems: eq. StochasticSolutionPeriodic...).
 * Periodic axes wrap the path and add the winding w*L (quasi-periodic mesh,
 * section 2).  The estimate is the arithmetic mean over the N paths; the
 * standard error uses the unbiased variance (sums kept in FP64).
 *
 * Conventions
 *   - Every function returns a status: MESH_SDD_OK (0), MESH_SDD_PENDING (1)
 *     or a negative error.  No exception crosses the ABI.  The text of the
 *     last error of the calling thread is returned by mesh_sdd_last_error().
 *   - Arrays are row-major [n_eta][n_xi] doubles (index j*n_xi + i), node
 *     (i, j) sitting at computational coordinates (i/(n_xi-1), j/(n_eta-1)).
 *     A periodic axis has n nodes of which node n-1 is the image of node 0
 *     (its values are ignored; x(xi + 1) = x(xi) + Lx, y(eta + 1) = y + Ly).
 *   - Boundary arrays hold, in this order, side 0 (xi = 0) x then y, side 1
 *     (xi = 1) x then y -- n_eta values each -- then side 2 (eta = 0) x then
 *     y, side 3 (eta = 1) x then y -- n_xi values each: 4*n_eta + 4*n_xi
 *     doubles.  Sides normal to a periodic axis are ignored.
 *   - Interface nodes (section 3.5): node (i, j) with i a multiple of
 *     (n_xi-1)/sub_xi or j a multiple of (n_eta-1)/sub_eta, not on a
 *     Dirichlet side; on a periodic axis the seam (index 0) is an interface.
 *     Order: row-major in (j, i).  Results are indexed by this rank.
 *   - Random numbers: path p of interface node r owns the word stream w_q =
 *     word (q mod 4) of Philox4x32-10 with counter
 *     (q div 4, p, r, instance_id << 16 | (mesh_step & 0xffff)) and key
 *     (seed low 32 bits, seed high 32 bits); substep k uses w_{3k}, w_{3k+1}
 *     (Box-Muller normals, uniforms ((w >> 9) + 1/2) 2^-23) and w_{3k+2}
 *     (bridge uniform).  A result is therefore a pure function of the inputs,
 *     the seed, instance_id and mesh_step: it is the same whether the
 *     request runs alone or batched with others.
 *   - Ownership: inputs are caller-owned and are copied before the call
 *     returns (submit included), so the caller may free or reuse them at
 *     once.  Device tables, meshes and partial sums are library-owned and
 *     stay resident until mesh_sdd_destroy.  Result arrays are caller-owned
 *     and are written by mesh_sdd_solve_interfaces / mesh_sdd_solve_batch, or
 *     by the mesh_sdd_poll that returns MESH_SDD_OK.
 *   - Threading: a context is safe for concurrent submit/poll from several
 *     threads.  One instance must not be used from two threads at once.
 *   - Device pointers are HIP device addresses on the context's device.  Data
 *     behind device input pointers must be complete when the call is made
 *     (written on the context's stream, or the writer's stream synchronised).
 */
#ifndef MESH_SDD_H
#define MESH_SDD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mesh_sdd_ctx mesh_sdd_ctx; /* device, stream, HBM budget, queue, tuning cache */
typedef struct mesh_sdd mesh_sdd;         /* one problem instance with its resident tables  */
typedef uint64_t mesh_sdd_ticket;

enum {
    MESH_SDD_OK = 0,
    MESH_SDD_PENDING = 1,
    MESH_SDD_E_INVAL = -1,     /* bad argument or descriptor                  */
    MESH_SDD_E_NOMEM = -2,     /* device or host allocation failed            */
    MESH_SDD_E_BUDGET = -3,    /* one request alone exceeds the HBM budget    */
    MESH_SDD_E_DEVICE = -4,    /* a HIP call failed                           */
    MESH_SDD_E_STATE = -5,     /* call out of order (e.g. solve before monitor) */
    MESH_SDD_E_CANCELLED = -6  /* request cancelled or context destroyed      */
};

enum { MESH_SDD_FP32 = 0, MESH_SDD_FP64 = 1 };

/* Problem instance.  struct_size must be sizeof(mesh_sdd_desc). */
typedef struct {
    uint32_t struct_size;
    int32_t n_xi, n_eta;             /* grid nodes per axis, >= 4                    */
    int32_t sub_xi, sub_eta;         /* subdomains per axis, (n-1) % sub == 0        */
    int32_t periodic_xi, periodic_eta;
    int32_t K;                       /* Euler-Maruyama substeps per mesh step, >= 1  */
    double Lx, Ly;                   /* physical extents, > 0                        */
    double tau;                      /* mesh time step Delta t, > 0                  */
    int32_t precision;               /* MESH_SDD_FP32: batched FP32 paths with FP64
                                        sums; MESH_SDD_FP64: plain FP64 path         */
    int32_t bridge;                  /* 1: Brownian-bridge test (section 3.4)        */
    uint64_t seed;                   /* Philox key                                   */
    uint32_t instance_id;            /* request-owned RNG identity, < 65536          */
    uint32_t reserved;
} mesh_sdd_desc;

/* One mesh step.  struct_size must be sizeof(mesh_sdd_step). */
typedef struct {
    uint32_t struct_size;
    int32_t inputs_on_device;        /* 1: the four pointers below are device ptrs   */
    const double *x_cur, *y_cur;     /* mesh at t^n, [n_eta][n_xi]                   */
    const double *bnd_t0, *bnd_t1;   /* boundary arrays at t^n and t^{n+1}; pass the
                                        same pointer twice if only one level exists */
    int64_t paths_per_node;          /* 1 <= N <= 2^31; ignored when target_se > 0   */
    double target_se;                /* > 0: N = min(max_paths, ceil(2 tau L^2/se^2)) */
    int64_t max_paths;               /* cap for target_se (0: 1e6)                   */
    uint32_t mesh_step;              /* enters the RNG counter (low 16 bits)         */
    uint32_t interface_stride;       /* 0 or 1: every interface node runs paths.
                                        s > 1 (section 3.6, subsampled interface):
                                        on each interface line only the nodes at
                                        multiples of s along the line run paths
                                        (line crossings always do); every other
                                        interface node takes the Keys cubic
                                        interpolant (a = -1/2) along its line of
                                        those estimates, of the boundary values at
                                        t^{n+1} where the line meets a Dirichlet side
                                        (Keys' end rule beyond it) and of the
                                        periodic images (plus the period) across a
                                        seam; its se is that of the same linear
                                        combination of independent estimates, its
                                        exit_frac NaN.  A node that runs paths keeps
                                        its own random stream, so its results equal
                                        those of the full run bit for bit.  s must
                                        divide (n_xi-1)/sub_xi and (n_eta-1)/sub_eta
                                        and leave >= 2 segments per grid line
                                        ((n-1)/s >= 2 on both axes): E_INVAL
                                        otherwise.  executed_path_steps counts the
                                        sampled nodes' paths only.                */
} mesh_sdd_step;

/* Per-node results, caller-owned arrays of length M (interface-node count). */
typedef struct {
    uint32_t struct_size;
    int32_t outputs_on_device;       /* 1: the five pointers are device ptrs         */
    double *mean_x, *mean_y;         /* estimate of (x, y) at t^{n+1}                */
    double *se_x, *se_y;             /* standard error (NaN when N == 1)             */
    double *exit_frac;               /* fraction of paths that left the domain       */
    uint64_t executed_path_steps;    /* out: EM substeps actually executed           */
    int64_t paths_per_node;          /* out: N used                                  */
    double device_ms;                /* out: path + finalize kernel time             */
} mesh_sdd_result;

/* Serving statistics of a context (mesh_sdd_ctx_stats). */
typedef struct {
    uint32_t struct_size;
    uint32_t reserved;
    uint64_t submitted, completed, failed, cancelled;
    uint64_t queued, running;        /* requests waiting / admitted now              */
    uint64_t ticks;                  /* persistent launches issued by the scheduler  */
    uint64_t hbm_in_use, hbm_budget; /* bytes admitted / allowed                     */
    double p50_ms, p99_ms, mean_ms;  /* submit-to-completion latency of completed    */
    double busy_ms;                  /* device time of all ticks                     */
    uint64_t executed_path_steps;    /* summed over completed requests               */
} mesh_sdd_stats;

/* Launch shape of the batched FP32 kernels of the section 3.4 solve (chosen
 * by the autotuner or set).  Only chunk_paths changes results (it sets how
 * the paths of a node are grouped into FP64 partial sums); every other
 * field changes speed only.  0 in an int field below means its default. */
typedef struct {
    uint32_t struct_size;
    int32_t block;                   /* cell-record kernel (monitor_table = 1) only:
                                        threads per workgroup (64, 128, 256, 512)    */
    int32_t waves_per_simd;          /* cell-record kernel only: residency (1..8)    */
    int32_t chunk_paths;             /* paths per work item (multiple of 64, 64..2048;
                                        default 128)                                 */
    int32_t monitor_table;           /* 0: automatic -- a launch that holds one
                                        instance whose FP32 node tables of rho and
                                        dt rho_xi fit the LDS (8 B per node) stages
                                        them whole; any other launch (several
                                        instances, or a larger grid) stages
                                        windows of them (and, on most grids, of
                                        dt rho_eta per node too) around
                                        blocks of interface nodes, and paths that
                                        leave a window read the cell records
                                        (1024-thread workgroups, item end states in
                                        a context buffer; identical results); 1:
                                        always from the cell records in L2          */
    int32_t table_level;             /* out (mesh_sdd_get_launch): how a launch
                                        holding this instance alone reads the
                                        tables: 0 cell records, 2 whole node tables
                                        in LDS, 3 windows in LDS.  Ignored by
                                        mesh_sdd_set_launch.                         */
    int32_t refill_lanes;            /* LDS kernels: a wave leaves its stepping loop
                                        for the lane refill once fewer than this
                                        many of its 64 lanes have a path in flight
                                        (1..64; default 56)                          */
    int32_t max_quarters;            /* LDS kernels: ... or after this many groups
                                        of four substeps (1..64; default 16)         */
    int32_t window_kind;             /* windowed kernel, grids whose tables the LDS
                                        cannot hold whole: 1 two-field windows (rho,
                                        dt rho_xi per node, up to 140 x 140 nodes),
                                        2 three-field windows (also dt rho_eta per
                                        node, 12 B per node, up to 114 x 114);
                                        default: three-field below 400 nodes per
                                        axis, two-field above.  A window that holds
                                        the whole grid is always used.               */
    int32_t window_margin;           /* window nodes beyond a block on each side
                                        (default 45 two-field, 30 three-field); the
                                        block is the window less twice the margin
                                        (at least 1 node): a wider margin keeps more
                                        paths inside, at more window refills         */
    int32_t job_split;               /* windowed kernel: a job holds at most 1/job_split
                                        of a workgroup's share of the launch's items
                                        (1..4096; default 32, and 256 on grids cut
                                        into several two-field windows)              */
} mesh_sdd_launch;

/* ---- context ------------------------------------------------------------ */

/* Execution context of the interface solves of section 3.4 (no paper
 * counterpart: device, stream, serving queue).
 * Create a context on HIP device `device`.  hbm_budget_bytes caps the device
 * memory of admitted requests (0: 90% of the free memory).  hip_stream: a
 * hipStream_t to launch on (NULL: the context creates its own, default
 * priority).  Starts the serving scheduler thread.  Errors: E_INVAL,
 * E_DEVICE, E_NOMEM. */
int mesh_sdd_ctx_create(int device, size_t hbm_budget_bytes, void *hip_stream, mesh_sdd_ctx **out);

/* Stop the scheduler (pending requests end with E_CANCELLED), free
 * everything the context owns.  Instances must be destroyed first
 * (E_STATE otherwise). */
int mesh_sdd_ctx_destroy(mesh_sdd_ctx *ctx);

/* Counters and latency percentiles of the serving loop (no paper
 * counterpart; the requests are section 3.4 interface solves). */
int mesh_sdd_ctx_stats(mesh_sdd_ctx *ctx, mesh_sdd_stats *out);

/* Fix the launch shape of the batched kernel of the section 3.4 solve
 * (overrides the autotuner for every later launch; results do not depend on
 * it except through chunk_paths, which sets the grouping of the FP64 sums);
 * NULL restores the tuned or default shapes.  E_INVAL on a field outside
 * its range. */
int mesh_sdd_set_launch(mesh_sdd_ctx *ctx, const mesh_sdd_launch *launch);

/* Launch shape that the next section 3.4 launch over `inst` alone would use
 * (defaults filled in). */
int mesh_sdd_get_launch(mesh_sdd *inst, mesh_sdd_launch *out);

/* Autotune the FP32 kernels for the shape bucket of `inst` (grid size and
 * periodicity): times launches of `inst` alone on a reduced path count of
 * `step` (about 6e9 path-steps each) and searches, one knob at a time, over
 * chunk_paths {64, 128, 256}, window_kind and window_margin (windowed grids
 * only), job_split {8, 32, 128, 256, 1024}, refill_lanes {48, 56, 60} and
 * max_quarters {8, 16, 32}.  The winner is kept in the context for every
 * later launch of that bucket alone (and for the per-instance knobs,
 * chunk_paths, window_kind and window_margin, inside batches and serving
 * ticks too).  Writes it to *out if non-NULL. */
int mesh_sdd_autotune(mesh_sdd *inst, const mesh_sdd_step *step, mesh_sdd_launch *out);

/* Autotune for a batch: first each distinct shape bucket of `insts` (as
 * mesh_sdd_autotune, on the first instance of the bucket), then the
 * launch-wide knobs of a multi-instance launch (job_split, refill_lanes,
 * max_quarters) by timing the whole batch at 1/scale_down of every step's
 * path count (at least 64 paths), then, timed the same way, each bucket's
 * chunk_paths {64, 128, 256} and, for grids no window holds whole, its
 * window_margin {default, 30, 38, 45} (a bucket tuned alone can prefer a
 * shape that the batch does not).  The launch-wide winner is kept for every
 * later launch of several instances (mesh_sdd_solve_batch, serving ticks)
 * and written to *out if non-NULL; the bucket knobs replace the buckets'.
 * All FP32. */
int mesh_sdd_autotune_batch(mesh_sdd *const *insts, const mesh_sdd_step *steps, int32_t count, int32_t scale_down,
                            mesh_sdd_launch *out);

/* Write the context's tuned shapes (per bucket and for multi-instance
 * launches) to a text file, one line each; mesh_sdd_tune_load reads such a
 * file back into a context (replacing its entries of the same keys).
 * E_INVAL on a file that cannot be written or parsed. */
int mesh_sdd_tune_save(mesh_sdd_ctx *ctx, const char *path);
int mesh_sdd_tune_load(mesh_sdd_ctx *ctx, const char *path);

/* ---- host-only helpers (no device needed) --------------------------------- */

/* Validate a descriptor (grid and partition of section 3.5, step of section
 * 3.4) without creating anything: MESH_SDD_OK or E_INVAL with the reason in
 * mesh_sdd_last_error(). */
int mesh_sdd_desc_check(const mesh_sdd_desc *desc);

/* Interface nodes of a descriptor's partition (section 3.5): returns M >= 0
 * (or a negative error) and, when i and j are not NULL, writes the nodes in
 * rank order into caller arrays of length M. */
int mesh_sdd_desc_interface_nodes(const mesh_sdd_desc *desc, int32_t *i, int32_t *j);

/* Work order of the FP32 kernels for a descriptor and an interface stride
 * (0 or 1: every interface node; else the sampling of section 3.6, with the
 * same validation as mesh_sdd_step.interface_stride).  The nodes that run
 * paths are stepped block by block (blocks in Z order, ranks ascending inside
 * a block); each block has the window of the monitor tables that the
 * windowed kernel stages in LDS around it, clamped to the grid, the whole
 * axis where it fits.  Kind 0: windows of (rho, dt rho_xi) per node, at
 * most 140 x 140 nodes, blocks of 50 nodes, 45 nodes of margin; kind 1:
 * windows that also hold dt rho_eta per node, 114 x 114 nodes when square,
 * blocks of 54 nodes, 30 nodes of margin.  Kind 1 where
 * its window holds the whole grid, else kind 0 where that one does, else
 * kind 1 for grids under 400 nodes per axis and kind 0 above.  The order changes no result.  Returns the
 * number of nodes Ms >= 0 or a negative error.  When `ranks` is not NULL,
 * writes the Ms interface ranks in work order (caller array of length Ms).
 * When `n_blocks` is not NULL, writes the block count there; when `blocks`
 * is not NULL too, writes one record of seven int32 per block -- first
 * position, end position, window i0, j0, width, height, kind -- into caller
 * room for max_blocks records (E_INVAL if that is too small).  Host only: no
 * device is touched. */
int mesh_sdd_desc_work_order(const mesh_sdd_desc *desc, uint32_t interface_stride, int32_t *ranks, int32_t *blocks,
                             int32_t max_blocks, int32_t *n_blocks);

/* ---- instances ----------------------------------------------------------- */

/* One problem instance: the computational grid and its s_xi x s_eta
 * subdomain partition (section 3.5), the mesh step tau and its K substeps
 * (section 3.4), the periodic axes (section 3.3) and the RNG identity.
 * Validate the descriptor (n >= 4, (n-1) % sub == 0, sub >= 1, K >= 1,
 * tau > 0, L > 0, instance_id < 65536, precision in {FP32, FP64}) and
 * allocate the instance's resident device buffers.  E_INVAL, E_NOMEM,
 * E_BUDGET (the instance alone exceeds the context's budget). */
int mesh_sdd_create(mesh_sdd_ctx *ctx, const mesh_sdd_desc *desc, mesh_sdd **out);

/* Free an instance (the resident tables of the monitor frozen for section
 * 3.4) and its device buffers.  E_STATE if it has requests in flight. */
int mesh_sdd_destroy(mesh_sdd *inst);

/* Freeze the monitor for the next solves (section 3.2): rho is
 * [n_eta][n_xi] doubles, > 0, host (is_device_ptr = 0) or device memory.
 * Builds the finite-difference gradient table on the device (section 3.4).
 * E_INVAL on a null pointer or a non-positive / non-finite value (host
 * input only; device input is not inspected). */
int mesh_sdd_set_monitor(mesh_sdd *inst, const double *rho, int is_device_ptr);

/* Number M of artificial interface nodes of the instance's partition
 * (paper section 3.5: the nodes where the subdomains' Dirichlet data are
 * estimated; the rule is stated in the conventions above), >= 0, or a
 * negative error. */
int mesh_sdd_num_interface_nodes(const mesh_sdd *inst);

/* Write the interface nodes (i, j) of section 3.5 in rank order (row-major
 * in (j, i)) into caller arrays of length M (host memory).  E_INVAL on a
 * NULL instance or, when M > 0, a NULL array. */
int mesh_sdd_interface_nodes(const mesh_sdd *inst, int32_t *i, int32_t *j);

/* ---- solving -------------------------------------------------------------- */

/* Blocking solve of one mesh step (paper section 3.4: N Euler-Maruyama paths
 * of K substeps of eq. WinslowGeneratorSDEDiscretization per interface node,
 * bilinear monitor, Brownian-bridge exit test, bicubic terminal value; the
 * estimator of eq. WinslowGeneratorRelaxedStochasticSolutionA, section 3.2,
 * or eq. StochasticSolutionPeriodicDomainSolution, section 3.3, on periodic
 * axes; mean over the N paths).  Results as mesh_sdd_result describes; the
 * FP32 kernel matches the FP64 oracle to 1e-5 per node (unit square) where
 * the substep resolves the drift (dt |grad b| well below 0.1, as with K =
 * 500 on the benchmark grids); with longer substeps the FP32 and FP64 paths
 * separate and the FP32 estimate agrees with the FP64 one statistically
 * (within 3 combined standard errors), not path by path.  E_STATE before set_monitor; E_INVAL on
 * a bad step (null pointers, N outside [1, 2^31], corner values of the
 * boundary arrays that disagree by more than 1e-12 (Lx + Ly), host inputs
 * that are not finite) and on a request too large for 32-bit work-item
 * numbers: FP32, more than 2^32 - 2^20 (node, path-chunk) items (nodes that
 * run paths x ceil(N / chunk_paths)); FP64, 2^24 or more (node, 256-path
 * block) pairs.  Nothing is allocated or launched for such a request. */
int mesh_sdd_solve_interfaces(mesh_sdd *inst, const mesh_sdd_step *step, mesh_sdd_result *result);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the same
 * solve as mesh_sdd_solve_interfaces (same kernels, same chunk plan, so the
 * same result bits), but every per-call device buffer (staged mesh and
 * boundary copies, padded meshes, partial sums, queue counters, job list,
 * end-state buffer, results before their copy-out) is carved from one static
 * device array of the library, 64 MiB per device, instead of being
 * allocated.  The call makes no hipMalloc / hipFree and uses no allocating
 * library routine; the instance's tables (mesh_sdd_create, set_monitor) are
 * its inputs.  Inputs and outputs must be device pointers
 * (step->inputs_on_device = 1, result->outputs_on_device = 1; E_INVAL
 * otherwise).  A solve that needs more than 64 MiB of scratch is refused
 * with E_INVAL before any work (e.g. 129^2 with 4x4 subdomains fits up to
 * about 1.9e5 paths per node at the default chunk of 128 paths); an interface
 * stride > 1 must have been used by an allocating solve of the instance
 * first (its node lists are built then; E_STATE otherwise).  Every call on
 * a device shares that device's array, which keeps the last call's contents
 * (whatever must start at zero is cleared by a fill kernel each call); calls
 * on one device are serialised by a process-wide lock, and a call blocks
 * until its results are in the output arrays.  Errors otherwise as
 * mesh_sdd_solve_interfaces. */
int mesh_sdd_solve_interfaces_noalloc(mesh_sdd *inst, const mesh_sdd_step *step, mesh_sdd_result *result);

/* Blocking solve of `count` instances (each as mesh_sdd_solve_interfaces,
 * section 3.4): all FP32 instances run in ONE
 * persistent launch over a shared (instance, node, path-chunk) work queue
 * (several launches, in order, where their items together exceed
 * 2^32 - 2^20); FP64 instances run one launch each.  Per-instance status codes go to
 * status[] (may be NULL); the return value is the first error or OK. */
int mesh_sdd_solve_batch(mesh_sdd *const *insts, const mesh_sdd_step *steps, mesh_sdd_result *results,
                         int32_t count, int32_t *status);

/* Non-blocking interface solve (section 3.4, as mesh_sdd_solve_interfaces):
 * snapshot the step's inputs and queue a request.  The
 * scheduler admits requests while the HBM in use plus the request's cost
 * stays within the budget, and runs all admitted requests' pending chunks
 * in persistent launches ("ticks"); a request that arrives while a tick is
 * running joins the next tick (continuous batching at chunk granularity).
 * E_BUDGET only if the request alone exceeds the budget. */
int mesh_sdd_submit(mesh_sdd *inst, const mesh_sdd_step *step, mesh_sdd_ticket *ticket);

/* Result of a submitted interface solve (section 3.4).
 * MESH_SDD_PENDING while the request runs; MESH_SDD_OK once done (the
 * result arrays given here are filled, the ticket is released); a negative
 * error if it failed (ticket released).  E_INVAL for an unknown ticket. */
int mesh_sdd_poll(mesh_sdd_ctx *ctx, mesh_sdd_ticket ticket, mesh_sdd_result *result);

/* Like poll (section 3.4 solve) but waits up to timeout_ms (< 0: forever)
 * for completion. */
int mesh_sdd_wait(mesh_sdd_ctx *ctx, mesh_sdd_ticket ticket, mesh_sdd_result *result, int64_t timeout_ms);

/* Cancel a queued interface solve (section 3.4) that has not been admitted
 * yet: it ends with E_CANCELLED.  E_STATE if it is already running or
 * finished, E_INVAL for an unknown ticket. */
int mesh_sdd_cancel(mesh_sdd_ctx *ctx, mesh_sdd_ticket ticket);

/* ---- the mesh step around the interface estimate (sections 2, 3.5-3.7) ------ */

/* Options of the deterministic parts of a mesh step (all FP64). */
typedef struct {
    uint32_t struct_size;
    int32_t fe_substeps;             /* forward-Euler steps over tau of the 2-D solves;
                                        0: the smallest L with tau / L <= fe_cfl /
                                        (2 / h_xi^2 + 2 / h_eta^2)                    */
    int32_t edge_substeps;           /* same for the 1-D edge generator (limit h^2/2)  */
    int32_t edge_generator;          /* mesh_sdd_mp_step only: 1 = tangential boundary
                                        values at t^{n+1} from the 1-D generator,
                                        0 = taken from step->bnd_t1                    */
    int32_t solver;                  /* subdomain solves: 0 automatic, 1 each subdomain
                                        resident in LDS (E_INVAL if one does not fit:
                                        at most 4096 interior nodes), 2 whole-grid
                                        sweeps in global memory                        */
    int32_t reserved;                /* must be 0                                      */
    double fe_cfl;                   /* fraction of the stability limit, (0, 1];
                                        0 means 0.9                                    */
} mesh_sdd_mp_opts;

/* Tangential boundary values at t^{n+1} (section 2): on every physical side
 * the component along the side follows the one-dimensional form of the
 * generator, v_t = (rho_s / rho) v_s + v_ss, with the monitor frozen at t^n
 * (the instance's table: set_monitor first), the end values fixed on a
 * Dirichlet axis and wrapped with the period on a periodic one; forward Euler
 * with centred differences.  Normal components, and the sides normal to a
 * periodic axis, are copied.  bnd_cur, bnd_new: boundary arrays in the layout
 * above (may be the same array), host or device memory (pointers_on_device).
 * E_STATE before set_monitor; E_INVAL on null pointers or bad options. */
int mesh_sdd_edge_generate(mesh_sdd *inst, const double *bnd_cur, double *bnd_new, const mesh_sdd_mp_opts *opts,
                           int pointers_on_device);

/* Subdomain solves (section 3.5): each subdomain of the partition is a
 * Dirichlet problem of eq. (Gen) with the monitor frozen at t^n, integrated
 * over tau from the mesh at t^n (x_cur, y_cur) by forward Euler with centred
 * differences.  Dirichlet data move linearly in time from the mesh at t^n to
 * their values at t^{n+1}: interface nodes take iface_x / iface_y (length M,
 * rank order, e.g. a result's mean_x / mean_y), physical-boundary nodes the
 * boundary arrays bnd_new, the images of a periodic seam their original plus
 * the period.  Writes the new mesh x_new, y_new ([n_eta][n_xi]; must not
 * alias the inputs).  Host or device memory (pointers_on_device).
 * E_STATE before set_monitor; E_INVAL on null pointers or bad options. */
int mesh_sdd_subdomain_solve(mesh_sdd *inst, const double *x_cur, const double *y_cur, const double *bnd_new,
                             const double *iface_x, const double *iface_y, double *x_new, double *y_new,
                             const mesh_sdd_mp_opts *opts, int pointers_on_device);

/* Single-domain reference of the same step (section 3.7): as
 * mesh_sdd_subdomain_solve without interfaces (Dirichlet data on the physical
 * boundary only; periodic axes wrap).  Always runs whole-grid sweeps. */
int mesh_sdd_single_domain_solve(mesh_sdd *inst, const double *x_cur, const double *y_cur, const double *bnd_new,
                                 double *x_new, double *y_new, const mesh_sdd_mp_opts *opts, int pointers_on_device);

/* One mesh step (sections 3.4-3.6): the boundary arrays at t^{n+1} (edge
 * generator, or step->bnd_t1), the interface estimate with the boundary data
 * moving from step->bnd_t0 to them (as mesh_sdd_solve_interfaces), then the
 * subdomain solves.  Writes the new mesh (x_new, y_new), the new boundary
 * arrays (bnd_new) and the interface estimate (result).  Inputs follow
 * step->inputs_on_device, outputs result->outputs_on_device.  Blocking.
 * Errors as the calls it is made of. */
int mesh_sdd_mp_step(mesh_sdd *inst, const mesh_sdd_step *step, const mesh_sdd_mp_opts *opts, double *x_new,
                     double *y_new, double *bnd_new, mesh_sdd_result *result);

/* Monitor of the next step from the solution on the new mesh (section 3.6):
 * rho = sqrt(1 + a |grad u|^2) at every node, u, x, y nodal [n_eta][n_xi];
 * grad u in physical coordinates from centred computational differences
 * (one-sided second order at Dirichlet edges; wrapped, with the period added
 * to the winding coordinate, on periodic axes) through the inverse mesh
 * Jacobian; a = alpha, or alpha / max |grad u|^2 when normalize != 0.
 * Installs rho as mesh_sdd_set_monitor does.  E_INVAL if alpha is negative
 * or not finite, or if |grad u| is not finite somewhere (vanishing mesh
 * Jacobian); E_STATE with requests in flight. */
int mesh_sdd_set_monitor_arclength(mesh_sdd *inst, const double *u, const double *x, const double *y, double alpha,
                                   int normalize, int pointers_on_device);

/* Copy the frozen monitor rho ([n_eta][n_xi], as installed) into rho_out
 * (host or device memory).  E_STATE before set_monitor. */
int mesh_sdd_get_monitor(mesh_sdd *inst, double *rho_out, int pointer_on_device);

/* Geometric mesh quality (section 3.7, eq. Q): Q(K) = tr(J^T J) / (2 |det J|)
 * per cell K, J the Jacobian of the bilinear cell map at the cell centre
 * (computational spacing 1/(n-1)); R(K) = Q_SD(K) / Q_SDD(K) of a
 * single-domain mesh (x_sd, y_sd) and a decomposed one (x_dd, y_dd) on the
 * instance's grid.  Writes *r_max and *r_mean (host) and, when r_cells is not
 * NULL, R per cell [(n_eta - 1)][(n_xi - 1)] (memory kind as the meshes).
 * E_INVAL on null pointers or a degenerate cell (R not finite). */
int mesh_sdd_mesh_quality(mesh_sdd *inst, const double *x_sd, const double *y_sd, const double *x_dd,
                          const double *y_dd, double *r_cells, double *r_max, double *r_mean,
                          int pointers_on_device);

/* Monitor transfer of the MᵏP variant (section 5: the monitor of each
 * sub-step is the piecewise-linear interpolant of (x^n, rho^n) at the nodes
 * of the current sub-mesh).  f_new [n_eta][n_xi] at the nodes (x_new, y_new)
 * from the nodal values f_old on the mesh (x_old, y_old), all on the
 * instance's grid: every old cell (i, j)-(i+1, j+1) is split along its
 * diagonal from node (i, j) to node (i+1, j+1); a new node takes the linear
 * interpolant of the triangle that contains it, or, outside the old mesh,
 * the linear extension of the triangle whose smallest barycentric coordinate
 * is largest.  Periodic axes extend the old mesh by its images (x + Lx along
 * xi, y + Ly along eta, f unchanged); image nodes of f_new take node 0's
 * value.  All six arrays are host or all device memory (pointers_on_device);
 * f_new must not alias an input.  Blocking.  Does not change the installed
 * monitor (pass f_new to mesh_sdd_set_monitor for that).  E_INVAL on null
 * pointers or non-finite host inputs. */
int mesh_sdd_transfer_field(mesh_sdd *inst, const double *x_old, const double *y_old, const double *f_old,
                            const double *x_new, const double *y_new, double *f_new, int pointers_on_device);

/* ---- diagnostics ----------------------------------------------------------- */

/* Per-path outcomes of interface node `node_rank`, paths [p_begin, p_end),
 * run by the instance's own path kernel arithmetic (FP32 or FP64) one path
 * per lane: value (vx, vy), exit flag, exit side (-1: survived) and
 * executed substeps.  If trace != NULL it receives, per path and substep,
 * (xi, eta, n1, n2) after the wrap and before any exit projection
 * ([p][K][4] doubles; entries after an exit are left as they were).
 * Host arrays.  For checking the path arithmetic on tiny cases. */
int mesh_sdd_debug_paths(mesh_sdd *inst, const mesh_sdd_step *step, int32_t node_rank, int64_t p_begin,
                         int64_t p_end, double *vx, double *vy, int32_t *exited, int32_t *side,
                         int32_t *steps, double *trace);

/* Text of the last error on the calling thread ("" if none); no paper
 * counterpart. */
const char *mesh_sdd_last_error(void);

/* Library version string (no paper counterpart). */
const char *mesh_sdd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MESH_SDD_H */
