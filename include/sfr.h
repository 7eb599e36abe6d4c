/*
 * sfr.h -- C ABI of the MI355X (gfx950) sparse fixed-rank decomposition
 * library: M = L + S with rank(L) = r and L kept as U B V^T (U in St_{m,r},
 * B in SPD_r, V in St_{n,r}), computed by FR-ADM (Alg. 1) with the
 * FixedRankOptStep L-step (Alg. 2) and its Nystrom variant FR-Nys (Alg. 3)
 * of Ros et al., "Fast and Robust Fixed-Rank Matrix Recovery".
 *
 * The problem solved is eq. (1), min ||S||_1 s.t. M = L + S, rank(L) = r,
 * through the augmented Lagrangian of eq. (4) with an l1 weight lambda
 * (lambda = 1 is the paper's literal form; lambda only rescales the penalty
 * mu, the minimisers of eq. (1) do not depend on it).
 *
 * Conventions for every entry point:
 *  - Matrices are dense, row-major.  "Device" pointers address GPU memory
 *    of the current HIP device (e.g. a torch CUDA tensor's data_ptr());
 *    "host" pointers address ordinary CPU memory.
 *  - The caller owns every buffer it passes; the library never frees or
 *    retains them after the call returns.  The handle owns its workspace
 *    (allocated in sfr_create, freed in sfr_destroy).
 *  - Calls are synchronous with respect to `hip_stream` (a hipStream_t,
 *    NULL for the legacy default stream): they enqueue their kernels on it
 *    and return after the outputs are written.
 *  - Return value: SFR_OK (0), an error (< 0: outputs left untouched) or a
 *    warning (> 0: outputs valid).  Arguments are validated on the host
 *    before any device work.
 *  - A handle serves one solve at a time; distinct handles are independent.
 *    Handles may be driven from several host threads on several streams.
 *    Solves whose rows are split over several cooperating workgroups (wide
 *    rows: n above about 1000 columns at r <= 10, above 512 at larger r)
 *    need all of those workgroups resident at once, so within one process
 *    such solves run one after the other (a process-wide lock, held until
 *    the solve's stream has drained); other solves run beside them.  Their
 *    waits are bounded: if the device is held by another process's kernels
 *    or by a running queue (sfr_queue_start) for too long, the solve
 *    returns SFR_ERR_DEVICE with its outputs untouched.
 *  - Kernel forms can be forced through the environment, read when a handle
 *    is created (SFR_SWEEP, SFR_EXCH), when a solve starts (SFR_FIRST) or when
 *    a pass is launched (SFR_SPASS): SFR_FIRST=sweep runs the first iteration
 *    through the general sweep instead of the one-pass form for V_0 = I;
 *    SFR_SWEEP=vector|mfma picks the FP32 sweep kernel, SFR_EXCH=gather|reduce
 *    the cluster exchange of the matrix-core sweep, SFR_SPASS=vector|mfma
 *    keeps the returned-S pass in its column-tile form (vector ALU, or the
 *    matrix cores where the rank allows) also for rows of at most 256
 *    columns.  Every form computes the same iteration; the default is chosen
 *    per shape.
 */
#ifndef SFR_H
#define SFR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sfr_ctx* sfr_handle;

typedef enum {
    SFR_OK = 0,
    SFR_ERR_ARG = -1,        /* invalid argument (sizes, NULL pointers, ranges) */
    SFR_ERR_NOMEM = -2,      /* device workspace allocation failed */
    SFR_ERR_DEVICE = -3,     /* HIP runtime error or device-side wait bound hit */
    SFR_ERR_RANK = -4,       /* rank(X V B) < r: P_O of eq. (7) is not unique */
    SFR_ERR_NONFINITE = -5,  /* NaN/Inf in M or in the iteration */
    SFR_ERR_HANDLE = -6,     /* NULL or wrong-kind handle */
    SFR_ERR_SCRATCH = -7,    /* sfr_solve_noalloc: the problem needs more device workspace than
                                its static scratch holds */
    SFR_ERR_BUSY = -8,       /* sfr_queue_submit: every slot holds a problem in flight */
    SFR_WARN_MAXITER = 1,    /* max_iter reached before the tolerance */
    SFR_WARN_NOT_SPD = 2     /* returned B has a non-positive eigenvalue (eq. (8) is
                                not guaranteed SPD away from the optimum, Appendix) */
} sfr_status;

typedef enum {
    SFR_F64 = 0,             /* M, S, U, V are double; all arithmetic in FP64 */
    SFR_F32 = 1              /* M, S, U, V are float; r x r algebra stays FP64 */
} sfr_precision;

/*
 * Options.  Zero-filled fields select the defaults; set struct_size to
 * sizeof(sfr_options).
 */
typedef struct {
    uint32_t struct_size;
    int32_t precision;       /* sfr_precision, default SFR_F64 */
    double rho;              /* continuation factor rho > 1 (Alg. 1), default 1.5 */
    double mu_bar;           /* penalty cap (Alg. 1), default 1e9 */
    int32_t max_iter;        /* iteration cap, default 300 */
    int32_t fixed_iters;     /* > 0: run exactly this many iterations, no tolerance test */
    int32_t nystrom_l;       /* > 0: FR-Nys handle with l sampled rows/columns (Alg. 3) */
    int32_t profile;         /* nonzero: time every general sweep launch with HIP start/stop
                                events bound to its dispatch and report the mean in
                                sfr_info.sweep_ms (the events add a few us per launch) */
    double mu_left;          /* FR-Nys: initial penalty of the m x l sub-solve (> 0) */
    double mu_top;           /* FR-Nys: initial penalty of the l x n sub-solve (> 0) */
    int32_t bf16;            /* nonzero (SFR_F32 FR-ADM handles only): BF16-operand contractions
                                for the leading iterations.  Such a sweep runs on the matrix cores
                                with its two bulk contractions (p = X V, Q = X^T P) taking BF16
                                operands with FP32 accumulation; the reconstruction l = a_i V^T,
                                M, Y and all stored values stay FP32, and the r x r algebra and the
                                reductions stay FP64.  The BF16 phase ends after bf16_iters iterations or at a
                                relative residual <= bf16_tol, whichever comes first; FP32
                                iterations then continue from its returned iterate (same buffers,
                                transforms and mu) under the handle's rule, within the same
                                iteration budget.  Both 0: every iteration in BF16.  Needs n >= the
                                matrix-core slice width (1024 columns for r <= 12, 512 above):
                                sfr_create returns SFR_ERR_ARG otherwise; sfr_tsvd ignores it. */
    int32_t bf16_iters;      /* >= 0, only with bf16 */
    double bf16_tol;         /* >= 0, only with bf16 */
} sfr_options;

/* Per-solve report. */
typedef struct {
    int32_t iters;           /* iterations of Alg. 1 performed (FR-Nys: of the m x l block) */
    int32_t iters_top;       /* FR-Nys: iterations of the l x n block; else 0 */
    int32_t converged;       /* 1 if the tolerance was met (or fixed_iters ran) */
    int32_t reserved0;
    double rel_residual;     /* ||M - L - S||_F / ||M||_F after the last iteration
                                (sfr_tsvd: ||B_k - B_{k-1}||_F / ||B_k||_F) */
    double min_eig_B;        /* smallest eigenvalue of the returned B */
    double mu_final;         /* penalty used by the last iteration */
    double sweep_ms;         /* profile != 0: mean duration of the fused sweep kernel over the
                                iterations 2..K (ms); else 0 */
    int32_t sweeps_timed;    /* number of launches averaged in sweep_ms */
    int32_t reserved1;
    double mu0;              /* the initial penalty mu_0 used: sfr_solve, the handle's mu or
                                1.25 / ||M||_2 for a handle created with mu <= 0;
                                sfr_solve_batch, the item's mu; else 0 */
    double orth_err;         /* max(||U^T U - I_r||_F, ||V^T V - I_r||_F) of the returned factors as
                                stored (their distance from St_{m,r} and St_{n,r}, eq. (7)),
                                accumulated in FP64 */
} sfr_info;

/*
 * Create a solver for m x n inputs and rank r.
 *   m, n >= 1, 1 <= r <= min(m, n, 1024).  Ranks up to 32 run the fused
 *   one-pass sweeps (FP64 or FP32).  Ranks 33 to 1024 (Table 2's r = 0.1 m,
 *   the clustering shapes of Sec. 5.3) run the large-rank engine: FP32
 *   FR-ADM and Alg. 4 only (precision SFR_F32, nystrom_l 0, bf16 0, else
 *   SFR_ERR_ARG), with the m x n contractions as matrix-core GEMM tiles and
 *   the r x r algebra in FP64 through Newton-Schulz inverse square roots; an
 *   r x r Gram that iteration cannot invert (condition number beyond about
 *   1e7) gives SFR_ERR_RANK.
 *   lambda > 0: weight of ||S||_1; the S-step threshold is lambda/mu_k.
 *   mu > 0: initial penalty mu_0 of Alg. 1 (finite).  mu <= 0 (finite,
 *     FR-ADM handles): each sfr_solve takes mu_0 = 1.25 / ||M||_2, with
 *     ||M||_2 the largest eigenvalue of B after Alg. 4 on M (run to a relative
 *     change of B of 1e-6, at most 60 steps, in the handle's workspace: the
 *     caller's outputs are written only by the solve that follows);
 *     sfr_info.mu0 reports it.  Alg. 1's literal
 *     mu_0 = 1 does not recover the planted L on the synthetic workloads;
 *     this scale of the initial threshold does.
 *   tol >= 0: stop at the first iteration k with
 *       ||M - L_{k+1} - S_{k+1}||_F / ||M||_F <= tol
 *     (Alg. 1 leaves "converged" unspecified; this is the reading taken).
 *   opt: NULL or options (see sfr_options).
 * FR-Nys handles (opt->nystrom_l = l > 0) need r <= l <= min(m, n) and
 * positive mu_left, mu_top; the argument mu is then unused.
 * Allocates the whole device workspace on the current HIP device; returns
 * SFR_ERR_NOMEM if it does not fit.
 */
sfr_status sfr_create(sfr_handle* out, int64_t m, int64_t n, int32_t r, double lambda, double mu,
                      double tol, const sfr_options* opt);

/*
 * FR-ADM (Alg. 1).
 *   M (device, m x ldm, ldm >= n): the data; read only.
 *   U (device, m x r), V (device, n x r), element type of the precision:
 *     the Stiefel factors of the returned L = U B V^T.
 *   B (device, r x r, double): the symmetric factor (Sym of eq. (8)).
 *   S (device, m x lds, lds >= n, or NULL): the returned sparse part
 *     S_{k+1} = P_ST_{lambda/mu_k}(M - L_{k+1} + Y_k/mu_k) of the last
 *     iteration.
 *   info (host, may be NULL): report.
 * Errors: SFR_ERR_HANDLE (NULL, FR-Nys or batched handle), SFR_ERR_ARG (NULL M/U/B/V,
 * ldm < n, lds < n), SFR_ERR_NONFINITE, SFR_ERR_RANK, SFR_ERR_DEVICE.
 */
sfr_status sfr_solve(sfr_handle h, const void* M, int64_t ldm, void* U, double* B, void* V, void* S,
                     int64_t lds, sfr_info* info, void* hip_stream);

/*
 * FR-Nys (Alg. 3) on a handle created with nystrom_l = l.
 *   perm (host, m entries): the random row shuffle; row i of the shuffled
 *     matrix is row perm[i] of M.  Must be a permutation of 0..m-1.
 *   Outputs as for sfr_solve, with L = U B V^T the Nystrom combination
 *   L_L (L_L[1:l,1:l])^+ L_T of the two sub-solves, rows in M's own order;
 *   B is diagonal positive (singular values of the r x r core).  S = M - L.
 */
sfr_status sfr_solve_nys(sfr_handle h, const void* M, int64_t ldm, const int64_t* perm, void* U, double* B,
                         void* V, void* S, int64_t lds, sfr_info* info, void* hip_stream);

/*
 * FixedRankOptFull (Appendix, Alg. 4): FixedRankOptStep (Alg. 2) repeated
 * on the fixed matrix M from B_0 = I_r, V_0 = I_{n x r}; the iterates
 * converge Q-linearly, at the rate (sigma_{r+1} / sigma_r)^2, to the rank-r
 * truncated SVD L = U B V^T of M (Eckart-Young, eq. (5); Appendix,
 * Theorem 2), provided rank(M V_0) = r.
 *   Uses an FR-ADM handle (sfr_create): its precision, tol, max_iter and
 *   fixed_iters apply; lambda and mu are not used.  Alg. 4 leaves
 *   "converged" unspecified; the reading taken is to stop after the first
 *   step k with ||B_k - B_{k-1}||_F <= tol ||B_k||_F (fixed_iters > 0:
 *   after exactly that many steps; max_iter reached: SFR_WARN_MAXITER).
 *   M (device, m x ldm, ldm >= n): read only.
 *   U (device, m x r), V (device, n x r), element type of the precision;
 *   B (device, r x r, double): the factors of the returned L = U B V^T.
 *   info (host, may be NULL): iters = steps performed, rel_residual = the
 *   last relative change of B, min_eig_B.
 * Errors: SFR_ERR_HANDLE (NULL, FR-Nys or batched handle), SFR_ERR_ARG (NULL M/U/B/V,
 * ldm < n), SFR_ERR_NONFINITE, SFR_ERR_RANK (rank(M V_i) < r), SFR_ERR_DEVICE.
 * On an error the outputs are left untouched.
 */
sfr_status sfr_tsvd(sfr_handle h, const void* M, int64_t ldm, void* U, double* B, void* V, sfr_info* info,
                    void* hip_stream);

/*
 * Batched FR-ADM (Alg. 1 with Alg. 2) for many small independent problems.
 * One item of a batch: the problem and its outputs.  All pointers are device
 * pointers, float data (FP32); B is double.
 *   m, n, r: sizes, 1 <= r <= min(m, n), within the handle's limits.
 *   lambda > 0, mu > 0 (mu_0), tol >= 0: as in sfr_create.
 *   M (m x ldm, ldm >= n): read only.
 *   U (m x r), B (r x r), V (n x r): factors of the returned L = U B V^T.
 *   S (m x lds, lds >= n) or NULL: the returned sparse part, as in sfr_solve.
 */
typedef struct {
    int64_t m, n;
    int32_t r;
    int32_t reserved0;
    double lambda, mu, tol;
    const void* M;
    int64_t ldm;
    void* U;
    double* B;
    void* V;
    void* S;
    int64_t lds;
} sfr_batch_item;

/*
 * Create a batched handle: `capacity` workspace slots for problems of at
 * most max_m x max_n and rank max_r (FP32 only).
 *   1 <= capacity <= 65536; 1 <= max_n <= 512; 1 <= max_m <= 2^22;
 *   1 <= max_r <= min(16, max_m, max_n).
 *   opt (required): precision must be SFR_F32 and nystrom_l 0; rho,
 *   mu_bar, max_iter and fixed_iters apply to every item (profile is
 *   ignored).  bf16, bf16_iters, bf16_tol: as for sfr_create, for the items
 *   that run the matrix-core form (rank bucket 8 to 16): their p = X V and
 *   Q = X^T P products take BF16 operands (FP32 accumulation) in the leading
 *   iterations, up to bf16_iters and while the residual is above bf16_tol,
 *   and FP32 iterations follow; other items are unaffected.
 * Each slot holds 2 Y buffers (max_m x max_n), 2 P (max_m x 16) and 2 Q
 * (max_n x 16) buffers in device memory; sfr_workspace_bytes reports the
 * total.  Returns SFR_ERR_NOMEM if it does not fit.
 */
sfr_status sfr_create_batch(sfr_handle* out, int32_t capacity, int64_t max_m, int64_t max_n, int32_t max_r,
                            const sfr_options* opt);

/*
 * Solve `count` (0 <= count <= capacity) independent problems with one
 * kernel launch, one workgroup per problem; each problem runs the same
 * iteration, stopping rule and outputs as sfr_solve on an FP32 handle.
 *   items (host, count entries): the problems.  Their output buffers must
 *     not overlap one another or any input.
 *   infos (host, count entries, may be NULL): per-item report (sweep_ms 0).
 *   statuses (host, count entries, may be NULL): per-item status, with the
 *     meaning of sfr_solve's return value; an item with an error leaves its
 *     outputs untouched (other items are unaffected).
 * Returns SFR_ERR_HANDLE (NULL or non-batched handle), SFR_ERR_ARG (an item
 * out of the handle's limits: nothing is run), SFR_ERR_DEVICE, or else the
 * first negative per-item status, or SFR_OK (warnings are per item only).
 */
sfr_status sfr_solve_batch(sfr_handle h, const sfr_batch_item* items, int32_t count, sfr_info* infos,
                           int32_t* statuses, void* hip_stream);

/*
 * Autotuner of a batched handle: for every (class, rank bucket) present
 * among `items` -- class 0: n > 128, class 1: n <= 128; buckets r = 1, 2, 3,
 * 4, 5, 6, 8, 10, 12, 16 -- times each form of the batched kernel's band
 * loop on those items (4 iterations, after one warm-up run) and records the
 * fastest in the handle; later sfr_solve_batch calls on the handle use it.
 * The forms are exact and give the same iteration within rounding: lane
 * groups of 8 or 16 lanes per row (class 1 only), one or two rows per
 * wavefront over 64 lanes, and the matrix-core band loop (r buckets >= 8).
 * Untuned (class, bucket) pairs keep the built-in choice.
 *   items (host, count entries): as for sfr_solve_batch; their output
 *     buffers are overwritten with 4-iteration results.
 *   table (host, 20 entries, may be NULL): receives the choice per
 *     [class * 10 + bucket index]: 0 not tuned, 1 lane groups, 2 one row per
 *     wavefront, 3 two rows, 4 matrix cores.
 * Errors: SFR_ERR_HANDLE (NULL or non-batched handle), SFR_ERR_ARG (an item
 * out of the handle's limits), SFR_ERR_DEVICE.
 */
sfr_status sfr_tune_batch(sfr_handle h, const sfr_batch_item* items, int32_t count, int32_t* table,
                          void* hip_stream);

/*
 * Queue form of a batched handle (continuous batching).  Persistent kernels
 * take problems one by one from a queue that the host appends to while they
 * run, and retire each problem as soon as it is solved: a problem submitted
 * while others are on the GPU starts as soon as a workgroup is free, and its
 * result does not wait for any other problem.  Admission is by slot: each
 * problem in flight holds one of the handle's `capacity` workspace slots
 * (device memory allocated by sfr_create_batch), freed when its result is
 * collected.  Each problem runs the iteration, stopping rule and outputs of
 * sfr_solve_batch; problems with r <= 6 go to one kernel (the two-rows-per-
 * wavefront form at the R = 6 bucket), the others to a second (the
 * matrix-core form at the R = 16 bucket).  A problem's result depends only
 * on the problem itself, not on what else is in flight.
 *
 * sfr_queue_start(h, grid_large, grid_small): launch the two persistent
 *   kernels on two streams of the handle, with grid_large and grid_small
 *   workgroups (0: three quarters and one quarter of the compute units).
 *   Allocates pinned host memory for the queue the first time.  While the
 *   queue runs, sfr_solve_batch and sfr_tune_batch return SFR_ERR_HANDLE.
 * sfr_queue_submit(h, item, ticket): host only, never blocks.  Validates
 *   the item (as sfr_solve_batch), takes a free slot, writes its descriptor
 *   and appends it to its kernel's queue; *ticket receives the slot.
 *   SFR_ERR_BUSY if every slot is in flight, SFR_ERR_ARG for an invalid item
 *   (nothing submitted).  The item's output buffers must stay valid until
 *   its result is collected.
 * sfr_queue_poll(h, ticket, done, info, status): host only, never blocks.
 *   *done = 1 once the problem is solved: its outputs are written, *info and
 *   *status (the problem's sfr_status) are filled and the slot is free
 *   again; else *done = 0.  An unused ticket gives SFR_ERR_ARG.
 * sfr_queue_stop(h): close the queue, wait until every submitted problem is
 *   solved and both kernels have ended.  Results not yet collected stay in
 *   the handle until the next sfr_queue_start.
 * A persistent kernel that finds no work for about a second ends by itself;
 * submit and poll relaunch it when work is pending.  Errors: SFR_ERR_HANDLE
 * (NULL or non-batched handle, queue not running / already running),
 * SFR_ERR_DEVICE, SFR_ERR_NOMEM (sfr_queue_start).
 */
sfr_status sfr_queue_start(sfr_handle h, int32_t grid_large, int32_t grid_small);
sfr_status sfr_queue_submit(sfr_handle h, const sfr_batch_item* item, int32_t* ticket);
sfr_status sfr_queue_poll(sfr_handle h, int32_t ticket, int32_t* done, sfr_info* info, int32_t* status);
sfr_status sfr_queue_stop(sfr_handle h);

/*
 * FR-ADM without any device allocation, for callers that cannot allocate:
 * code under HIP graph capture, tight serving loops, hosts that forbid
 * hipMalloc.  The same solve as sfr_create(m, n, r, lambda, mu, tol, opt)
 * followed by sfr_solve(h, M, ldm, U, B, V, S, lds, info, hip_stream) and
 * sfr_destroy(h), with the same arguments, results and statuses, and the same
 * kernels.
 *   Workspace: a static device array of 128 MiB per device (held by each
 *     device the library runs on until the process ends) instead of a
 *     handle's allocations.  It holds the two m x n dual buffers Y and the
 *     factor, partial-sum and exchange buffers (and a padded copy of M when
 *     M is not 16-byte aligned with ldm a multiple of 4 (FP32) or 2 (FP64),
 *     or n is not): FP32 problems up to about 3000 x 3000 fit (less at
 *     larger r).  A problem that needs more returns SFR_ERR_SCRATCH before
 *     any device work.  No hipMalloc, hipFree, pinned host memory or HIP
 *     event is used; progress is read by synchronising hip_stream.
 *   Options: as for sfr_create, except that nystrom_l and profile must be 0
 *     and r <= 32 (SFR_ERR_ARG otherwise).
 *   Concurrency: every call on one device uses that device's one scratch
 *     array and host-side state, which keep the last call's contents (the
 *     call initialises everything it reads); calls that overlap on one
 *     device race and must not be made.
 * Errors: those of sfr_create and sfr_solve (outputs left untouched), and
 * SFR_ERR_SCRATCH.
 */
sfr_status sfr_solve_noalloc(int64_t m, int64_t n, int32_t r, double lambda, double mu, double tol,
                             const sfr_options* opt, const void* M, int64_t ldm, void* U, double* B, void* V,
                             void* S, int64_t lds, sfr_info* info, void* hip_stream);

/* Release the handle and its workspace.  NULL is accepted. */
sfr_status sfr_destroy(sfr_handle h);

/* Device workspace owned by the handle, in bytes. */
sfr_status sfr_workspace_bytes(sfr_handle h, uint64_t* bytes);

/* Static description of a status code. */
const char* sfr_status_string(sfr_status s);

/* Library version as "major.minor.patch". */
const char* sfr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SFR_H */
