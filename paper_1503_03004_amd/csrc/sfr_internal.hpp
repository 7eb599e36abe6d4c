// Internal declarations of the S-FR HIP library (gfx950).
//
// Device-resident solver state and kernel argument blocks for the FR-ADM
// iteration (Alg. 1) with its L-step FixedRankOptStep (Alg. 2) evaluated in
// one pass over the data per iteration:
//
//   X_k = M - S_k + Y_k/mu_k             formed in registers, never stored
//   P   = X_k V_k          (m x r)       row-owned dot products
//   Q   = X_k^T P          (n x r)       = X^T X V, column partials
//   U   = P B C1,          C1 = (B G_P B)^{-1/2},   G_P = P^T P
//   V   = Q K C2,          K  = B C1 B,  C2 = (K G_Q K)^{-1/2},  G_Q = Q^T Q
//   B   = Sym(C1 B G_Q K C2)
//
// The first two lines are the two Stiefel projections of eq. (7) in their
// A (A^T A)^{-1/2} form (A = X V B and A = X^T U B); the last is the SPD
// step of eq. (8), using U^T X V = C1 B P^T X V = C1 B Q^T V.  The small
// r x r algebra runs in FP64 in one workgroup; the m x n work runs in the
// storage precision T (float or double).
//
// Within a sweep, the S- and dual steps of the previous iteration are fused
// in front of the L-step input: with R = M - L_k + Y_{k-1}/mu_{k-1},
//   Y_k = clamp(mu_{k-1} R, -lambda, lambda)
//   S_k = R - Y_k / mu_{k-1}           (soft threshold, notation section)
//   X_k = L_k + (Y_k - Y_{k-1})/mu_{k-1} + Y_k/mu_k
// so each sweep reads M and Y_{k-1} and writes Y_k: 3 words per element.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sfr {

constexpr int kMaxR = 32;           // ranks of the fused sweeps
constexpr int kMaxRLarge = 1024;     // ranks of the large-rank engine (lr.hip)
constexpr int kTPB = 256;            // threads per workgroup of the streaming kernels
constexpr int kGramU = 8;            // P loads in flight per thread of the Gram kernel
constexpr int kXCD = 8;              // accelerator complex dies on MI355X
constexpr uint32_t kSpinLimit = 1u << 24;
// Residual partials the step kernel loads in its first round (one per
// sweep workgroup; more are summed by a tail loop).
constexpr int kMaxDyPartials = 2048;
// Upper bound on the Gram partials of one pass (one per Gram workgroup).
constexpr int kMaxGramPartials = 256;
// Threads of the step kernel.  It adds the Gram partials itself while each
// of its threads has at most kStepPartialLoads of them to load (one round
// of loads); beyond that a reduction kernel adds them first.
constexpr int kStepTPB = 512;
constexpr int kStepPartialLoads = 64;

// Status codes mirrored from the public header (kept numerically equal).
enum : int32_t {
    kOK = 0, kErrArg = -1, kErrNoMem = -2, kErrDevice = -3, kErrRank = -4,
    kErrNonFinite = -5, kErrHandle = -6, kErrScratch = -7, kErrBusy = -8,
    kWarnMaxIter = 1, kWarnNotSPD = 2
};

// Solver state kept in device memory for one solve.  Written by the FP64
// step kernel, read by the streaming kernels.
struct DevState {
    // problem (fixed during a solve)
    int32_t m, n, r, R;
    int32_t max_iter, fixed_iters;
    double lambda, rho, mu_bar, tol;
    const void* M;      // caller's data, row-major
    int64_t ldm;        // leading dimension of M (elements)
    // progress
    int32_t k;          // index of the next sweep (1-based)
    int32_t done;       // 1 once the iteration has stopped
    int32_t status;     // kOK or a negative error code, or kWarnMaxIter
    int32_t iters;      // completed iterations once done
    int32_t exch_timeout;  // set if a cluster exchange wait hit its bound
    int32_t tsvd;       // 1: FixedRankOptFull (Alg. 4) on X = M, stop on the change of B
    int32_t stop_after; // > 0: the step of this iteration ends the solve (a fixed-count FR-ADM solve
                        // whose last residual is taken by the S pass instead of one more sweep)
    double nrmM;        // ||M||_F
    double mu;          // mu_k used by the next sweep's L-step input
    double mu_prev;     // mu_{k-1} used by the next sweep's S/Y step
    double res;         // last residual ||M - L - S||_F / ||M||_F
    double min_eig_B;   // filled by the finalize step
    double max_eig_B;   // largest eigenvalue of B (launch_max_eig)
    double orth_err;    // max(||U^T U - I||_F, ||V^T V - I||_F) of the returned factors
    double B[kMaxR * kMaxR];
    double TU[kMaxR * kMaxR];     // a_i = P_i TU gives L rows (L = A V^T)
    double TUbar[kMaxR * kMaxR];  // U = P TUbar
    double TV[kMaxR * kMaxR];     // V = Q TV
    float TUf[kMaxR * kMaxR];
    float TVf[kMaxR * kMaxR];
    // eigenbases of the two Grams of the previous step (warm start of the
    // next Jacobi eigendecompositions)
    double E1[kMaxR * kMaxR];
    double E2[kMaxR * kMaxR];
};

template <typename T> __host__ __device__ inline const T* st_TU(const DevState* s);
template <> __host__ __device__ inline const float* st_TU<float>(const DevState* s) { return s->TUf; }
template <> __host__ __device__ inline const double* st_TU<double>(const DevState* s) { return s->TU; }
template <typename T> __host__ __device__ inline const T* st_TV(const DevState* s);
template <> __host__ __device__ inline const float* st_TV<float>(const DevState* s) { return s->TVf; }
template <> __host__ __device__ inline const double* st_TV<double>(const DevState* s) { return s->TV; }

// Arguments of one sweep launch.  Parities of the ping-pong buffers are
// fixed per launch (sweep k reads buffer (k-1)&1 and writes buffer k&1).
template <typename T>
struct SweepArgs {
    const DevState* st;
    const T* Yprev;      // Y_{k-1}, m x ldy (mode 2 only)
    T* Ynext;            // Y_k (modes 1, 2)
    int64_t ldy;
    const T* Pprev;      // P from sweep k-1, m x R (modes 1, 2)
    T* Pnext;            // P of sweep k, m x R
    const T* Qprev;      // Q from sweep k-1 (or V_1 = I), n x R
    T* Qpart;            // per-cluster column partials, ncl x n x R
    double* dy2part;     // per-workgroup ||Y_k - Y_{k-1}||^2 (mode 0: ||M||^2)
    unsigned long long* exch;  // cluster exchange slots (tagged words)
    int32_t m, n;
    int32_t mode;        // 0: X = M (k = 1); 1: Y_{k-1} = 0 (k = 2); 2: general
    int32_t lpr;         // lanes per row in the row pass (4..64)
    int32_t nv;          // vectors per lane per row
    int32_t W;           // columns per member slice = lpr * VEC * nv
    int32_t c;           // members per cluster (column slices)
    int32_t cpx;         // clusters per XCD (xcd_local layout)
    int32_t xcd_local;   // 1: members of a cluster share an XCD; 0: contiguous workgroups
    int32_t ncl;         // clusters
    int32_t nbands;      // ceil(m / H)
    int32_t nbl_max;     // max bands per cluster (tag stride)
};

// Column-partial reduction and Gram partials (one launch per iteration).
template <typename T>
struct GramArgs {
    const DevState* st;
    const T* Qpart;      // ncl x n x R
    T* Qnext;            // n x R
    const T* Pnext;      // m x R
    double* GQpart;      // nqb x E
    double* GPpart;      // npb x E
    int32_t m, n, ncl;
    int32_t rows_q;      // Q rows per workgroup
    int32_t nqb;         // workgroups for Q
    int32_t rows_p;      // P rows per workgroup
    int32_t npb;         // workgroups for P
};

// Relative off-diagonal size at which the Jacobi sweeps of an inverse
// square root stop, the rest being a second-order expansion with relative
// error O(tau^3 r^2): about 1e-16 for FP64 solves; for FP32 solves about
// 1e-11 r^2, far below the FP32 rounding of the m x n work (~1e-7).
constexpr double kDkTauF64 = 4e-6;
constexpr double kDkTauF32 = 2e-4;
// The step kernel's Newton-Schulz inverse square roots are accurate to
// about cond eps; above these bounds on the condition number of the Gram
// products it takes the Jacobi path instead (result error ~1e-10 at the
// FP64 bound, ~1e-6 at the FP32 one, against parity bars of 1e-9 and 1e-5).
constexpr double kNsKappaF64 = 1e6;
constexpr double kNsKappaF32 = 1e10;

// FP64 r x r step (one workgroup).  It adds npb (nqb) partials of G_P
// (G_Q); 1 once launch_gram_reduce has left the sums in partial 0.
struct StepArgs {
    DevState* st;
    const double* GPpart; int32_t npb;
    const double* GQpart; int32_t nqb;
    const double* dy2part; int32_t ndy;
    double* res_hist;     // res_hist[k-1] = residual of iteration k
    double ns_kappa;      // kNsKappaF64 or kNsKappaF32
    double dk_tau;        // kDkTauF64 or kDkTauF32 (Jacobi path)
};

// The ping-pong buffers of one solve (P, Q: m x R, n x R; Y: m x n with
// leading dimension ldy).  Kernels that run after the iteration pick the
// returned iterate's buffers from the iteration count in DevState.
template <typename T>
struct PingPong {
    T* P[2];
    T* Q[2];
    const T* Y[2];
};

// Arguments of the dense S pass.  With st set (FR-ADM), Y, A, Vt and mu are
// taken from the ping-pong buffers and the state of the returned iterate;
// otherwise the explicit pointers and mu are used.
template <typename T>
struct LowrankArgs {
    DevState* st;
    PingPong<T> pp;
    const T* M;
    int64_t ldm;
    const T* Y;
    int64_t ldy;
    const T* A;
    const T* Vt;
    T* S;
    int64_t lds;
    int m, n, mode, rows_per_blk;
    int min_eig;   // with st: also write min eig(B) into the state
    double lam, mu;
    double* rpart; // with st, FR-ADM: per-workgroup ||Y_{K+1} - Y_K||^2 of the returned iterate, or nullptr
};

// Partials of the returned iterate's residual held by the S pass: one per
// workgroup of its grid (at most this many for an m x n pass).
int lowrank_res_parts(int m, int n);
// Residual ||M - L_{K+1} - S_{K+1}||_F / ||M||_F = ||Y_{K+1} - Y_K||_F / (mu_K ||M||_F)
// of a solve stopped by stop_after, from the S pass's partials (fixed order):
// into the state and res_hist[K - 1].
hipError_t launch_res_final(DevState* st, const double* rpart, int count, double* res_hist, hipStream_t s);

// One problem of a batched solve (batch.hip): the caller's arguments, the
// slot's workspace and, on return, its results.  Device memory.
struct BatchItemDev {
    int32_t m, n, r, ldy;           // ldy: row pitch of the Y workspace
    double lambda, mu0, tol;
    const float* M;
    int64_t ldm;
    float* U;
    double* B;
    float* V;
    float* S;                        // may be NULL
    int64_t lds;
    float* Y0;
    float* Y1;
    float* P0;
    float* P1;
    float* Q0;
    float* Q1;
    // results
    int32_t iters, status;
    double res, min_eig_B, mu_final;
    double orth_err;                 // max(||U^T U - I||_F, ||V^T V - I||_F) of the written factors
    int32_t seq, reserved;           // queue form: submission number, copied to the done flag
};

// Queue form of the batched solver (batch_queue_kernel): the claim counter
// in device memory, and the host's side of the queue in pinned coherent
// memory (the host writes it while the kernel runs).
struct BatchQueueDev {
    int32_t head;      // next entry to claim
    int32_t pad[63];
};
constexpr int kQueueMaxCap = 65536;
struct BatchQueueHost {
    int32_t tail;      // entries submitted
    int32_t closed;    // 1: leave once drained
    int32_t pad[14];
    int32_t order[kQueueMaxCap];   // entry e -> slot (ring of the handle's capacity)
};

struct BatchParams {
    double rho, mu_bar;
    int32_t max_iter, fixed_iters;
    // BF16-operand p and Q products (matrix-core form) for the leading
    // iterations: up to bf16_iters and while the residual is above bf16_tol
    int32_t bf16, bf16_iters;
    double bf16_tol;
};

// Forms of the batched kernel's band loop (all exact; they differ in speed):
// lane groups of 8/16 lanes per row (narrow problems), one or two rows per
// wavefront over 64 lanes, or the matrix-core loop (R >= 8).
enum : int { kBVAuto = 0, kBVNarrow = 1, kBVRow1 = 2, kBVRow2 = 3, kBVMfma = 4 };
int batch_default_variant(int R, bool narrow);
bool batch_variant_valid(int R, int variant);
// narrow: the items have n <= 128; variant kBVAuto picks the default form
hipError_t launch_batch(BatchItemDev* items, int count, int R, bool narrow, int variant, const BatchParams& bp,
                        hipStream_t s);
// orth_err of every successful item of a batch (one workgroup per item),
// from the factors it wrote.
hipError_t launch_batch_orth(BatchItemDev* items, int count, hipStream_t s);
// Persistent queue form: `grid` workgroups; small: the R = 6 two-rows form
// (r <= 6), else the R = 16 matrix-core form (r <= 16).
hipError_t launch_batch_queue(BatchItemDev* items, const BatchParams& bp, BatchQueueDev* q, BatchQueueHost* hq,
                              int32_t* done, int cap, int small, int grid, hipStream_t s);

// Host-side launchers (sweep.hip / small.hip / dense.hip).  The sweep takes
// an optional start/stop event pair bound to its dispatch.
template <typename T>
hipError_t launch_sweep(const SweepArgs<T>& a, int R, int grid, size_t lds, hipStream_t s,
                        hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
template <typename T>
hipError_t launch_gram(const GramArgs<T>& a, int R, hipStream_t s);
// Sum the nqb (npb) partials of each of the E entries of G_Q (G_P) into
// partial 0, in a fixed order.
hipError_t launch_gram_reduce(const DevState* st, double* GQpart, int nqb, double* GPpart, int npb, int E,
                              hipStream_t s);
template <typename T>
size_t sweep_lds_bytes_c(int R, int lpr, int W, int c);
template <typename T>
int sweep_threads(int R);     // workgroup size of the sweep for rank bucket R
template <typename T>
int sweep_max_width(int R);   // widest column slice the sweep's column pass holds
// Exchange slots cycled by a cluster (bands in flight between its members).
constexpr int kExchSlots = 8;
// Clusters of at least this many members exchange by reduce-then-broadcast
// in the matrix-core sweep's 4-tile forms (all-gather reads 16 R c words a
// band per member, reduce-then-broadcast about 16 R + c).
constexpr int kRbMinMembers = 12;
// ... and at least this many bands per cluster (each band then waits twice).
constexpr int kRbMinBands = 8;
// Set the dynamic LDS limit of the sweep kernel that launch_sweep takes for
// rank bucket R, lpr lanes per row and W-column slices, and report its
// occupancy.
template <typename T>
hipError_t sweep_prepare(int R, int lpr, int W, size_t lds, int* blocks_per_cu);

// Matrix-core sweep (sweep_mfma.hip): FP32, R <= 32, member slices of
// sweep_mfma_width(R, tiles) columns, 16-row bands, 512-thread workgroups.
// tiles: 16-column tiles per wavefront, 0 for the bucket's default form; 8
// selects the wide form of the R = 16 bucket (1024-column slices).
bool sweep_mfma_supported(int R);
// rb: the reduce-then-broadcast exchange (4-tile forms, R > 12), whose
// reduced words follow the partial words in the exchange buffer.
bool sweep_mfma_rb_supported(int R, int tiles);
size_t sweep_mfma_lds_bytes(int R, int tiles, bool rb);
int sweep_mfma_width(int R, int tiles);
hipError_t sweep_mfma_prepare(int R, int tiles, bool rb, size_t lds, int* blocks_per_cu);
// bf16: the contractions take BF16 operands (FP32 accumulation)
hipError_t launch_sweep_mfma(const SweepArgs<float>& a, int R, int tiles, bool rb, int grid, size_t lds,
                             hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr, bool bf16 = false);

hipError_t launch_step(const StepArgs& a, int R, hipStream_t s);
// Once per process and rank bucket before the first launch_step (the step
// kernel's LDS size).
hipError_t step_prepare(int R);
hipError_t launch_final_small(DevState* st, int R, hipStream_t s);
// Largest eigenvalue of the returned B into st->max_eig_B.
hipError_t launch_max_eig(DevState* st, int R, hipStream_t s);
// Continue a stopped iteration from its returned iterate K under a new
// stopping rule (no-op if it stopped with an error, or with no budget left).
hipError_t launch_refine_start(DevState* st, int fixed_iters, double tol, int max_iter, hipStream_t s);

template <typename T>
hipError_t launch_init_q(T* Q, int n, int r, int R, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, size_t count, hipStream_t s);
template <typename T>
hipError_t launch_copy_pad(const T* src, int64_t lds, T* dst, int64_t ldd, int m, int n, hipStream_t s);
template <typename T>
hipError_t launch_factors(const DevState* st, const PingPong<T>& pp, int m, int n, int r, int R, T* U, T* V,
                          double* B, hipStream_t s);
template <typename T>
hipError_t launch_lowrank_pass(LowrankArgs<T> a, int R, hipStream_t s, int* parts = nullptr);
// max(||U^T U - I_r||_F, ||V^T V - I_r||_F) of stored factors U (m x r) and
// V (n x r), accumulated in FP64, into *out.  Up (nu x r(r+1)/2) and Vp
// (nv x r(r+1)/2) receive the partial Grams of nu and nv row blocks.  With
// st set, nothing is done unless that solve finished without error.
template <typename T>
hipError_t launch_orth(const DevState* st, const T* U, int m, const T* V, int n, int r, double* Up, int nu,
                       double* Vp, int nv, double* out, hipStream_t s);
template <typename T>
hipError_t launch_nys_gather(const T* M, int64_t ldm, const int64_t* perm, int m, int n, int l,
                             T* C, T* Rb, hipStream_t s);

}  // namespace sfr
