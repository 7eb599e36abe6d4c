// FR-ADM (Alg. 1 with the Alg. 2 L-step) for ranks above the fused sweeps'
// limit (32 < r <= 1024; Table 2's r = 0.1 m and the clustering shapes of
// Sec. 5.3), FP32 data.
//
// At these ranks the three m x n contractions of an iteration carry
// 6 r flops per element, far above the HBM ridge, so they run as tiled
// GEMMs on the matrix cores (v_mfma_f32_16x16x4_f32, exact FP32 products,
// FP32 accumulation) instead of one streaming pass:
//   lstep:  l = A_k V_k^T (K = R) fused with the S/dual step of iteration
//           k - 1 and the next L-step input (same algebra as the fused
//           sweep: Y_k = clamp(mu_{k-1} R, +-lambda),
//           X_k = l + (Y_k - Y_{k-1})/mu_{k-1} + Y_k/mu_k); writes Y_k, X_k
//   P_k = X_k V_k          (m x R, K = n, split over K)
//   Q_k = X_k^T P_k        (n x R, K = m, split over K)
//   A_{k+1} = P_k TU_k,  V_{k+1} = Q_k TV_k     (K = R)
// The Grams G_P = P^T P and G_Q = Q^T Q accumulate in FP64 (split over
// rows, partials added in a fixed order), and the r x r algebra of
// App. A.5 (eq. (7), eq. (8)) runs in FP64 as R x R tiled products.  Its
// two inverse square roots, (B G_P B)^{-1/2} and (K G_Q K)^{-1/2}, come from
// the coupled Newton-Schulz iteration
//   Y_0 = A / s,  Z_0 = I,  T = (3 I - Z Y) / 2,  Y <- Y T,  Z <- T Z
// (Z -> (A/s)^{-1/2}; s = ||A||_F), which needs only matrix products: an
// R x R eigendecomposition does not fit one workgroup at these ranks.  The
// smallest and largest eigenvalues of the returned B come from a Householder
// tridiagonalisation and Sturm-sequence bisection.
//
// Ranks are padded to R (a multiple of 16); padded rows and columns of the
// factors are zero and padded diagonal blocks of the r x r matrices are the
// identity, so every product is block diagonal and exact on the leading
// r x r block.
#include "engine.hpp"

#include <string.h>

#include <algorithm>
#include <climits>
#include <cmath>

namespace sfr {

typedef float lr_f32x4 __attribute__((ext_vector_type(4)));

constexpr int kLrTPB = 256;          // threads of the GEMM-shaped kernels
constexpr int kLrBK = 16;            // K depth of one LDS stage
constexpr int kLrBM = 128;           // output tile rows (FP32 GEMMs)
constexpr int kT64 = 32;             // output tile of the FP64 R x R products
constexpr int kNsIters = 24;         // Newton-Schulz iterations queued per inverse square root
constexpr int kNsMore = 40;          // further iterations run in one workgroup if those do not converge
constexpr int kNsMoreMaxR = 128;     // ... for R up to this (one workgroup's R^3 products stay short)
constexpr double kNsTol = 1e-8;      // ||Z Y - I||_F at which one last iteration finishes it
constexpr int kEigTPB = 1024;

// Device-side progress of the large-rank step beyond DevState.
struct LrState {
    int32_t ns_done_at[2];   // Newton-Schulz iteration at which instance 0/1 converged (INT_MAX: not yet)
    int32_t ns_used[2];
    double ns_scale[2];      // s of each instance
};

__device__ __forceinline__ lr_f32x4 lr_mfma(float a, float b, lr_f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// FP32 GEMM core: acc (a BM x BN tile, four wavefronts of BM/2 x BN/2) +=
// A[m0.., k] B[k, n0..] over k in [kbeg, kend).  A is stored [M][K] (lda) or,
// with AT, [K][M]; B is stored [K][N] (ldb) or, with BT, [N][K].  Each LDS
// stage holds a BM x 16 slice of A and a 16 x BN slice of B; consecutive
// threads load consecutive addresses of the contiguous dimension.
// Lane layout of v_mfma_f32_16x16x4_f32 (lane l, lr = l % 16, lq = l / 16):
// it supplies A[lr][lq] and B[lq][lr] and receives D[4 lq + e][lr].
template <int BM, int BN, bool AT, bool BT>
struct LrGemm {
    static constexpr int WM = BM / 2, WN = BN / 2, FM = WM / 16, FN = WN / 16;
    float (*As)[kLrBK + 1];
    float (*Bs)[BN + 1];

    __device__ void run(const float* __restrict__ A, int64_t lda, const float* __restrict__ B, int64_t ldb, int M,
                        int N, int m0, int n0, int kbeg, int kend, lr_f32x4 (&acc)[FM][FN])
    {
        const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
        const int wm = (wave >> 1) * WM, wn = (wave & 1) * WN;
        const int lr = lane & 15, lq = lane >> 4;
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) acc[i][j] = lr_f32x4{0.f, 0.f, 0.f, 0.f};
        constexpr int NA = BM * kLrBK / kLrTPB, NB = BN * kLrBK / kLrTPB;
        float ra[NA], rb[NB];
        auto fetch = [&](int k0) {
#pragma unroll
            for (int u = 0; u < NA; ++u) {
                const int e = threadIdx.x + u * kLrTPB;
                int i, k;
                if (!AT) { i = e / kLrBK; k = e % kLrBK; } else { k = e / BM; i = e % BM; }
                const int gi = m0 + i, gk = k0 + k;
                const bool ok = gi < M && gk < kend;
                ra[u] = ok ? (AT ? A[(int64_t)gk * lda + gi] : A[(int64_t)gi * lda + gk]) : 0.f;
            }
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                const int e = threadIdx.x + u * kLrTPB;
                int k, j;
                if (!BT) { k = e / BN; j = e % BN; } else { j = e / kLrBK; k = e % kLrBK; }
                const int gj = n0 + j, gk = k0 + k;
                const bool ok = gj < N && gk < kend;
                rb[u] = ok ? (BT ? B[(int64_t)gj * ldb + gk] : B[(int64_t)gk * ldb + gj]) : 0.f;
            }
        };
        auto stash = [&]() {
#pragma unroll
            for (int u = 0; u < NA; ++u) {
                const int e = threadIdx.x + u * kLrTPB;
                int i, k;
                if (!AT) { i = e / kLrBK; k = e % kLrBK; } else { k = e / BM; i = e % BM; }
                As[i][k] = ra[u];
            }
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                const int e = threadIdx.x + u * kLrTPB;
                int k, j;
                if (!BT) { k = e / BN; j = e % BN; } else { j = e / kLrBK; k = e % kLrBK; }
                Bs[k][j] = rb[u];
            }
        };
        if (kbeg < kend) fetch(kbeg);
        for (int k0 = kbeg; k0 < kend; k0 += kLrBK) {
            __syncthreads();
            stash();
            __syncthreads();
            if (k0 + kLrBK < kend) fetch(k0 + kLrBK);   // next stage in flight during the products
#pragma unroll
            for (int kk = 0; kk < kLrBK; kk += 4) {
                float a[FM], b[FN];
#pragma unroll
                for (int i = 0; i < FM; ++i) a[i] = As[wm + 16 * i + lr][kk + lq];
#pragma unroll
                for (int j = 0; j < FN; ++j) b[j] = Bs[kk + lq][wn + 16 * j + lr];
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j) acc[i][j] = lr_mfma(a[i], b[j], acc[i][j]);
            }
        }
    }
};

// C (+ z * zstride for split z) = A B over the K range of split z.
template <int BN, bool AT, bool BT>
__global__ void __launch_bounds__(kLrTPB) lr_gemm_kernel(const float* A, int64_t lda, const float* B, int64_t ldb,
                                                         float* C, int64_t ldc, int64_t zstride, int M, int N, int K,
                                                         int kc, const DevState* st)
{
    if (st && st->done) return;
    constexpr int BM = kLrBM;
    using G = LrGemm<BM, BN, AT, BT>;
    __shared__ float As[BM][kLrBK + 1];
    __shared__ float Bs[kLrBK][BN + 1];
    G g{As, Bs};
    lr_f32x4 acc[G::FM][G::FN];
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    const int kbeg = blockIdx.z * kc, kend = min(K, kbeg + kc);
    g.run(A, lda, B, ldb, M, N, m0, n0, kbeg, kend, acc);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * G::WM, wn = (wave & 1) * G::WN;
    float* Cz = C + (int64_t)blockIdx.z * zstride;
#pragma unroll
    for (int i = 0; i < G::FM; ++i)
#pragma unroll
        for (int j = 0; j < G::FN; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = m0 + wm + 16 * i + 4 * (lane >> 4) + e;
                const int col = n0 + wn + 16 * j + (lane & 15);
                if (row < M && col < N) Cz[(int64_t)row * ldc + col] = acc[i][j][e];
            }
}

// out = sum over z < S of part[z] (fixed order).
__global__ void lr_splitk_sum_kernel(const float* part, int64_t zstride, int S, float* out, int64_t count,
                                     const DevState* st)
{
    if (st && st->done) return;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    float s = 0.f;
    for (int z = 0; z < S; ++z) s += part[(int64_t)z * zstride + e];
    out[e] = s;
}

// ---------------------------------------------------------------------------
// The fused L-step input of iteration k (mode 1: Y_{k-1} = 0; 2: general)
// or the returned S of iterate K (mode 3).  l = A V^T on a 128 x 64 tile,
// staged through LDS, then one coalesced elementwise pass over the tile.
constexpr int kLstepBN = 64;

struct LstepArgs {
    const DevState* st;
    const float* A;     // m x R
    const float* V;     // n x R
    int R;
    const float* M; int64_t ldm;
    const float* Yprev; int64_t ldy;    // modes 2, 3 (may be NULL in mode 3: Y = 0)
    float* Ynext;       // modes 1, 2
    float* X; int64_t ldx;              // modes 1, 2
    float* S; int64_t lds;              // mode 3
    double* dy2part;    // per workgroup ||Y_k - Y_{k-1}||^2 (modes 1, 2)
    int m, n, mode;
};

__global__ void __launch_bounds__(kLrTPB) lr_lstep_kernel(LstepArgs a)
{
    const DevState* st = a.st;
    if (a.mode != 3 && st->done) return;
    if (a.mode == 3 && (!st->done || st->status < 0 || st->exch_timeout)) return;
    constexpr int BM = kLrBM, BN = kLstepBN;
    using G = LrGemm<BM, BN, false, true>;
    __shared__ float As[BM][kLrBK + 1];
    __shared__ float Bs[kLrBK][BN + 1];
    __shared__ float Ls[BM][BN + 4];
    __shared__ double red[kLrTPB / 64];
    G g{As, Bs};
    lr_f32x4 acc[G::FM][G::FN];
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    g.run(a.A, a.R, a.V, a.R, a.m, a.n, m0, n0, 0, a.R, acc);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * G::WM, wn = (wave & 1) * G::WN;
#pragma unroll
    for (int i = 0; i < G::FM; ++i)
#pragma unroll
        for (int j = 0; j < G::FN; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) Ls[wm + 16 * i + 4 * (lane >> 4) + e][wn + 16 * j + (lane & 15)] = acc[i][j][e];
    __syncthreads();
    const float lam = (float)st->lambda;
    double acc2 = 0.0;
    if (a.mode == 3) {
        // S_{K+1} = P_ST_{lambda/mu_K}(M - L_{K+1} + Y_K / mu_K)
        const float t = (float)(st->lambda / st->mu_prev), imu = (float)(1.0 / st->mu_prev);
        for (int e = tid; e < BM * BN; e += kLrTPB) {
            const int i = e / BN, j = e % BN;
            const int gi = m0 + i, gj = n0 + j;
            if (gi >= a.m || gj >= a.n) continue;
            const float y = a.Yprev ? a.Yprev[(int64_t)gi * a.ldy + gj] : 0.f;
            const float Rr = a.M[(int64_t)gi * a.ldm + gj] - Ls[i][j] + y * imu;
            const float p = Rr - t, q = Rr + t;
            a.S[(int64_t)gi * a.lds + gj] = (p > 0.f ? p : 0.f) + (q < 0.f ? q : 0.f);
        }
        return;
    }
    const float mu_prev = (float)st->mu_prev;
    const float imu_prev = (float)(1.0 / st->mu_prev);
    const float imu_cur = (float)(1.0 / st->mu);
    for (int e = tid; e < BM * BN; e += kLrTPB) {
        const int i = e / BN, j = e % BN;
        const int gi = m0 + i, gj = n0 + j;
        if (gi >= a.m || gj >= a.n) continue;
        const float yp = (a.mode == 2) ? a.Yprev[(int64_t)gi * a.ldy + gj] : 0.f;
        const float l = Ls[i][j];
        const float Rr = a.M[(int64_t)gi * a.ldm + gj] - l + yp * imu_prev;
        const float y = fminf(fmaxf(mu_prev * Rr, -lam), lam);
        const float dy = y - yp;
        acc2 += (double)(dy * dy);
        a.Ynext[(int64_t)gi * a.ldy + gj] = y;
        a.X[(int64_t)gi * a.ldx + gj] = l + dy * imu_prev + y * imu_cur;
    }
    for (int off = 32; off > 0; off >>= 1) acc2 += __shfl_xor(acc2, off, 64);
    if (lane == 0) red[wave] = acc2;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < kLrTPB / 64; ++w) t += red[w];
        a.dy2part[blockIdx.y * gridDim.x + blockIdx.x] = t;
    }
}

// ||M||_F^2 partials (iteration 1, whose L-step input is M itself).
__global__ void lr_norm_kernel(const float* M, int64_t ldm, int m, int n, double* part)
{
    __shared__ double red[kLrTPB / 64];
    double s = 0.0;
    for (int i = blockIdx.x; i < m; i += gridDim.x)
        for (int j = threadIdx.x; j < n; j += kLrTPB) {
            const double v = M[(int64_t)i * ldm + j];
            s = fma(v, v, s);
        }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kLrTPB / 64; ++w) t += red[w];
        part[blockIdx.x] = t;
    }
}

// ---------------------------------------------------------------------------
// FP64 Gram G = C^T C of an FP32 K x N matrix C (ldc), split over rows:
// workgroup (bx, by, z) owns the 32 x 32 tile (by, bx) over rows of split z.
// Rows and columns >= r are the identity block (after the sum).
__global__ void __launch_bounds__(256) lr_gram_kernel(const float* C, int64_t ldc, int K, int N, int kc,
                                                      double* part, const DevState* st)
{
    if (st && st->done) return;
    __shared__ double Ls[32][kT64 + 1], Rs[32][kT64 + 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int i0 = blockIdx.y * kT64, j0 = blockIdx.x * kT64;
    const int kbeg = blockIdx.z * kc, kend = min(K, kbeg + kc);
    double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int k0 = kbeg; k0 < kend; k0 += 32) {
        for (int e = threadIdx.x; e < 32 * kT64; e += 256) {
            const int kk = e / kT64, c = e % kT64;
            const int gk = k0 + kk;
            Ls[kk][c] = (gk < kend && i0 + c < N) ? (double)C[(int64_t)gk * ldc + i0 + c] : 0.0;
            Rs[kk][c] = (gk < kend && j0 + c < N) ? (double)C[(int64_t)gk * ldc + j0 + c] : 0.0;
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < 32; ++kk) {
            const double l0 = Ls[kk][2 * ty], l1 = Ls[kk][2 * ty + 1];
            const double r0 = Rs[kk][2 * tx], r1 = Rs[kk][2 * tx + 1];
            acc[0][0] = fma(l0, r0, acc[0][0]);
            acc[0][1] = fma(l0, r1, acc[0][1]);
            acc[1][0] = fma(l1, r0, acc[1][0]);
            acc[1][1] = fma(l1, r1, acc[1][1]);
        }
        __syncthreads();
    }
    double* P = part + (size_t)blockIdx.z * N * N;
    for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v) {
            const int i = i0 + 2 * ty + u, j = j0 + 2 * tx + v;
            if (i < N && j < N) P[(size_t)i * N + j] = acc[u][v];
        }
}

__global__ void lr_gram_sum_kernel(const double* part, int S, int N, int r, double* G, const DevState* st)
{
    if (st && st->done) return;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N * N) return;
    const int i = e / N, j = e % N;
    double s = 0.0;
    for (int z = 0; z < S; ++z) s += part[(size_t)z * N * N + e];
    G[e] = (i >= r || j >= r) ? (i == j ? 1.0 : 0.0) : s;
}

// ---------------------------------------------------------------------------
// FP64 R x R products of the r x r algebra.  One launch computes one or two
// products (blockIdx.z), C = alpha * op(A) op(B) (op: transpose if the flag
// is set); epilogues:
//   kPlain    C = alpha A B, and Cf = (float) C if Cf != NULL
//   kNsT      T = 1.5 I - 0.5 (A B) and the tile's ||A B - I||_F^2 partial
enum { kPlain = 0, kNsT = 1 };

struct Prod64 {
    const double* A;
    const double* B;
    double* C;
    float* Cf;
    int ta, tb;
    double alpha;
};

struct Gate64 {
    const DevState* st;
    const LrState* ls;
    int which, iter;    // Newton-Schulz gating: skip if instance `which` converged before `iter`
};

__device__ __forceinline__ bool gate_closed(const Gate64& g)
{
    if (g.st && g.st->done) return true;
    if (g.ls && g.ls->ns_done_at[g.which] < g.iter) return true;
    return false;
}

typedef double lr_f64x4 __attribute__((ext_vector_type(4)));
constexpr int kT64K = 64;   // K depth of one LDS stage of the FP64 products

// One 32 x 32 tile of op(A) op(B) (R x R, FP64) on v_mfma_f64_16x16x4_f64:
// wavefront w of the workgroup owns the 16 x 16 quadrant (w / 2, w % 2).
// The instruction takes A[l % 16][l / 16] and B[l / 16][l % 16] from lane l
// (as the FP32 one does) but returns D[l / 16 + 4 e][l % 16] in its e-th
// register (checked on the device: the FP32 16x16x4 form returns
// D[4 (l / 16) + e][l % 16] instead).  K is staged through LDS
// in chunks of 64, all of a chunk's loads in flight at once.
__device__ __forceinline__ void tile64(const double* __restrict__ A, int ta, const double* __restrict__ B, int tb,
                                       int N, int i0, int j0, double (*As)[kT64K + 1], double (*Bs)[kT64 + 1],
                                       lr_f64x4& acc)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int qi = 16 * (wave >> 1), qj = 16 * (wave & 1);
    acc = lr_f64x4{0.0, 0.0, 0.0, 0.0};
    constexpr int NL = kT64 * kT64K / 256;   // loads per thread per operand and chunk
    for (int k0 = 0; k0 < N; k0 += kT64K) {
        double va[NL], vb[NL];
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            const int e = tid + 256 * u;
            // A: row i (of 32), column k (of 64); consecutive threads take the
            // contiguous index of the stored layout
            int i, k;
            if (ta) { k = e / kT64; i = e % kT64; } else { i = e / kT64K; k = e % kT64K; }
            const int gi = i0 + i, gk = k0 + k;
            va[u] = (gi < N && gk < N) ? (ta ? A[(size_t)gk * N + gi] : A[(size_t)gi * N + gk]) : 0.0;
            int kb, j;
            if (tb) { j = e / kT64K; kb = e % kT64K; } else { kb = e / kT64; j = e % kT64; }
            const int gj = j0 + j, gkb = k0 + kb;
            vb[u] = (gj < N && gkb < N) ? (tb ? B[(size_t)gj * N + gkb] : B[(size_t)gkb * N + gj]) : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NL; ++u) {
            const int e = tid + 256 * u;
            int i, k;
            if (ta) { k = e / kT64; i = e % kT64; } else { i = e / kT64K; k = e % kT64K; }
            As[i][k] = va[u];
            int kb, j;
            if (tb) { j = e / kT64K; kb = e % kT64K; } else { kb = e / kT64; j = e % kT64; }
            Bs[kb][j] = vb[u];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kT64K; kk += 4)
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(As[qi + (lane & 15)][kk + (lane >> 4)],
                                                      Bs[kk + (lane >> 4)][qj + (lane & 15)], acc, 0, 0, 0);
    }
}

template <int MODE>
__global__ void __launch_bounds__(256) lr_gemm64_kernel(Prod64 p0, Prod64 p1, int N, Gate64 gate, double* part)
{
    if (gate_closed(gate)) return;
    const Prod64& p = blockIdx.z == 0 ? p0 : p1;
    __shared__ double As[kT64][kT64K + 1], Bs[kT64K][kT64 + 1];
    __shared__ double red[4];
    const int i0 = blockIdx.y * kT64, j0 = blockIdx.x * kT64;
    lr_f64x4 acc;
    tile64(p.A, p.ta, p.B, p.tb, N, i0, j0, As, Bs, acc);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double r2 = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int i = i0 + 16 * (wave >> 1) + (lane >> 4) + 4 * e, j = j0 + 16 * (wave & 1) + (lane & 15);
        if (i >= N || j >= N) continue;
        const double w = p.alpha * acc[e];
        if constexpr (MODE == kNsT) {
            const double d = w - (i == j ? 1.0 : 0.0);
            r2 = fma(d, d, r2);
            p.C[(size_t)i * N + j] = (i == j ? 1.5 : 0.0) - 0.5 * w;
        } else {
            p.C[(size_t)i * N + j] = w;
            if (p.Cf) p.Cf[(size_t)i * N + j] = (float)w;
        }
    }
    if constexpr (MODE == kNsT) {
        for (int off = 32; off > 0; off >>= 1) r2 += __shfl_xor(r2, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r2;
        __syncthreads();
        if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
    }
}

// B = Sym(T) = (T + T^T) / 2 on the leading r x r block, identity on the
// padded block.
__global__ void lr_sym_kernel(const double* T, double* B, int N, const DevState* st)
{
    if (st->done) return;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N * N) return;
    const int i = e / N, j = e % N, r = st->r;
    B[e] = (i < r && j < r) ? 0.5 * (T[(size_t)i * N + j] + T[(size_t)j * N + i]) : (i == j ? 1.0 : 0.0);
}

// Newton-Schulz start (one workgroup): the scale s is 1.25 times a
// power-iteration estimate of lambda_max of the leading r x r block (8 steps
// of x <- A x / ||A x|| from the normalised ones vector; ||A x|| approaches
// lambda_max from below, so A / s keeps its spectrum inside the iteration's
// (0, 2) convergence region as long as the estimate is above 0.63
// lambda_max).  Y_0 = A / s there and the identity on the padded block (a
// fixed point of the iteration), Z_0 = I.
constexpr int kPowerSteps = 8;
constexpr double kPowerMargin = 1.25;

__global__ void __launch_bounds__(1024) lr_ns_init_kernel(const double* A, int N, double* Y0, double* Z0,
                                                          DevState* st, LrState* ls, int which)
{
    if (st->done) return;
    __shared__ double red[16];
    __shared__ double x[kMaxRLarge];
    __shared__ double nrm;
    const int r = st->r, tid = threadIdx.x;
    auto block_sum = [&](double v) -> double {
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        __syncthreads();
        if ((tid & 63) == 0) red[tid >> 6] = v;
        __syncthreads();
        double t = 0.0;
        for (int w = 0; w < 16; ++w) t += red[w];
        return t;
    };
    // non-finite entries make the estimate non-finite: reported below
    for (int i = tid; i < r; i += 1024) x[i] = 1.0 / sqrt((double)r);
    __syncthreads();
    double lam = 0.0;
    for (int it = 0; it < kPowerSteps; ++it) {
        double y = 0.0;
        if (tid < r) {   // y_i = sum_j A_ji x_j (A symmetric): coalesced over i
            double y1 = 0.0, y2 = 0.0, y3 = 0.0;
            int j = 0;
            for (; j + 3 < r; j += 4) {
                y = fma(A[(size_t)j * N + tid], x[j], y);
                y1 = fma(A[(size_t)(j + 1) * N + tid], x[j + 1], y1);
                y2 = fma(A[(size_t)(j + 2) * N + tid], x[j + 2], y2);
                y3 = fma(A[(size_t)(j + 3) * N + tid], x[j + 3], y3);
            }
            for (; j < r; ++j) y = fma(A[(size_t)j * N + tid], x[j], y);
            y = (y + y1) + (y2 + y3);
        }
        const double s2 = block_sum(tid < r ? y * y : 0.0);
        lam = sqrt(s2);
        if (!(lam > 0.0) || !isfinite(lam)) break;
        if (tid < r) x[tid] = y / lam;
        __syncthreads();
    }
    if (!(lam > 0.0) || !isfinite(lam)) {
        if (tid == 0) {
            st->status = kErrNonFinite;
            st->iters = st->k - 1;
            st->done = 1;
        }
        return;
    }
    const double sc = kPowerMargin * lam;
    const double inv = 1.0 / sc;
    for (int e = tid; e < N * N; e += 1024) {
        const int i = e / N, j = e % N;
        const double id = (i == j) ? 1.0 : 0.0;
        Y0[e] = (i < r && j < r) ? A[e] * inv : id;
        Z0[e] = id;
    }
    if (tid == 0) {
        ls->ns_scale[which] = sc;
        ls->ns_done_at[which] = INT_MAX;
        ls->ns_used[which] = 0;
    }
}

// Newton-Schulz update of iteration j: (Y, Z) in parity j & 1 -> Y T, T Z in
// parity (j + 1) & 1.  Every workgroup adds the residual partials of
// iteration j (fixed order, so all take the same decision); at
// ||Z Y - I||_F <= kNsTol this is the last update, recorded by workgroup 0.
__global__ void __launch_bounds__(256) lr_ns_update_kernel(const double* Yc, const double* Zc, const double* T,
                                                           double* Yn, double* Zn, int N, const double* part,
                                                           int nparts, Gate64 gate, LrState* ls)
{
    if (gate_closed(gate)) return;
    __shared__ int conv;
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int b = 0; b < nparts; ++b) s += part[b];
        conv = (sqrt(s) <= kNsTol) ? 1 : 0;
    }
    __syncthreads();
    const bool last = conv != 0;
    // product: z = 0: Yn = Yc T; z = 1: Zn = T Zc
    const double* A = blockIdx.z == 0 ? Yc : T;
    const double* B = blockIdx.z == 0 ? T : Zc;
    double* C = blockIdx.z == 0 ? Yn : Zn;
    __shared__ double As[kT64][kT64K + 1], Bs[kT64K][kT64 + 1];
    const int i0 = blockIdx.y * kT64, j0 = blockIdx.x * kT64;
    lr_f64x4 acc;
    tile64(A, 0, B, 0, N, i0, j0, As, Bs, acc);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int i = i0 + 16 * (wave >> 1) + (lane >> 4) + 4 * e, j = j0 + 16 * (wave & 1) + (lane & 15);
        if (i < N && j < N) C[(size_t)i * N + j] = acc[e];
    }
    if (last && blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0) {
        ls->ns_done_at[gate.which] = gate.iter;
        ls->ns_used[gate.which] = gate.iter + 1;
    }
}

// One workgroup's product C = A B of R x R FP64 matrices (the fallback
// Newton-Schulz iterations).
__device__ void wg_prod64(const double* A, const double* B, double* C, int N)
{
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
        const int i = e / N, j = e % N;
        double s = 0.0;
        for (int k = 0; k < N; ++k) s = fma(A[(size_t)i * N + k], B[(size_t)k * N + j], s);
        C[e] = s;
    }
}

// Finish instance `which`: C = Z_final / sqrt(s).  If the queued iterations
// did not converge, continue in this workgroup for up to kNsMore more (R <=
// kNsMoreMaxR), and fail with SFR_ERR_RANK (the Gram is numerically
// singular: eq. (7) has no unique projector) if that does not converge
// either.
__global__ void __launch_bounds__(1024) lr_ns_finish_kernel(double* Yb0, double* Zb0, double* Yb1, double* Zb1,
                                                            double* T, int N, double* C, DevState* st, LrState* ls,
                                                            int which, int queued)
{
    if (st->done) return;
    __shared__ int conv;
    __shared__ double red[16];
    int fin;
    if (ls->ns_done_at[which] != INT_MAX) {
        fin = (ls->ns_done_at[which] + 1) & 1;
    } else {
        double* Y[2] = {Yb0, Yb1};
        double* Z[2] = {Zb0, Zb1};
        int j = queued;   // (Y, Z) of iteration `queued` are in parity queued & 1
        bool ok = false;
        const int more = (N <= kNsMoreMaxR) ? kNsMore : 0;
        for (int it = 0; it < more; ++it, ++j) {
            const int c = j & 1, nx = (j + 1) & 1;
            wg_prod64(Z[c], Y[c], T, N);                  // W = Z Y
            __syncthreads();
            double r2 = 0.0;
            for (int e = threadIdx.x; e < N * N; e += 1024) {
                const double w = T[e], d = w - ((e / N == e % N) ? 1.0 : 0.0);
                r2 = fma(d, d, r2);
                T[e] = ((e / N == e % N) ? 1.5 : 0.0) - 0.5 * w;
            }
            for (int off = 32; off > 0; off >>= 1) r2 += __shfl_xor(r2, off, 64);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r2;
            __syncthreads();
            if (threadIdx.x == 0) {
                double s = 0.0;
                for (int w = 0; w < 16; ++w) s += red[w];
                conv = (sqrt(s) <= kNsTol) ? 1 : (isfinite(s) ? 0 : -1);
            }
            __syncthreads();
            if (conv < 0) break;
            wg_prod64(Y[c], T, Y[nx], N);
            wg_prod64(T, Z[c], Z[nx], N);
            __syncthreads();
            if (conv) { ok = true; ++j; break; }
        }
        if (!ok) {
            if (threadIdx.x == 0) {
                st->status = kErrRank;
                st->iters = st->k - 1;
                st->done = 1;
            }
            return;
        }
        fin = j & 1;
        if (threadIdx.x == 0) ls->ns_used[which] = j;
    }
    const double* Zf = fin ? Zb1 : Zb0;
    const double sc = 1.0 / sqrt(ls->ns_scale[which]);
    const int r = st->r;
    for (int e = threadIdx.x; e < N * N; e += 1024) {
        const int i = e / N, j = e % N;
        C[e] = (i < r && j < r) ? Zf[e] * sc : (i == j ? 1.0 : 0.0);
    }
}

// ---------------------------------------------------------------------------
// Start of step k: the convergence test of iteration k - 1 (or ||M||_F at
// k = 1), as in the fused path's step.
__global__ void __launch_bounds__(256) lr_step_begin_kernel(DevState* st, const double* dy2part, int ndy,
                                                            double* res_hist)
{
    if (st->done) return;
    __shared__ double red[4];
    double s = 0.0;
    for (int e = threadIdx.x; e < ndy; e += 256) s += dy2part[e];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double total = red[0] + red[1] + red[2] + red[3];
    const int k = st->k;
    if (k == 1) {
        const double nrm = sqrt(total);
        st->nrmM = nrm;
        if (!(nrm > 0.0) || !isfinite(nrm)) { st->status = kErrNonFinite; st->iters = 0; st->done = 1; }
        return;
    }
    if (st->tsvd) return;
    const double res = sqrt(total) / (st->mu_prev * st->nrmM);
    const int kdone = k - 1;
    bool stop = false;
    int32_t status = kOK;
    if (!isfinite(res)) { stop = true; status = kErrNonFinite; }
    else if (st->fixed_iters > 0) { stop = kdone >= st->fixed_iters; }
    else if (res <= st->tol) { stop = true; }
    else if (kdone >= st->max_iter) { stop = true; status = kWarnMaxIter; }
    res_hist[kdone - 1] = res;
    st->res = res;
    if (stop) { st->status = status; st->iters = kdone; st->done = 1; }
}

// End of step k: continuation (FR-ADM), or the change-of-B stopping rule
// (Alg. 4), then k + 1.
__global__ void __launch_bounds__(1024) lr_step_end_kernel(DevState* st, const double* Bnew, const double* Bold,
                                                           int N, double* res_hist)
{
    if (st->done) return;
    const int k = st->k;
    if (st->tsvd) {
        __shared__ double red[2][16];
        double d2 = 0.0, n2 = 0.0;
        const int r = st->r;
        for (int e = threadIdx.x; e < N * N; e += 1024) {
            if (e / N >= r || e % N >= r) continue;
            const double d = Bnew[e] - Bold[e];
            d2 = fma(d, d, d2);
            n2 = fma(Bnew[e], Bnew[e], n2);
        }
        for (int off = 32; off > 0; off >>= 1) {
            d2 += __shfl_xor(d2, off, 64);
            n2 += __shfl_xor(n2, off, 64);
        }
        if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = d2; red[1][threadIdx.x >> 6] = n2; }
        __syncthreads();
        if (threadIdx.x != 0) return;
        d2 = 0.0; n2 = 0.0;
        for (int w = 0; w < 16; ++w) { d2 += red[0][w]; n2 += red[1][w]; }
        const double res = sqrt(d2 / n2);
        bool stop = false;
        int32_t status = kOK;
        if (!isfinite(res)) { stop = true; status = kErrNonFinite; }
        else if (st->fixed_iters > 0) { stop = k >= st->fixed_iters; }
        else if (res <= st->tol) { stop = true; }
        else if (k >= st->max_iter) { stop = true; status = kWarnMaxIter; }
        res_hist[k - 1] = res;
        st->res = res;
        st->k = k + 1;
        if (stop) { st->status = status; st->iters = k; st->done = 1; }
        return;
    }
    if (threadIdx.x != 0) return;
    const double mu = st->mu;
    st->mu_prev = mu;
    const double nm = st->rho * mu;
    st->mu = nm < st->mu_bar ? nm : st->mu_bar;
    st->k = k + 1;
}

// ---------------------------------------------------------------------------
// Extreme eigenvalues of the leading r x r block of a symmetric matrix:
// Householder reduction to tridiagonal form (in `W`, r x r workspace; the
// reflector v and the vector p of each step in LDS), then Sturm-sequence
// multisection for the smallest and largest eigenvalue: every thread counts
// the eigenvalues below its own point of the bracket, so each round shrinks
// the bracket 1024-fold.
__device__ int sturm_below(const double* d, const double* e2, int n, double x)
{
    // eigenvalues of the tridiagonal (d, e) below x: negative pivots of the
    // LDL^T factorisation of T - x I
    int c = 0;
    double q = 1.0;
    for (int i = 0; i < n; ++i) {
        q = d[i] - x - ((i > 0) ? e2[i - 1] / q : 0.0);
        if (q == 0.0) q = -1e-300;
        c += (q < 0.0);
    }
    return c;
}

__global__ void __launch_bounds__(kEigTPB) lr_extreme_eig_kernel(const double* B, int N, int r, double* W,
                                                                 double* vec, DevState* st, int want_min,
                                                                 int want_max)
{
    if (!st->done || st->status < 0 || st->exch_timeout) return;
    double* part = vec;   // 16 x n partial sums of the tridiagonalisation's products
    __shared__ double red[kEigTPB / 64];
    __shared__ double v[kMaxRLarge], p[kMaxRLarge], d[kMaxRLarge], e2[kMaxRLarge];
    __shared__ double lohi[2];
    __shared__ int bracket;
    const int tid = threadIdx.x, n = r;
    for (int x = tid; x < n * n; x += kEigTPB) W[x] = B[(size_t)(x / n) * N + x % n];
    __syncthreads();
    auto block_sum = [&](double s) -> double {
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
        __syncthreads();
        if ((tid & 63) == 0) red[tid >> 6] = s;
        __syncthreads();
        double t = 0.0;
        for (int w = 0; w < kEigTPB / 64; ++w) t += red[w];
        return t;
    };
    for (int k = 0; k + 2 < n; ++k) {
        const int len = n - k - 1;   // trailing block: rows and columns k+1 .. n-1
        double s = 0.0;
        for (int i = tid; i < len; i += kEigTPB) {
            const double x = W[(size_t)(k + 1 + i) * n + k];
            s = fma(x, x, s);
        }
        const double nx = sqrt(block_sum(s));
        const double x0 = W[(size_t)(k + 1) * n + k];
        const double alpha = (x0 >= 0.0) ? -nx : nx;
        // v = (x - alpha e1) / ||x - alpha e1|| (no reflection if x is already along e1)
        const double v0 = x0 - alpha;
        const double vn2 = nx * nx - x0 * x0 + v0 * v0;
        const bool reflect = vn2 > 0.0 && nx > 0.0;
        const double vinv = reflect ? 1.0 / sqrt(vn2) : 0.0;
        for (int i = tid; i < len; i += kEigTPB) v[i] = (i == 0 ? v0 : W[(size_t)(k + 1 + i) * n + k]) * vinv;
        if (tid == 0) {
            d[k] = W[(size_t)k * n + k];
            const double ek = reflect ? alpha : x0;
            e2[k] = ek * ek;
        }
        __syncthreads();
        if (!reflect) continue;
        // p = 2 A_sub v (A_sub symmetric): wavefront w sums the rows
        // j = w, w + 16, ... for the columns i = lane + 64 c (consecutive
        // lanes on consecutive entries of a row, every load independent);
        // the 16 partial vectors go through `part` and are added in order
        {
            const int wv = tid >> 6, ln = tid & 63;
            const int nch = (len + 63) >> 6;
            double acc[kMaxRLarge / 64];
#pragma unroll
            for (int c = 0; c < kMaxRLarge / 64; ++c) acc[c] = 0.0;
            for (int j = wv; j < len; j += kEigTPB / 64) {
                const double* row = W + (size_t)(k + 1 + j) * n + (k + 1);
                const double vj = v[j];
#pragma unroll
                for (int c = 0; c < kMaxRLarge / 64; ++c) {
                    const int i = ln + 64 * c;
                    if (c < nch && i < len) acc[c] = fma(row[i], vj, acc[c]);
                }
            }
#pragma unroll
            for (int c = 0; c < kMaxRLarge / 64; ++c) {
                const int i = ln + 64 * c;
                if (c < nch && i < len) part[(size_t)wv * n + i] = acc[c];
            }
            __syncthreads();
            for (int i = tid; i < len; i += kEigTPB) {
                double q = 0.0;
                for (int w = 0; w < kEigTPB / 64; ++w) q += part[(size_t)w * n + i];
                p[i] = 2.0 * q;
            }
            __syncthreads();
        }
        double vp = 0.0;
        for (int i = tid; i < len; i += kEigTPB) vp = fma(v[i], p[i], vp);
        vp = block_sum(vp);
        for (int i = tid; i < len; i += kEigTPB) p[i] -= vp * v[i];   // w
        __syncthreads();
        // A_sub -= v w^T + w v^T: wavefront w on the rows i = w, w + 16, ...,
        // consecutive lanes on consecutive columns
        {
            const int wv = tid >> 6, ln = tid & 63;
            for (int i = wv; i < len; i += kEigTPB / 64) {
                const double vi = v[i], wi = p[i];
                double* row = W + (size_t)(k + 1 + i) * n + (k + 1);
                for (int j = ln; j < len; j += 64) row[j] -= vi * p[j] + wi * v[j];
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        if (n >= 2) {
            d[n - 2] = W[(size_t)(n - 2) * n + (n - 2)];
            const double en = W[(size_t)(n - 1) * n + (n - 2)];
            e2[n - 2] = en * en;
        }
        d[n - 1] = W[(size_t)(n - 1) * n + (n - 1)];
        // Gershgorin bracket of the whole spectrum
        double lo = INFINITY, hi = -INFINITY;
        for (int i = 0; i < n; ++i) {
            const double rad = (i > 0 ? sqrt(e2[i - 1]) : 0.0) + (i + 1 < n ? sqrt(e2[i]) : 0.0);
            lo = fmin(lo, d[i] - rad);
            hi = fmax(hi, d[i] + rad);
        }
        const double pad = 1e-12 * fmax(fabs(lo), fabs(hi)) + 1e-300;
        lohi[0] = lo - pad;
        lohi[1] = hi + pad;
    }
    __syncthreads();
    // the eigenvalue with `target` eigenvalues below it, by multisection:
    // thread t evaluates the count at a + (t + 1) (b - a) / (T + 1)
    auto kth = [&](int target) -> double {
        double a = lohi[0], b = lohi[1];
        for (int round = 0; round < 8; ++round) {
            const double h = (b - a) / (double)(kEigTPB + 1);
            if (!(h > 0.0)) break;
            if (tid == 0) bracket = kEigTPB;   // first point with more than `target` below
            __syncthreads();
            const double x = a + h * (double)(tid + 1);
            if (sturm_below(d, e2, n, x) > target) atomicMin(&bracket, tid);
            __syncthreads();
            const int t = bracket;
            const double na = (t == 0) ? a : a + h * (double)t;
            const double nb = (t == kEigTPB) ? b : a + h * (double)(t + 1);
            __syncthreads();
            if (nb - na >= b - a) break;
            a = na;
            b = nb;
        }
        return 0.5 * (a + b);
    };
    double wmin = 0.0, wmax = 0.0;
    if (want_min) wmin = kth(0);
    if (want_max) wmax = kth(n - 1);
    if (tid == 0) {
        if (want_min) st->min_eig_B = wmin;
        if (want_max) st->max_eig_B = wmax;
    }
}

}  // namespace sfr

// ---------------------------------------------------------------------------
// Host side: the large-rank engine.
namespace sfr {

__global__ void lr_identity_kernel(double* A, int N)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < N * N) A[e] = (e / N == e % N) ? 1.0 : 0.0;
}

// V_1 = I_{n x r} padded to R columns (rows >= r zero).
__global__ void lr_v1_kernel(float* V1, int n, int r, int R)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * R) return;
    const int i = (int)(e / R), j = (int)(e % R);
    V1[e] = (i == j && j < r) ? 1.f : 0.f;
}

// The leading r x r block of the R x R B of the returned iterate.
__global__ void lr_copy_b_kernel(const double* Bk, int R, int r, double* B, const DevState* st)
{
    if (!st->done || st->status < 0 || st->exch_timeout) return;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < r * r) B[e] = Bk[(size_t)(e / r) * R + e % r];
}

// orth_err = max(||G_U - I||_F, ||G_V - I||_F) from the two r x r Grams.
__global__ void __launch_bounds__(256) lr_orth_dist_kernel(const double* GU, const double* GV, int r, DevState* st)
{
    if (!st->done || st->status < 0 || st->exch_timeout) return;
    __shared__ double red[2][4];
    double su = 0.0, sv = 0.0;
    for (int e = threadIdx.x; e < r * r; e += 256) {
        const double id = (e / r == e % r) ? 1.0 : 0.0;
        const double du = GU[e] - id, dv = GV[e] - id;
        su = fma(du, du, su);
        sv = fma(dv, dv, sv);
    }
    for (int off = 32; off > 0; off >>= 1) {
        su += __shfl_xor(su, off, 64);
        sv += __shfl_xor(sv, off, 64);
    }
    if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = su; red[1][threadIdx.x >> 6] = sv; }
    __syncthreads();
    if (threadIdx.x == 0)
        st->orth_err = fmax(sqrt(red[0][0] + red[0][1] + red[0][2] + red[0][3]),
                            sqrt(red[1][0] + red[1][1] + red[1][2] + red[1][3]));
}

struct LrPlan {
    int S = 1, kc = 0;   // split count and K chunk
};

struct LrEngine {
    int m = 0, n = 0, r = 0, R = 0, hist_len = 0;
    LrPlan pP, pQ, gP, gQ, gU, gV;
    float* Y[2] = {nullptr, nullptr};
    float* X = nullptr;
    float* P[2] = {nullptr, nullptr};
    float* Q[2] = {nullptr, nullptr};
    float* Ak = nullptr;
    float* Vk = nullptr;
    float* V1 = nullptr;
    float* part = nullptr;
    double* gpart = nullptr;
    double* dy2part = nullptr;
    int ndy = 1;
    double *Gp = nullptr, *Gq = nullptr;
    double* B[2] = {nullptr, nullptr};
    double* TU[2] = {nullptr, nullptr};
    double* TUbar[2] = {nullptr, nullptr};
    double* TV[2] = {nullptr, nullptr};
    float* TUf[2] = {nullptr, nullptr};
    float* TUbarf[2] = {nullptr, nullptr};
    float* TVf[2] = {nullptr, nullptr};
    double *A1 = nullptr, *C1 = nullptr, *Km = nullptr, *A2 = nullptr, *C2 = nullptr, *T0 = nullptr, *T1 = nullptr;
    double* NY[2] = {nullptr, nullptr};
    double* NZ[2] = {nullptr, nullptr};
    double *NT = nullptr, *nspart = nullptr;
    double *eigW = nullptr, *eigv = nullptr;
    DevState* st = nullptr;
    LrState* ls = nullptr;
    double* res_hist = nullptr;
    DevState* host_state = nullptr;
    DevState* host_poll = nullptr;
    hipEvent_t poll_ev[2] = {nullptr, nullptr};
    std::vector<void*> allocs;
    size_t bytes = 0;
};

#define LRCHK(x)                                   \
    do {                                           \
        if ((x) != hipSuccess) {                   \
            (void)hipGetLastError();               \
            return SFR_ERR_DEVICE;                 \
        }                                          \
    } while (0)

static int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Split of a K-long GEMM with `tiles` output tiles: enough splits to put
// about two workgroups on every CU, each split at least 256 deep.
static LrPlan split_plan(int64_t K, int tiles, int cus)
{
    LrPlan p;
    const int want = std::max(1, cdiv(2 * cus, tiles));
    p.S = std::max(1, std::min({want, 32, (int)std::max<int64_t>(1, K / 256)}));
    p.kc = ((cdiv(K, p.S) + kLrBK - 1) / kLrBK) * kLrBK;
    p.S = cdiv(K, p.kc);
    return p;
}

static LrPlan gram_plan(int64_t K, int R, int cus)
{
    LrPlan p;
    const int tiles = cdiv(R, kT64) * cdiv(R, kT64);
    const int want = std::max(1, cdiv(cus, tiles));
    p.S = std::max(1, std::min({want, 64, (int)std::max<int64_t>(1, K / 64)}));
    p.kc = ((cdiv(K, p.S) + 31) / 32) * 32;
    p.S = cdiv(K, p.kc);
    return p;
}

static int bn_of(int N) { return N <= 64 ? 64 : 128; }

// C = A B (FP32, MFMA), split over K into `part` when plan.S > 1.
static hipError_t lr_gemm(const float* A, int64_t lda, bool at, const float* B, int64_t ldb, bool bt, float* C,
                          int64_t ldc, int M, int N, int K, const LrPlan& plan, float* part, const DevState* st,
                          hipStream_t s)
{
    const int BN = bn_of(N);
    const bool split = plan.S > 1;
    float* out = split ? part : C;
    const int64_t ldo = split ? N : ldc;
    const int64_t zs = (int64_t)M * N;
    dim3 grid((unsigned)cdiv(N, BN), (unsigned)cdiv(M, kLrBM), (unsigned)plan.S);
    const int kc = split ? plan.kc : ((K + kLrBK - 1) / kLrBK) * kLrBK;
#define GO(bn, AT_, BT_) \
    hipLaunchKernelGGL((lr_gemm_kernel<bn, AT_, BT_>), grid, dim3(kLrTPB), 0, s, A, lda, B, ldb, out, ldo, zs, M, N, K, kc, st)
    if (BN == 64) {
        if (at) { if (bt) GO(64, true, true); else GO(64, true, false); }
        else { if (bt) GO(64, false, true); else GO(64, false, false); }
    } else {
        if (at) { if (bt) GO(128, true, true); else GO(128, true, false); }
        else { if (bt) GO(128, false, true); else GO(128, false, false); }
    }
#undef GO
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !split) return e;
    // the partials are dense M x N; C may have a leading dimension: N == ldc here
    const int64_t cnt = (int64_t)M * N;
    hipLaunchKernelGGL(lr_splitk_sum_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, part, zs, plan.S,
                       C, cnt, st);
    return hipGetLastError();
}

// G = C^T C in FP64 (C: K x N FP32, ldc), identity outside the leading r x r block.
static hipError_t lr_gram(const float* C, int64_t ldc, int K, int N, int r, const LrPlan& plan, double* gpart,
                          double* G, const DevState* st, hipStream_t s)
{
    dim3 grid((unsigned)cdiv(N, kT64), (unsigned)cdiv(N, kT64), (unsigned)plan.S);
    hipLaunchKernelGGL(lr_gram_kernel, grid, dim3(256), 0, s, C, ldc, K, N, plan.kc, gpart, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(lr_gram_sum_kernel, dim3((unsigned)cdiv((int64_t)N * N, 256)), dim3(256), 0, s, gpart, plan.S,
                       N, r, G, st);
    return hipGetLastError();
}

static hipError_t lr_prod(const LrEngine& e, const double* A, bool ta, const double* B, bool tb, double* C,
                          float* Cf, hipStream_t s)
{
    Prod64 p{A, B, C, Cf, ta ? 1 : 0, tb ? 1 : 0, 1.0};
    Gate64 g{e.st, nullptr, 0, 0};
    const int t = cdiv(e.R, kT64);
    hipLaunchKernelGGL(lr_gemm64_kernel<kPlain>, dim3(t, t, 1), dim3(256), 0, s, p, p, e.R, g, (double*)nullptr);
    return hipGetLastError();
}

// C = A^{-1/2} (Newton-Schulz instance `which`).
static hipError_t lr_invsqrt(const LrEngine& e, const double* A, double* C, int which, hipStream_t s)
{
    const int N = e.R, t = cdiv(N, kT64);
    hipLaunchKernelGGL(lr_ns_init_kernel, dim3(1), dim3(1024), 0, s, A, N, e.NY[0], e.NZ[0], e.st, e.ls, which);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    for (int j = 0; j < kNsIters; ++j) {
        const int c = j & 1, nx = (j + 1) & 1;
        Gate64 g{e.st, e.ls, which, j};
        Prod64 p{e.NZ[c], e.NY[c], e.NT, nullptr, 0, 0, 1.0};
        hipLaunchKernelGGL(lr_gemm64_kernel<kNsT>, dim3(t, t, 1), dim3(256), 0, s, p, p, N, g, e.nspart);
        hipLaunchKernelGGL(lr_ns_update_kernel, dim3(t, t, 2), dim3(256), 0, s, e.NY[c], e.NZ[c], e.NT, e.NY[nx],
                           e.NZ[nx], N, e.nspart, t * t, g, e.ls);
    }
    hipLaunchKernelGGL(lr_ns_finish_kernel, dim3(1), dim3(1024), 0, s, e.NY[0], e.NZ[0], e.NY[1], e.NZ[1], e.NT, N,
                       C, e.st, e.ls, which, kNsIters);
    return hipGetLastError();
}

void lr_destroy(LrEngine* e)
{
    if (!e) return;
    free_all(e->allocs);
    if (e->host_state) (void)hipHostFree(e->host_state);
    if (e->host_poll) (void)hipHostFree(e->host_poll);
    for (int b = 0; b < 2; ++b)
        if (e->poll_ev[b]) (void)hipEventDestroy(e->poll_ev[b]);
    delete e;
}

size_t lr_bytes(const LrEngine* e) { return e ? e->bytes : 0; }

sfr_status lr_create(LrEngine** out, int m, int n, int r, int hist_len)
{
    *out = nullptr;
    if (r <= kMaxR || r > kMaxRLarge || r > m || r > n) return SFR_ERR_ARG;
    LrEngine* e = new (std::nothrow) LrEngine();
    if (!e) return SFR_ERR_NOMEM;
    e->m = m; e->n = n; e->r = r;
    e->R = ((r + 15) / 16) * 16;
    e->hist_len = hist_len;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        delete e;
        return SFR_ERR_DEVICE;
    }
    const int R = e->R;
    const int bn = bn_of(R);
    e->pP = split_plan(n, cdiv(m, kLrBM) * cdiv(R, bn), cus);
    e->pQ = split_plan(m, cdiv(n, kLrBM) * cdiv(R, bn), cus);
    e->gP = gram_plan(m, R, cus);
    e->gQ = gram_plan(n, R, cus);
    e->gU = gram_plan(m, r, cus);
    e->gV = gram_plan(n, r, cus);
    e->ndy = cdiv(m, kLrBM) * cdiv(n, kLstepBN);
    const size_t mn = (size_t)m * n;
    bool ok = true;
    auto fa = [&](float** p, size_t cnt) { if (ok) ok = dev_alloc(e->allocs, e->bytes, (void**)p, cnt * 4); };
    auto da = [&](double** p, size_t cnt) { if (ok) ok = dev_alloc(e->allocs, e->bytes, (void**)p, cnt * 8); };
    for (int b = 0; b < 2; ++b) fa(&e->Y[b], mn);
    fa(&e->X, mn);
    for (int b = 0; b < 2; ++b) { fa(&e->P[b], (size_t)m * R); fa(&e->Q[b], (size_t)n * R); }
    fa(&e->Ak, (size_t)m * R);
    fa(&e->Vk, (size_t)n * R);
    fa(&e->V1, (size_t)n * R);
    const size_t pf = std::max({(size_t)(e->pP.S > 1 ? e->pP.S : 0) * m * R, (size_t)(e->pQ.S > 1 ? e->pQ.S : 0) * n * R,
                                (size_t)16});
    fa(&e->part, pf);
    const size_t gp = std::max({(size_t)e->gP.S * R * R, (size_t)e->gQ.S * R * R, (size_t)e->gU.S * r * r,
                                (size_t)e->gV.S * r * r});
    da(&e->gpart, gp);
    da(&e->dy2part, (size_t)std::max(e->ndy, 1024));
    const size_t RR = (size_t)R * R;
    da(&e->Gp, RR); da(&e->Gq, RR);
    for (int b = 0; b < 2; ++b) {
        da(&e->B[b], RR); da(&e->TU[b], RR); da(&e->TUbar[b], RR); da(&e->TV[b], RR);
        fa(&e->TUf[b], RR); fa(&e->TUbarf[b], RR); fa(&e->TVf[b], RR);
        da(&e->NY[b], RR); da(&e->NZ[b], RR);
    }
    da(&e->A1, RR); da(&e->C1, RR); da(&e->Km, RR); da(&e->A2, RR); da(&e->C2, RR); da(&e->T0, RR); da(&e->T1, RR);
    da(&e->NT, RR);
    da(&e->nspart, (size_t)cdiv(R, kT64) * cdiv(R, kT64));
    da(&e->eigW, (size_t)r * r);
    da(&e->eigv, (size_t)(kEigTPB / 64) * r);
    if (ok) ok = dev_alloc(e->allocs, e->bytes, (void**)&e->st, sizeof(DevState));
    if (ok) ok = dev_alloc(e->allocs, e->bytes, (void**)&e->ls, sizeof(LrState));
    da(&e->res_hist, (size_t)std::max(hist_len, kResHistMin) + 2);
    if (ok && hipHostMalloc((void**)&e->host_state, sizeof(DevState), hipHostMallocDefault) != hipSuccess) {
        e->host_state = nullptr;
        ok = false;
    }
    if (ok && hipHostMalloc((void**)&e->host_poll, 2 * sizeof(DevState), hipHostMallocDefault) != hipSuccess) {
        e->host_poll = nullptr;
        ok = false;
    }
    for (int b = 0; b < 2 && ok; ++b)
        if (hipEventCreateWithFlags(&e->poll_ev[b], hipEventDisableTiming) != hipSuccess) {
            e->poll_ev[b] = nullptr;
            ok = false;
        }
    if (ok) {
        hipLaunchKernelGGL(lr_v1_kernel, dim3((unsigned)cdiv((int64_t)n * R, 256)), dim3(256), 0, 0, e->V1, n, r, R);
        ok = hipGetLastError() == hipSuccess && hipDeviceSynchronize() == hipSuccess;
    }
    if (!ok) {
        (void)hipGetLastError();
        lr_destroy(e);
        return SFR_ERR_NOMEM;
    }
    *out = e;
    return SFR_OK;
}

// Step k of Alg. 1 (or of Alg. 4 with tsvd): the products, the Grams and the
// FP64 r x r algebra; every kernel returns at once once the solve is done.
static sfr_status lr_enqueue_iter(LrEngine& e, int k, const float* M, int64_t ldm, bool tsvd, hipStream_t s)
{
    const int m = e.m, n = e.n, R = e.R;
    const int b = (k - 1) & 1, nb = k & 1;
    const float* Xs;
    int64_t ldx;
    int ndy = e.ndy;
    if (k == 1 || tsvd) {
        if (k == 1) {
            const int nblk = std::min(m, 1024);
            hipLaunchKernelGGL(lr_norm_kernel, dim3(nblk), dim3(kLrTPB), 0, s, M, ldm, m, n, e.dy2part);
            LRCHK(hipGetLastError());
            ndy = nblk;
        }
        const float* Vin = e.V1;
        if (k > 1) {
            LRCHK(lr_gemm(e.Q[b], R, false, e.TVf[b], R, false, e.Vk, R, n, R, R, LrPlan{}, e.part, e.st, s));
            Vin = e.Vk;
        }
        LRCHK(lr_gemm(M, ldm, false, Vin, R, false, e.P[nb], R, m, R, n, e.pP, e.part, e.st, s));
        Xs = M;
        ldx = ldm;
    } else {
        LRCHK(lr_gemm(e.P[b], R, false, e.TUf[b], R, false, e.Ak, R, m, R, R, LrPlan{}, e.part, e.st, s));
        LRCHK(lr_gemm(e.Q[b], R, false, e.TVf[b], R, false, e.Vk, R, n, R, R, LrPlan{}, e.part, e.st, s));
        LstepArgs a;
        a.st = e.st;
        a.A = e.Ak; a.V = e.Vk; a.R = R;
        a.M = M; a.ldm = ldm;
        a.Yprev = e.Y[b]; a.ldy = n;
        a.Ynext = e.Y[nb];
        a.X = e.X; a.ldx = n;
        a.S = nullptr; a.lds = 0;
        a.dy2part = e.dy2part;
        a.m = m; a.n = n;
        a.mode = (k == 2) ? 1 : 2;
        hipLaunchKernelGGL(lr_lstep_kernel, dim3((unsigned)cdiv(n, kLstepBN), (unsigned)cdiv(m, kLrBM)), dim3(kLrTPB),
                           0, s, a);
        LRCHK(hipGetLastError());
        LRCHK(lr_gemm(e.X, n, false, e.Vk, R, false, e.P[nb], R, m, R, n, e.pP, e.part, e.st, s));
        Xs = e.X;
        ldx = n;
    }
    // Q = X^T P: A operand X stored [K = m][M = n]
    LRCHK(lr_gemm(Xs, ldx, true, e.P[nb], R, false, e.Q[nb], R, n, R, m, e.pQ, e.part, e.st, s));
    LRCHK(lr_gram(e.P[nb], R, m, R, e.r, e.gP, e.gpart, e.Gp, e.st, s));
    LRCHK(lr_gram(e.Q[nb], R, n, R, e.r, e.gQ, e.gpart, e.Gq, e.st, s));
    hipLaunchKernelGGL(lr_step_begin_kernel, dim3(1), dim3(256), 0, s, e.st, e.dy2part, ndy, e.res_hist);
    LRCHK(hipGetLastError());
    // r x r algebra (App. A.5): C1 = (B0 G_P B0)^{-1/2}, U = P B0 C1,
    // K = B0 C1 B0, C2 = (K G_Q K)^{-1/2}, V = Q K C2,
    // B = Sym(C1 B0 G_Q K C2), a_i = P_i B0 C1 B
    const double* B0 = e.B[b];
    LRCHK(lr_prod(e, B0, false, e.Gp, false, e.T0, nullptr, s));
    LRCHK(lr_prod(e, e.T0, false, B0, false, e.A1, nullptr, s));
    LRCHK(lr_invsqrt(e, e.A1, e.C1, 0, s));
    LRCHK(lr_prod(e, B0, false, e.C1, false, e.TUbar[nb], e.TUbarf[nb], s));
    LRCHK(lr_prod(e, e.TUbar[nb], false, B0, false, e.Km, nullptr, s));
    LRCHK(lr_prod(e, e.Km, false, e.Gq, false, e.T0, nullptr, s));
    LRCHK(lr_prod(e, e.T0, false, e.Km, false, e.A2, nullptr, s));
    LRCHK(lr_invsqrt(e, e.A2, e.C2, 1, s));
    LRCHK(lr_prod(e, e.Km, false, e.C2, false, e.TV[nb], e.TVf[nb], s));
    LRCHK(lr_prod(e, e.TUbar[nb], true, e.Gq, false, e.T0, nullptr, s));   // C1 B0 G_Q = (B0 C1)^T G_Q
    LRCHK(lr_prod(e, e.T0, false, e.Km, false, e.T1, nullptr, s));
    LRCHK(lr_prod(e, e.T1, false, e.C2, false, e.T0, nullptr, s));
    hipLaunchKernelGGL(lr_sym_kernel, dim3((unsigned)cdiv((int64_t)R * R, 256)), dim3(256), 0, s, e.T0, e.B[nb], R,
                       e.st);
    LRCHK(hipGetLastError());
    LRCHK(lr_prod(e, e.TUbar[nb], false, e.B[nb], false, e.TU[nb], e.TUf[nb], s));
    hipLaunchKernelGGL(lr_step_end_kernel, dim3(1), dim3(1024), 0, s, e.st, e.B[nb], e.B[b], R, e.res_hist);
    LRCHK(hipGetLastError());
    return SFR_OK;
}

// Iterate on M (FR-ADM, or Alg. 4 with tsvd) until the device stops; then
// the host learns the returned iterate K from the state.
static sfr_status lr_iterate(LrEngine& e, const Params& p, double mu0, const float* M, int64_t ldm, bool tsvd,
                             hipStream_t s)
{
    DevState& h = *e.host_state;
    memset(&h, 0, sizeof(DevState));
    h.m = e.m; h.n = e.n; h.r = e.r; h.R = e.R;
    h.max_iter = p.max_iter; h.fixed_iters = p.fixed_iters;
    h.lambda = p.lambda; h.rho = p.rho; h.mu_bar = p.mu_bar; h.tol = p.tol;
    h.M = M; h.ldm = ldm;
    h.k = 1;
    h.mu = mu0; h.mu_prev = mu0;
    h.tsvd = tsvd ? 1 : 0;
    LRCHK(hipMemcpyAsync(e.st, &h, offsetof(DevState, B), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(lr_identity_kernel, dim3((unsigned)cdiv((int64_t)e.R * e.R, 256)), dim3(256), 0, s, e.B[0], e.R);
    LRCHK(hipGetLastError());
    const int limit = (p.fixed_iters > 0 ? p.fixed_iters : p.max_iter) + (tsvd ? 0 : 1);
    if (p.fixed_iters > 0) {
        for (int k = 1; k <= limit; ++k) {
            const sfr_status es = lr_enqueue_iter(e, k, M, ldm, tsvd, s);
            if (es != SFR_OK) return es;
        }
    } else {
        // batches of up to 4, one running ahead of the host's check, cut at
        // the forecast stop
        const int batch = 4;
        int k = 1, launched = 0, checked = 0;
        StopForecast fc;
        auto enqueue_batch = [&](int count) -> sfr_status {
            for (int j = 0; j < count && k <= limit; ++j, ++k) {
                const sfr_status es = lr_enqueue_iter(e, k, M, ldm, tsvd, s);
                if (es != SFR_OK) return es;
            }
            const int slot = launched & 1;
            LRCHK(hipMemcpyAsync(&e.host_poll[slot], e.st, offsetof(DevState, B), hipMemcpyDeviceToHost, s));
            LRCHK(hipEventRecord(e.poll_ev[slot], s));
            ++launched;
            return SFR_OK;
        };
        sfr_status es = enqueue_batch(batch);
        if (es != SFR_OK) return es;
        for (;;) {
            if (k <= limit) {
                const int count = fc.size(k, batch, checked == launched);
                if (count > 0) {
                    es = enqueue_batch(count);
                    if (es != SFR_OK) return es;
                }
            }
            if (checked == launched) break;   // k > limit
            const int slot = checked & 1;
            LRCHK(hipEventSynchronize(e.poll_ev[slot]));
            ++checked;
            if (e.host_poll[slot].done) break;
            fc.observe(e.host_poll[slot]);
        }
    }
    LRCHK(hipMemcpyAsync(e.host_state, e.st, offsetof(DevState, B), hipMemcpyDeviceToHost, s));
    LRCHK(hipStreamSynchronize(s));
    if (!h.done) return SFR_ERR_DEVICE;
    if (h.status < 0) return (sfr_status)h.status;
    return SFR_OK;
}

// Outputs of the returned iterate K = iters: U = P_K TUbar_K, V = Q_K TV_K,
// B = B_K, S (optional), min eig(B) and the factors' orthogonality.
static sfr_status lr_outputs(LrEngine& e, const float* M, int64_t ldm, float* U, double* B, float* V, float* S,
                             int64_t lds, bool want_min, hipStream_t s)
{
    const int K = e.host_state->iters;
    const int kb = K & 1, m = e.m, n = e.n, r = e.r, R = e.R;
    LRCHK(lr_gemm(e.P[kb], R, false, e.TUbarf[kb], R, false, U, r, m, r, R, LrPlan{}, e.part, nullptr, s));
    LRCHK(lr_gemm(e.Q[kb], R, false, e.TVf[kb], R, false, V, r, n, r, R, LrPlan{}, e.part, nullptr, s));
    hipLaunchKernelGGL(lr_copy_b_kernel, dim3((unsigned)cdiv((int64_t)r * r, 256)), dim3(256), 0, s, e.B[kb], R, r, B,
                       e.st);
    LRCHK(hipGetLastError());
    if (S) {
        LRCHK(lr_gemm(e.P[kb], R, false, e.TUf[kb], R, false, e.Ak, R, m, R, R, LrPlan{}, e.part, nullptr, s));
        LRCHK(lr_gemm(e.Q[kb], R, false, e.TVf[kb], R, false, e.Vk, R, n, R, R, LrPlan{}, e.part, nullptr, s));
        LstepArgs a;
        memset(&a, 0, sizeof(a));
        a.st = e.st;
        a.A = e.Ak; a.V = e.Vk; a.R = R;
        a.M = M; a.ldm = ldm;
        a.Yprev = (K >= 2) ? e.Y[kb] : nullptr;
        a.ldy = n;
        a.S = S; a.lds = lds;
        a.m = m; a.n = n;
        a.mode = 3;
        hipLaunchKernelGGL(lr_lstep_kernel, dim3((unsigned)cdiv(n, kLstepBN), (unsigned)cdiv(m, kLrBM)), dim3(kLrTPB),
                           0, s, a);
        LRCHK(hipGetLastError());
    }
    if (want_min) {
        hipLaunchKernelGGL(lr_extreme_eig_kernel, dim3(1), dim3(kEigTPB), 0, s, e.B[kb], R, r, e.eigW, e.eigv, e.st,
                           1, 0);
        LRCHK(hipGetLastError());
    }
    // orthogonality of the stored factors (FP64 Grams, r x r)
    double* GU = e.Gp;   // free after the iteration
    double* GV = e.Gq;
    LRCHK(lr_gram(U, r, m, r, r, e.gU, e.gpart, GU, nullptr, s));
    LRCHK(lr_gram(V, r, n, r, r, e.gV, e.gpart, GV, nullptr, s));
    hipLaunchKernelGGL(lr_orth_dist_kernel, dim3(1), dim3(256), 0, s, GU, GV, r, e.st);
    LRCHK(hipGetLastError());
    LRCHK(hipMemcpyAsync(e.host_state, e.st, offsetof(DevState, B), hipMemcpyDeviceToHost, s));
    LRCHK(hipStreamSynchronize(s));
    return SFR_OK;
}

static sfr_status lr_fill_info(const LrEngine& e, sfr_info* info, double mu0)
{
    const DevState& h = *e.host_state;
    if (info) {
        memset(info, 0, sizeof(*info));
        info->iters = h.iters;
        info->converged = (h.status == kOK) ? 1 : 0;
        info->rel_residual = h.res;
        info->min_eig_B = h.min_eig_B;
        info->mu_final = h.mu_prev;
        info->mu0 = mu0;
        info->orth_err = h.orth_err;
    }
    if (h.status == kWarnMaxIter) return SFR_WARN_MAXITER;
    if (!(h.min_eig_B > 0.0)) return SFR_WARN_NOT_SPD;
    return SFR_OK;
}

sfr_status lr_solve(LrEngine* e, const Params& prm, bool mu_auto, const float* M, int64_t ldm, float* U, double* B,
                    float* V, float* S, int64_t lds, sfr_info* info, hipStream_t s)
{
    double mu0 = prm.mu0;
    sfr_status st;
    if (mu_auto) {
        // mu_0 = 1.25 / ||M||_2 from Alg. 4 on M (as on the fused path)
        Params p = prm;
        p.tol = 1e-6;
        p.fixed_iters = 0;
        p.max_iter = 60;
        st = lr_iterate(*e, p, 1.0, M, ldm, true, s);
        if (st < 0) {
            if (info) memset(info, 0, sizeof(*info));
            return st;
        }
        const int kb = e->host_state->iters & 1;
        hipLaunchKernelGGL(lr_extreme_eig_kernel, dim3(1), dim3(kEigTPB), 0, s, e->B[kb], e->R, e->r, e->eigW, e->eigv,
                           e->st, 0, 1);
        LRCHK(hipGetLastError());
        double smax = 0.0;
        LRCHK(hipMemcpyAsync(&smax, &e->st->max_eig_B, sizeof(double), hipMemcpyDeviceToHost, s));
        LRCHK(hipStreamSynchronize(s));
        if (!(smax > 0.0) || !std::isfinite(smax)) {
            if (info) memset(info, 0, sizeof(*info));
            return SFR_ERR_NONFINITE;
        }
        mu0 = 1.25 / smax;
    }
    st = lr_iterate(*e, prm, mu0, M, ldm, false, s);
    if (st == SFR_OK) st = lr_outputs(*e, M, ldm, U, B, V, S, lds, true, s);
    if (st < 0) {
        if (info) memset(info, 0, sizeof(*info));
        return st;
    }
    return lr_fill_info(*e, info, mu0);
}

sfr_status lr_tsvd(LrEngine* e, const Params& prm, const float* M, int64_t ldm, float* U, double* B, float* V,
                   sfr_info* info, hipStream_t s)
{
    sfr_status st = lr_iterate(*e, prm, 1.0, M, ldm, true, s);
    if (st == SFR_OK) st = lr_outputs(*e, M, ldm, U, B, V, nullptr, 0, true, s);
    if (st < 0) {
        if (info) memset(info, 0, sizeof(*info));
        return st;
    }
    return lr_fill_info(*e, info, 0.0);
}

}  // namespace sfr
