// Once-per-solve kernels: initial factors, returned factors, the returned S
// of Alg. 1 (soft threshold of the last residual), the gather of the two
// Nystrom blocks of Alg. 3, and the dense S = M - L of its combine.
#include "sfr_internal.hpp"
#include "small_la.hpp"

#include <stdlib.h>
#include <string.h>

#include <algorithm>

namespace sfr {

template <typename T>
__global__ void init_q_kernel(T* Q, int n, int r, int R)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * R) return;
    const int j = (int)(e / R), k = (int)(e % R);
    Q[e] = (j == k && k < r) ? T(1) : T(0);
}

template <typename T>
hipError_t launch_init_q(T* Q, int n, int r, int R, hipStream_t s)
{
    const int64_t cnt = (int64_t)n * R;
    hipLaunchKernelGGL(init_q_kernel<T>, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, Q, n, r, R);
    return hipGetLastError();
}

__global__ void fill_u64_kernel(unsigned long long* p, size_t count)
{
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (size_t)gridDim.x * blockDim.x)
        p[e] = 0ull;
}

hipError_t launch_fill_u64(unsigned long long* p, size_t count, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    unsigned grid = (unsigned)((count + 255) / 256);
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(fill_u64_kernel, dim3(grid), dim3(256), 0, s, p, count);
    return hipGetLastError();
}

template <typename T>
__global__ void copy_pad_kernel(const T* src, int64_t lds, T* dst, int64_t ldd, int m, int n)
{
    const int i = blockIdx.y;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < ldd; j += gridDim.x * blockDim.x)
        dst[(int64_t)i * ldd + j] = (j < n) ? src[(int64_t)i * lds + j] : T(0);
}

template <typename T>
hipError_t launch_copy_pad(const T* src, int64_t lds, T* dst, int64_t ldd, int m, int n, hipStream_t s)
{
    unsigned gx = (unsigned)((ldd + 255) / 256);
    if (gx > 64) gx = 64;
    hipLaunchKernelGGL(copy_pad_kernel<T>, dim3(gx, m), dim3(256), 0, s, src, lds, dst, ldd, m, n);
    return hipGetLastError();
}

// Returned factors: U = P TUbar (m x r), V = Q TV (n x r), B; and the row
// factors A = P TU, Vt = Q TV (R wide, zero padded) used by the S pass.
// P and Q are the ping-pong buffers of the iteration: the returned iterate
// K = st->iters reads P[K & 1], Q[K & 1] and writes A, Vt into the other
// pair.  Nothing is written unless the solve finished without error.
template <typename T>
__global__ void factors_kernel(const DevState* st, PingPong<T> pp, int m, int n, int r, int R, T* U, T* V,
                               double* B)
{
    if (!st->done || st->status < 0 || st->exch_timeout) return;
    const int K = st->iters;
    const T* P = pp.P[K & 1];
    const T* Q = pp.Q[K & 1];
    T* A = pp.P[(K + 1) & 1];
    T* Vt = pp.Q[(K + 1) & 1];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nu = (int64_t)m * R, nvv = (int64_t)n * R;
    if (e < nu) {
        const int i = (int)(e / R), k = (int)(e % R);
        double su = 0.0, sa = 0.0;
        for (int t = 0; t < R; ++t) {
            const double pt = (double)P[(int64_t)i * R + t];
            su = fma(pt, st->TUbar[t * kMaxR + k], su);
            sa = fma(pt, st->TU[t * kMaxR + k], sa);
        }
        if (k < r) U[(int64_t)i * r + k] = (T)su;
        A[e] = (T)sa;
    } else if (e < nu + nvv) {
        const int64_t f = e - nu;
        const int j = (int)(f / R), k = (int)(f % R);
        double sv = 0.0;
        for (int t = 0; t < R; ++t) sv = fma((double)Q[(int64_t)j * R + t], st->TV[t * kMaxR + k], sv);
        if (k < r) V[(int64_t)j * r + k] = (T)sv;
        Vt[f] = (T)sv;
    } else if (e < nu + nvv + (int64_t)r * r) {
        const int64_t f = e - nu - nvv;
        const int i = (int)(f / r), j = (int)(f % r);
        B[f] = st->B[i * kMaxR + j];
    }
}

// VEC consecutive elements; one 16-byte access when VEC * sizeof(T) == 16.
template <typename T, int VEC>
__device__ __forceinline__ void vload(const T* p, T (&v)[VEC])
{
    if constexpr (VEC * sizeof(T) == 16) {
        const float4 x = *reinterpret_cast<const float4*>(p);
        __builtin_memcpy(v, &x, 16);
    } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) v[e] = p[e];
    }
}
template <typename T, int VEC>
__device__ __forceinline__ void vstore(T* p, const T (&v)[VEC])
{
    if constexpr (VEC * sizeof(T) == 16) {
        float4 x;
        __builtin_memcpy(&x, v, 16);
        *reinterpret_cast<float4*>(p) = x;
    } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) p[e] = v[e];
    }
}

// Dense pass over an m x n matrix with the rank-R term l_ij = A_i . Vt_j:
//   mode 0 (FR-ADM S):  S = P_ST_{lambda/mu}(M - l + Y/mu), Y may be NULL;
//                       optionally also min eig(B) into the state
//   mode 1 (FR-Nys S):  S = M - l
// A workgroup owns a column tile of 256 * VEC columns and a band of rows;
// each thread keeps its VEC columns of Vt in registers and streams 16-byte
// vectors down the band.  The row factor A_i is uniform over the
// workgroup.  Vector paths need n, ldm, ldy, lds multiples of VEC and
// 16-byte aligned bases; otherwise VEC = 1.
constexpr int kLowrankRows = 64;   // rows of a lowrank_pass workgroup's band

template <typename T, int VEC, int R>
__global__ void __launch_bounds__(256) lowrank_pass_kernel(LowrankArgs<T> a)
{
    const T* M = a.M;
    const int64_t ldm = a.ldm, ldy = a.ldy, lds = a.lds;
    const int m = a.m, n = a.n, mode = a.mode, rows_per_blk = a.rows_per_blk;
    T* S = a.S;
    const T* Y = a.Y;
    const T* A = a.A;
    const T* Vt = a.Vt;
    double mu = a.mu;
    const double lam = a.lam;
    if (a.st) {
        // FR-ADM: the returned iterate K picks the buffers (see factors_kernel)
        const DevState* st = a.st;
        if (!st->done || st->status < 0 || st->exch_timeout) return;
        const int K = st->iters;
        Y = (K >= 2) ? a.pp.Y[K & 1] : nullptr;
        A = a.pp.P[(K + 1) & 1];
        Vt = a.pp.Q[(K + 1) & 1];
        mu = st->mu_prev;
        if (a.min_eig && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < 64) {
            // smallest eigenvalue of the returned B (Appendix, Lemma 2): one
            // wavefront of the first workgroup, before its share of the pass
            __shared__ double Aw[R * LDP], Ew[R * LDP];
            __shared__ __align__(16) double csw[2 * 16];
            const double w = wmin_eig<R>(st->B, kMaxR, st->r, Aw, Ew, csw);
            if (threadIdx.x == 0) a.st->min_eig_B = w;
        }
    }
    const int tid = threadIdx.x;
    const int j0 = blockIdx.x * 256 * VEC;
    const T t = (T)(lam / mu), imu = (T)(1.0 / mu);
    const int i0 = blockIdx.y * rows_per_blk;
    const int i1 = min(m, i0 + rows_per_blk);
    const int jj = tid * VEC;
    const int j = j0 + jj;
    // the band's row factors (one coalesced load, then broadcast reads)
    __shared__ T Ab[kLowrankRows * R];
    for (int e = tid; e < (i1 - i0) * R; e += 256) Ab[e] = A[(int64_t)i0 * R + e];
    __syncthreads();
    // ||Y_{K+1} - Y_K||^2 of this thread's elements (a.rpart: the residual of
    // the returned iterate, in the sweep's clamp form Y_{K+1} = clamp(mu_K R))
    const bool want_res = (a.rpart != nullptr) && (mode == 0);
    const T muT = (T)mu, lamT = (T)lam;
    double racc = 0.0;
    if (j < n) {
    // this thread's VEC columns of Vt stay in registers for the whole band
    T vk[R][VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e)
#pragma unroll
        for (int k = 0; k < R; ++k) vk[k][e] = (j + e < n) ? Vt[(int64_t)(j + e) * R + k] : T(0);
    const bool full = (VEC == 1) || (j + VEC <= n);
    // RU rows per step: the M (and Y) loads of all of them are in flight
    // together before any is used
    constexpr int RU = (sizeof(T) == 4) ? 8 : 4;
    for (int i = i0; i < i1; i += RU) {
        T mv[RU][VEC], yv[RU][VEC];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) { mv[u][e] = T(0); yv[u][e] = T(0); }
            if (full && i + u < i1) {
                vload<T, VEC>(M + (int64_t)(i + u) * ldm + j, mv[u]);
                if (mode == 0 && Y) vload<T, VEC>(Y + (int64_t)(i + u) * ldy + j, yv[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            if (i + u >= i1) break;
            T av[R];
#pragma unroll
            for (int k = 0; k < R; ++k) av[k] = Ab[(i + u - i0) * R + k];
            T out[VEC];
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                T l = 0;
#pragma unroll
                for (int k = 0; k < R; ++k) l = fma(av[k], vk[k][e], l);
                if (mode == 0) {
                    const T Rr = mv[u][e] - l + yv[u][e] * imu;
                    const T a = Rr - t, b = Rr + t;
                    out[e] = (a > T(0) ? a : T(0)) + (b < T(0) ? b : T(0));
                    if (want_res && full && j + e < n) {
                        const T y = fmin(fmax(muT * Rr, -lamT), lamT);
                        const double dy = (double)(y - yv[u][e]);
                        racc = fma(dy, dy, racc);
                    }
                } else {
                    out[e] = mv[u][e] - l;
                }
            }
            if (full) vstore<T, VEC>(S + (int64_t)(i + u) * lds + j, out);
        }
    }
    }
    if (want_res) {
        // workgroup sum in a fixed order: wavefronts by shuffles, then the
        // four wavefront sums in order
        __shared__ double rred[4];
        for (int off = 32; off > 0; off >>= 1) racc += __shfl_xor(racc, off, 64);
        if ((tid & 63) == 0) rred[tid >> 6] = racc;
        __syncthreads();
        if (tid == 0)
            a.rpart[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = (rred[0] + rred[1]) + (rred[2] + rred[3]);
    }
}

// Narrow rows (n <= kNarrowCols, 16-byte vectors).  The column-tile form
// above keeps one column vector per thread, so for narrow matrices all but
// n / VEC of its 256 threads idle (262144 x 48: 12 of 256).  Here thread t
// takes column vector t mod CPV (CPV = n / VEC vectors a row) of the band's
// rows t div CPV, t div CPV + RPP, ... (RPP = 256 div CPV rows at a time),
// with the M (and Y) loads of up to kNarrowInFlight rows in flight together.
// The arithmetic per element is that of lowrank_pass_kernel.
constexpr int kNarrowCols = 256;
constexpr int kNarrowRows = 128;      // rows of a workgroup's band
constexpr int kNarrowInFlight = 8;

template <typename T, int R>
__global__ void __launch_bounds__(256) lowrank_narrow_kernel(LowrankArgs<T> a)
{
    constexpr int VEC = 16 / sizeof(T);
    constexpr int NR = kNarrowInFlight;
    const T* M = a.M;
    const int64_t ldm = a.ldm, ldy = a.ldy, lds = a.lds;
    const int m = a.m, n = a.n, mode = a.mode;
    T* S = a.S;
    const T* Y = a.Y;
    const T* A = a.A;
    const T* Vt = a.Vt;
    double mu = a.mu;
    const double lam = a.lam;
    if (a.st) {
        // FR-ADM: the returned iterate K picks the buffers (see factors_kernel)
        const DevState* st = a.st;
        if (!st->done || st->status < 0 || st->exch_timeout) return;
        const int K = st->iters;
        Y = (K >= 2) ? a.pp.Y[K & 1] : nullptr;
        A = a.pp.P[(K + 1) & 1];
        Vt = a.pp.Q[(K + 1) & 1];
        mu = st->mu_prev;
        if (a.min_eig && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < 64) {
            __shared__ double Aw[R * LDP], Ew[R * LDP];
            __shared__ __align__(16) double csw[2 * 16];
            const double w = wmin_eig<R>(st->B, kMaxR, st->r, Aw, Ew, csw);
            if (threadIdx.x == 0) a.st->min_eig_B = w;
        }
    }
    const int tid = threadIdx.x;
    const int cpv = n / VEC;                    // the host takes this form for n % VEC == 0, n <= kNarrowCols
    const int rpp = 256 / cpv;
    const int cv = tid % cpv, rr = tid / cpv;
    const bool tact = rr < rpp;
    const int j = cv * VEC;
    const int i0 = blockIdx.y * kNarrowRows;
    const int i1 = min(m, i0 + kNarrowRows);
    __shared__ T Ab[kNarrowRows * R];
    for (int e = tid; e < (i1 - i0) * R; e += 256) Ab[e] = A[(int64_t)i0 * R + e];
    T vk[R][VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e)
#pragma unroll
        for (int k = 0; k < R; ++k) vk[k][e] = Vt[(int64_t)(j + e) * R + k];
    __syncthreads();
    const T t = (T)(lam / mu), imu = (T)(1.0 / mu);
    const bool want_res = (a.rpart != nullptr) && (mode == 0);
    const bool use_y = (mode == 0) && (Y != nullptr);
    const T muT = (T)mu, lamT = (T)lam;
    double racc = 0.0;
    if (tact) {
        for (int ib = i0 + rr; ib < i1; ib += NR * rpp) {
            T mv[NR][VEC], yv[NR][VEC];
#pragma unroll
            for (int u = 0; u < NR; ++u) {
                const int i = ib + u * rpp;
#pragma unroll
                for (int e = 0; e < VEC; ++e) { mv[u][e] = T(0); yv[u][e] = T(0); }
                if (i < i1) {
                    vload<T, VEC>(M + (int64_t)i * ldm + j, mv[u]);
                    if (use_y) vload<T, VEC>(Y + (int64_t)i * ldy + j, yv[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < NR; ++u) {
                const int i = ib + u * rpp;
                if (i >= i1) break;
                T av[R];
#pragma unroll
                for (int k = 0; k < R; ++k) av[k] = Ab[(i - i0) * R + k];
                T out[VEC];
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    T l = 0;
#pragma unroll
                    for (int k = 0; k < R; ++k) l = fma(av[k], vk[k][e], l);
                    if (mode == 0) {
                        const T Rr = mv[u][e] - l + yv[u][e] * imu;
                        const T lo = Rr - t, hi = Rr + t;
                        out[e] = (lo > T(0) ? lo : T(0)) + (hi < T(0) ? hi : T(0));
                        if (want_res) {
                            const T y = fmin(fmax(muT * Rr, -lamT), lamT);
                            const double dy = (double)(y - yv[u][e]);
                            racc = fma(dy, dy, racc);
                        }
                    } else {
                        out[e] = mv[u][e] - l;
                    }
                }
                vstore<T, VEC>(S + (int64_t)i * lds + j, out);
            }
        }
    }
    if (want_res) {
        // workgroup sum in a fixed order: wavefronts by shuffles, then the
        // four wavefront sums in order
        __shared__ double rred[4];
        for (int off = 32; off > 0; off >>= 1) racc += __shfl_xor(racc, off, 64);
        if ((tid & 63) == 0) rred[tid >> 6] = racc;
        __syncthreads();
        if (tid == 0)
            a.rpart[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = (rred[0] + rred[1]) + (rred[2] + rred[3]);
    }
}

template <typename T>
static hipError_t lowrank_narrow_dispatch(const LowrankArgs<T>& a, int R, hipStream_t s, int* parts)
{
    dim3 grid(1u, (unsigned)((a.m + kNarrowRows - 1) / kNarrowRows));
    if (parts) *parts = (int)(grid.x * grid.y);
    switch (R) {
#define CASE(rr)                                                                                \
    case rr: hipLaunchKernelGGL((lowrank_narrow_kernel<T, rr>), grid, dim3(256), 0, s, a); \
        break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(8) CASE(10) CASE(12) CASE(16) CASE(20) CASE(24)
        CASE(32)
#undef CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Matrix-core form of the FP32 pass (R >= 8).  The rank-R term of a tile of
// 16 rows x 16 columns is one matrix-core product over K = R (padded to a
// multiple of 4), taken transposed, D = Vt_tile A_tile^T, so that lane
// (c, g) = (lane % 16, lane / 16) of a wavefront receives row c, columns
// 4g .. 4g + 3 of the tile: exactly the M, Y and S elements it then reads
// and writes as one 16-byte vector each.  A wavefront owns 64 columns (four
// tiles, whose Vt operands stay in registers) of the workgroup's 64-row band
// and walks it 16 rows at a time, the next rows' loads in flight.  After l
// the arithmetic per element is that of lowrank_pass_kernel.
typedef float dn_f32x4 __attribute__((ext_vector_type(4)));
constexpr int kLrmCols = 256;   // columns of a matrix-core workgroup (four wavefronts x 64)

template <int R>
__global__ void __launch_bounds__(256) lowrank_mfma_kernel(LowrankArgs<float> a)
{
    constexpr int KS = (R + 3) / 4;           // 4-deep steps of K
    constexpr int AP = 4 * KS;                // padded row-factor pitch in LDS
    constexpr int NST = kLowrankRows / 16;    // 16-row steps of the band
    const float* M = a.M;
    const int64_t ldm = a.ldm, ldy = a.ldy, lds = a.lds;
    const int m = a.m, n = a.n, mode = a.mode;
    float* S = a.S;
    const float* Y = a.Y;
    const float* A = a.A;
    const float* Vt = a.Vt;
    double mu = a.mu;
    const double lam = a.lam;
    if (a.st) {
        // FR-ADM: the returned iterate K picks the buffers (see factors_kernel)
        const DevState* st = a.st;
        if (!st->done || st->status < 0 || st->exch_timeout) return;
        const int K = st->iters;
        Y = (K >= 2) ? a.pp.Y[K & 1] : nullptr;
        A = a.pp.P[(K + 1) & 1];
        Vt = a.pp.Q[(K + 1) & 1];
        mu = st->mu_prev;
        if (a.min_eig && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < 64) {
            __shared__ double Aw[R * LDP], Ew[R * LDP];
            __shared__ __align__(16) double csw[2 * 16];
            const double w = wmin_eig<R>(st->B, kMaxR, st->r, Aw, Ew, csw);
            if (threadIdx.x == 0) a.st->min_eig_B = w;
        }
    }
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c = lane & 15, g = lane >> 4;
    const int i0 = blockIdx.y * kLowrankRows;
    const int i1 = min(m, i0 + kLowrankRows);
    const int jw = blockIdx.x * kLrmCols + wave * 64;
    // the band's row factors, zero past rank R and past the band's last row
    __shared__ float Ab[kLowrankRows * AP];
    for (int e = tid; e < kLowrankRows * AP; e += 256) {
        const int ii = e / AP, k = e % AP;
        Ab[e] = (i0 + ii < i1 && k < R) ? A[(int64_t)(i0 + ii) * R + k] : 0.f;
    }
    // Vt operands of the wavefront's four tiles: column jw + 16 t + c, rank 4 s + g
    float va[4][KS];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int col = jw + 16 * t + c;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int k = 4 * s + g;
            va[t][s] = (col < n && k < R) ? Vt[(int64_t)col * R + k] : 0.f;
        }
    }
    __syncthreads();
    const float th = (float)(lam / mu), imu = (float)(1.0 / mu);
    const bool want_res = (a.rpart != nullptr) && (mode == 0);
    const float muT = (float)mu, lamT = (float)lam;
    const bool use_y = (mode == 0) && (Y != nullptr);
    double racc = 0.0;
    // n is a multiple of 4: a lane's four columns of a tile are all in range or all out
    bool cok[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) cok[t] = jw + 16 * t + 4 * g < n;
    dn_f32x4 mv[2][4], yv[2][4];
    auto issue = [&](int stp, int b) {
        const int row = i0 + 16 * stp + c;
        const bool rok = row < i1;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int col = jw + 16 * t + 4 * g;
            const bool ok = rok && cok[t];
            mv[b][t] = dn_f32x4{0.f, 0.f, 0.f, 0.f};
            yv[b][t] = dn_f32x4{0.f, 0.f, 0.f, 0.f};
            if (ok) {
                mv[b][t] = *reinterpret_cast<const dn_f32x4*>(M + (int64_t)row * ldm + col);
                if (use_y) yv[b][t] = *reinterpret_cast<const dn_f32x4*>(Y + (int64_t)row * ldy + col);
            }
        }
    };
    issue(0, 0);
#pragma unroll
    for (int stp = 0; stp < NST; ++stp) {
        const int b = stp & 1;
        if (stp + 1 < NST) issue(stp + 1, b ^ 1);
        float vb[KS];
#pragma unroll
        for (int s = 0; s < KS; ++s) vb[s] = Ab[(16 * stp + c) * AP + 4 * s + g];
        dn_f32x4 acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            acc[t] = dn_f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < KS; ++s) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(va[t][s], vb[s], acc[t], 0, 0, 0);
        }
        const int row = i0 + 16 * stp + c;
        const bool rok = row < i1;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const bool ok = rok && cok[t];
            dn_f32x4 out;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float l = acc[t][e];
                if (mode == 0) {
                    const float Rr = mv[b][t][e] - l + yv[b][t][e] * imu;
                    const float lo = Rr - th, hi = Rr + th;
                    out[e] = (lo > 0.f ? lo : 0.f) + (hi < 0.f ? hi : 0.f);
                    if (want_res && ok) {
                        const float y = fminf(fmaxf(muT * Rr, -lamT), lamT);
                        const double dy = (double)(y - yv[b][t][e]);
                        racc = fma(dy, dy, racc);
                    }
                } else {
                    out[e] = mv[b][t][e] - l;
                }
            }
            if (ok) *reinterpret_cast<dn_f32x4*>(S + (int64_t)row * lds + jw + 16 * t + 4 * g) = out;
        }
    }
    if (want_res) {
        // workgroup sum in a fixed order: wavefronts by shuffles, then the
        // four wavefront sums in order
        __shared__ double rred[4];
        for (int off = 32; off > 0; off >>= 1) racc += __shfl_xor(racc, off, 64);
        if (lane == 0) rred[wave] = racc;
        __syncthreads();
        if (tid == 0)
            a.rpart[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = (rred[0] + rred[1]) + (rred[2] + rred[3]);
    }
}

// Rows of a column-tile workgroup's band: kLowrankRows, or fewer (down to 8)
// for small m, so that a small matrix still spreads over the device.
static int lowrank_band_rows(int m)
{
    if (m >= 64 * kLowrankRows) return kLowrankRows;
    const int rows = (m + 63) / 64;
    return std::max(8, std::min(kLowrankRows, (rows + 7) / 8 * 8));
}

int lowrank_res_parts(int m, int n)
{
    // the most workgroups any form of the pass launches (column tiles of 256
    // columns at the smallest band)
    return ((n + 255) / 256) * ((m + 7) / 8);
}

__global__ void __launch_bounds__(256) res_final_kernel(DevState* st, const double* rpart, int count,
                                                        double* res_hist)
{
    if (!st->done || st->status < 0 || st->exch_timeout || st->stop_after <= 0) return;
    __shared__ double red[256];
    const int t = threadIdx.x;
    double s = 0.0;
    for (int e = t; e < count; e += 256) s += rpart[e];
    red[t] = s;
    __syncthreads();
    if (t == 0) {
        double tot = 0.0;
        for (int w = 0; w < 256; ++w) tot += red[w];
        const double res = sqrt(tot) / (st->mu_prev * st->nrmM);
        st->res = res;
        if (st->iters >= 1) res_hist[st->iters - 1] = res;
    }
}

hipError_t launch_res_final(DevState* st, const double* rpart, int count, double* res_hist, hipStream_t s)
{
    hipLaunchKernelGGL(res_final_kernel, dim3(1), dim3(256), 0, s, st, rpart, count, res_hist);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_factors(const DevState* st, const PingPong<T>& pp, int m, int n, int r, int R, T* U, T* V,
                          double* B, hipStream_t s)
{
    const int64_t cnt = (int64_t)m * R + (int64_t)n * R + (int64_t)r * r;
    hipLaunchKernelGGL(factors_kernel<T>, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, st, pp, m, n, r,
                       R, U, V, B);
    return hipGetLastError();
}

template <typename T, int VEC>
static hipError_t lowrank_dispatch(const LowrankArgs<T>& a, int R, hipStream_t s, int* parts)
{
    dim3 grid((unsigned)((a.n + 256 * VEC - 1) / (256 * VEC)), (unsigned)((a.m + a.rows_per_blk - 1) / a.rows_per_blk));
    if (parts) *parts = (int)(grid.x * grid.y);
    switch (R) {
#define CASE(rr)                                                                               \
    case rr: hipLaunchKernelGGL((lowrank_pass_kernel<T, VEC, rr>), grid, dim3(256), 0, s, a); \
        break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(8) CASE(10) CASE(12) CASE(16) CASE(20) CASE(24)
        CASE(32)
#undef CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static hipError_t lowrank_mfma_dispatch(const LowrankArgs<float>& a, int R, hipStream_t s, int* parts)
{
    dim3 grid((unsigned)((a.n + kLrmCols - 1) / kLrmCols), (unsigned)((a.m + kLowrankRows - 1) / kLowrankRows));
    if (parts) *parts = (int)(grid.x * grid.y);
    switch (R) {
#define CASE(rr)                                                                           \
    case rr: hipLaunchKernelGGL((lowrank_mfma_kernel<rr>), grid, dim3(256), 0, s, a); \
        break;
        CASE(8) CASE(10) CASE(12) CASE(16) CASE(20) CASE(24) CASE(32)
#undef CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Rank buckets that take the matrix-core FP32 pass (SFR_SPASS=vector keeps
// the vector form for every bucket).
static bool lowrank_mfma_bucket(int R)
{
    const char* v = getenv("SFR_SPASS");
    const bool off = v != nullptr && strcmp(v, "vector") == 0;
    return !off && (R == 8 || R == 10 || R == 12 || R == 16 || R == 20 || R == 24 || R == 32);
}

// Narrow matrices take the row-packed form (SFR_SPASS=vector or =mfma keeps
// the column-tile forms, to test them).
static bool lowrank_narrow_ok()
{
    const char* v = getenv("SFR_SPASS");
    return v == nullptr || strcmp(v, "narrow") == 0 || strcmp(v, "auto") == 0;
}

// Vector paths need n, ldm, ldy, lds multiples of VEC and 16-byte aligned
// bases (both Y buffers when they are picked on the device); so do the
// row-packed narrow form and the matrix-core form (FP32, rank buckets from 8).
template <typename T>
hipError_t launch_lowrank_pass(LowrankArgs<T> a, int R, hipStream_t s, int* parts)
{
    constexpr int V = 16 / sizeof(T);
    a.rows_per_blk = lowrank_band_rows(a.m);
    auto al = [](const void* p) { return ((uintptr_t)p % 16) == 0; };
    bool ys = a.st ? (al(a.pp.Y[0]) && al(a.pp.Y[1])) : (!a.Y || al(a.Y));
    const bool vec = (a.n % V == 0) && (a.ldm % V == 0) && (a.lds % V == 0) && al(a.M) && al(a.S) &&
                     (a.ldy % V == 0) && ys;
    if (vec && a.n <= kNarrowCols && lowrank_narrow_ok()) return lowrank_narrow_dispatch<T>(a, R, s, parts);
    if constexpr (sizeof(T) == 4) {
        if (vec && lowrank_mfma_bucket(R)) return lowrank_mfma_dispatch(a, R, s, parts);
    }
    if (vec) return lowrank_dispatch<T, V>(a, R, s, parts);
    return lowrank_dispatch<T, 1>(a, R, s, parts);
}

// Alg. 3: C = Mt[:, 0:l] (m x l), Rb = Mt[0:l, :] (l x n) with row i of the
// shuffled matrix Mt being row perm[i] of M.
template <typename T>
__global__ void nys_gather_kernel(const T* M, int64_t ldm, const int64_t* perm, int m, int n, int l,
                                  T* C, T* Rb)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nc = (int64_t)m * l, nr = (int64_t)l * n;
    if (e < nc) {
        const int i = (int)(e / l), j = (int)(e % l);
        C[e] = M[perm[i] * ldm + j];
    } else if (e < nc + nr) {
        const int64_t f = e - nc;
        const int i = (int)(f / n), j = (int)(f % n);
        Rb[f] = M[perm[i] * ldm + j];
    }
}

template <typename T>
hipError_t launch_nys_gather(const T* M, int64_t ldm, const int64_t* perm, int m, int n, int l, T* C, T* Rb,
                             hipStream_t s)
{
    const int64_t cnt = (int64_t)m * l + (int64_t)l * n;
    hipLaunchKernelGGL(nys_gather_kernel<T>, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, M, ldm, perm,
                       m, n, l, C, Rb);
    return hipGetLastError();
}

// Orthogonality of the returned Stiefel factors (U in St_{m,r}, V in
// St_{n,r}, eq. (7)) as stored.  Pass 1: workgroup b < nu sums the Gram of
// U's row block b, the others V's, over the packed upper triangle
// (r(r+1)/2 entries), each entry in row order.  Pass 2 adds the blocks in
// order and takes the two Frobenius distances to I_r.
__device__ __forceinline__ void tri_index(int e, int r, int& p, int& q)
{
    p = 0;
    while (e >= r - p) { e -= r - p; ++p; }
    q = p + e;
}

// Rows of a block are staged through LDS in chunks of kOrthChunk (one
// coalesced load of the chunk's contiguous r-wide rows), then thread t adds
// the products of its entries t, t + 256, ... (r <= 32: at most three) over
// the chunk's rows, in row order.
constexpr int kOrthChunk = 128;

// Small ranks (r <= kOrthSmallR): thread t accumulates all r(r+1)/2 entries
// over rows t, t + 256, ... of the block in registers, eight rows' loads in
// flight at a time; the block then adds the 256 thread sums of each entry
// (wavefront shuffles, then the four wavefront sums in order).  Tall
// factors (the 262144 x 3 photometric U) stream at full width this way.
constexpr int kOrthSmallR = 8;

template <typename T>
__device__ void orth_block_small(const T* X, int r, int i0, int i1, double* out)
{
    constexpr int RM = kOrthSmallR, EM = RM * (RM + 1) / 2, RU = 8;
    double acc[EM];
#pragma unroll
    for (int e = 0; e < EM; ++e) acc[e] = 0.0;
    const int t = threadIdx.x;
    for (int i = i0 + t; i < i1; i += 256 * RU) {
        double x[RU][RM];
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            const int iu = i + 256 * u;
#pragma unroll
            for (int p = 0; p < RM; ++p) x[u][p] = (iu < i1 && p < r) ? (double)X[(int64_t)iu * r + p] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < RU; ++u) {
            int e = 0;
#pragma unroll
            for (int p = 0; p < RM; ++p)
#pragma unroll
                for (int q = p; q < RM; ++q) {
                    acc[e] = fma(x[u][p], x[u][q], acc[e]);
                    ++e;
                }
        }
    }
    __shared__ double wsum[4][EM];
    const int lane = t & 63, wave = t >> 6;
#pragma unroll
    for (int e = 0; e < EM; ++e) {
        double v = acc[e];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) wsum[wave][e] = v;
    }
    __syncthreads();
    // entry e of the packed triangle of an r x r Gram (p <= q < r) from the
    // RM x RM layout of the accumulators
    if (t < r * (r + 1) / 2) {
        int p, q, e = t;
        p = 0;
        while (e >= r - p) { e -= r - p; ++p; }
        q = p + e;
        const int em = p * RM - p * (p - 1) / 2 + (q - p);
        out[t] = (wsum[0][em] + wsum[1][em]) + (wsum[2][em] + wsum[3][em]);
    }
}

template <typename T>
__global__ void __launch_bounds__(256) orth_partial_kernel(const DevState* st, const T* U, int m, const T* V, int n,
                                                           int r, double* Up, int nu, double* Vp, int nv)
{
    if (st && (!st->done || st->status < 0 || st->exch_timeout)) return;
    if (r <= kOrthSmallR) {
        const bool isU = (int)blockIdx.x < nu;
        const int b = isU ? (int)blockIdx.x : (int)blockIdx.x - nu;
        const int nb = isU ? nu : nv;
        const int rows = isU ? m : n;
        const int per = (rows + nb - 1) / nb;
        const int i0 = b * per, i1 = min(rows, i0 + per);
        orth_block_small<T>(isU ? U : V, r, i0, i1, (isU ? Up : Vp) + (size_t)b * (r * (r + 1) / 2));
        return;
    }
    __shared__ double xs[kOrthChunk * kMaxR];
    const bool isU = (int)blockIdx.x < nu;
    const int b = isU ? (int)blockIdx.x : (int)blockIdx.x - nu;
    const int nb = isU ? nu : nv;
    const int rows = isU ? m : n;
    const T* X = isU ? U : V;
    const int E = r * (r + 1) / 2;
    double* out = (isU ? Up : Vp) + (size_t)b * E;
    const int per = (rows + nb - 1) / nb;
    const int i0 = b * per, i1 = min(rows, i0 + per);
    const int t = threadIdx.x;
    constexpr int EU = (kMaxR * (kMaxR + 1) / 2 + 255) / 256;
    int pp[EU], qq[EU];
    double a[EU];
#pragma unroll
    for (int u = 0; u < EU; ++u) {
        a[u] = 0.0;
        pp[u] = 0;
        qq[u] = 0;
        if (t + 256 * u < E) tri_index(t + 256 * u, r, pp[u], qq[u]);
    }
    for (int c0 = i0; c0 < i1; c0 += kOrthChunk) {
        const int cnt = min(kOrthChunk, i1 - c0) * r;
        const T* src = X + (int64_t)c0 * r;
        for (int k = t; k < cnt; k += 256) xs[k] = (double)src[k];
        __syncthreads();
        const int nr = cnt / r;
#pragma unroll
        for (int u = 0; u < EU; ++u) {
            if (t + 256 * u < E) {
                const double* xp = xs + pp[u];
                const double* xq = xs + qq[u];
                double acc = a[u];
                for (int i = 0; i < nr; ++i) acc = fma(xp[i * r], xq[i * r], acc);
                a[u] = acc;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < EU; ++u)
        if (t + 256 * u < E) out[t + 256 * u] = a[u];
}

__global__ void __launch_bounds__(256) orth_final_kernel(const DevState* st, int r, const double* Up, int nu,
                                                         const double* Vp, int nv, double* out)
{
    if (st && (!st->done || st->status < 0 || st->exch_timeout)) return;
    __shared__ double red[2][256];
    const int E = r * (r + 1) / 2;
    double su = 0.0, sv = 0.0;
    for (int e = threadIdx.x; e < E; e += 256) {
        int p, q;
        tri_index(e, r, p, q);
        // partials added in order, eight loads in flight at a time
        double gu = 0.0, gv = 0.0;
        for (int b0 = 0; b0 < nu; b0 += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = Up[(size_t)min(b0 + u, nu - 1) * E + e];
#pragma unroll
            for (int u = 0; u < 8; ++u) gu += (b0 + u < nu) ? v[u] : 0.0;
        }
        for (int b0 = 0; b0 < nv; b0 += 8) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = Vp[(size_t)min(b0 + u, nv - 1) * E + e];
#pragma unroll
            for (int u = 0; u < 8; ++u) gv += (b0 + u < nv) ? v[u] : 0.0;
        }
        const double w = (p == q) ? 1.0 : 2.0;
        const double du = gu - (p == q ? 1.0 : 0.0), dv = gv - (p == q ? 1.0 : 0.0);
        su += w * du * du;
        sv += w * dv * dv;
    }
    red[0][threadIdx.x] = su;
    red[1][threadIdx.x] = sv;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = fmax(sqrt(red[0][0]), sqrt(red[1][0]));
}

// Small ranks (r <= kOrthSmallR, at most 72 entries of the two Grams): up to
// kOrthPartsSmall row blocks per factor, so that tall factors spread over the
// device.  Thread t sums slice t / W of the partials of entry t mod W
// (W = 2E: the U entries, then the V entries), its loads in flight together;
// the slice sums are added in slice order and the entries' squared
// deviations from I in a fixed tree.
constexpr int kOrthPartsSmall = 256;

__global__ void __launch_bounds__(256) orth_final_small_kernel(const DevState* st, int r, const double* Up, int nu,
                                                               const double* Vp, int nv, double* out)
{
    if (st && (!st->done || st->status < 0 || st->exch_timeout)) return;
    __shared__ double part[256];
    __shared__ double dev[2][256];
    constexpr int CH = 32;
    const int E = r * (r + 1) / 2, W = 2 * E;   // W <= 72
    const int S = 256 / W;
    const int t = threadIdx.x;
    const int sl = t / W, w = t % W;
    double g = 0.0;
    if (sl < S) {
        const bool isU = w < E;
        const int e = isU ? w : w - E;
        const int cnt = isU ? nu : nv;
        const double* base = isU ? Up : Vp;
        const int per = (cnt + S - 1) / S;
        const int b0 = sl * per, b1 = min(cnt, b0 + per);
        for (int bb = b0; bb < b1; bb += CH) {
            double v[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u) v[u] = base[(size_t)min(bb + u, cnt - 1) * E + e];
#pragma unroll
            for (int u = 0; u < CH; ++u) g += (bb + u < b1) ? v[u] : 0.0;
        }
    }
    part[t] = g;
    __syncthreads();
    double cu = 0.0, cv = 0.0;
    if (t < W) {
        double gw = 0.0;
        for (int q = 0; q < S; ++q) gw += part[q * W + t];
        const bool isU = t < E;
        int p, q;
        tri_index(isU ? t : t - E, r, p, q);
        const double d = gw - (p == q ? 1.0 : 0.0);
        const double c = (p == q ? 1.0 : 2.0) * d * d;
        cu = isU ? c : 0.0;
        cv = isU ? 0.0 : c;
    }
    dev[0][t] = cu;
    dev[1][t] = cv;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) {
            dev[0][t] += dev[0][t + h];
            dev[1][t] += dev[1][t + h];
        }
        __syncthreads();
    }
    if (t == 0) *out = fmax(sqrt(dev[0][0]), sqrt(dev[1][0]));
}

// At most this many row blocks per factor: the final sum stays short.
constexpr int kOrthParts = 32;

template <typename T>
hipError_t launch_orth(const DevState* st, const T* U, int m, const T* V, int n, int r, double* Up, int nu,
                       double* Vp, int nv, double* out, hipStream_t s)
{
    if (r < 1 || r > kMaxR) return hipErrorInvalidValue;
    const bool small = r <= kOrthSmallR;
    const int parts = small ? kOrthPartsSmall : kOrthParts;
    nu = std::max(1, std::min({nu, m, parts}));
    nv = std::max(1, std::min({nv, n, parts}));
    hipLaunchKernelGGL(orth_partial_kernel<T>, dim3((unsigned)(nu + nv)), dim3(256), 0, s, st, U, m, V, n, r, Up,
                       nu, Vp, nv);
    if (small)
        hipLaunchKernelGGL(orth_final_small_kernel, dim3(1), dim3(256), 0, s, st, r, Up, nu, Vp, nv, out);
    else
        hipLaunchKernelGGL(orth_final_kernel, dim3(1), dim3(256), 0, s, st, r, Up, nu, Vp, nv, out);
    return hipGetLastError();
}

#define INST(T)                                                                                              \
    template hipError_t launch_orth<T>(const DevState*, const T*, int, const T*, int, int, double*, int,     \
                                       double*, int, double*, hipStream_t);                                  \
    template hipError_t launch_init_q<T>(T*, int, int, int, hipStream_t);                                    \
    template hipError_t launch_copy_pad<T>(const T*, int64_t, T*, int64_t, int, int, hipStream_t);          \
    template hipError_t launch_factors<T>(const DevState*, const PingPong<T>&, int, int, int, int, T*, T*,    \
                                          double*, hipStream_t);                                             \
    template hipError_t launch_lowrank_pass<T>(LowrankArgs<T>, int, hipStream_t, int*);                            \
    template hipError_t launch_nys_gather<T>(const T*, int64_t, const int64_t*, int, int, int, T*, T*,       \
                                             hipStream_t);
INST(float)
INST(double)
#undef INST

}  // namespace sfr
