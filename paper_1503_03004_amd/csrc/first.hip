// The first sweep of a solve.  FR-ADM (Alg. 1) and FixedRankOptFull
// (Alg. 4) start from B_0 = I_r and V_0 = I_{n x r}, with S_0 = Y_0 = 0, so the
// first L-step input is X = M and P = X V_0 B_0 is simply the first r
// columns of M.  The sweep then needs no row product and no exchange between
// the workgroups that share a row: what remains is Q = M^T P, the column
// partials of which the Gram kernel sums, and ||M||_F for the residual
// scale.  One pass over M (4 or 8 bytes an element) instead of the general
// sweep's band loop.
//
// Wide rows: workgroup (x, y) takes the column slice of 256 VEC columns x
// (one 16-byte vector per thread) and the rows of row group y, staging the group's P rows
// in LDS kFirstChunk at a time, with the M loads of eight rows in flight.
// Row group y writes its own Q partial (one of ncl), so every sum keeps a
// fixed order.
#include "engine.hpp"

namespace sfr {

constexpr int kFirstChunk = 64;    // P rows staged in LDS at a time
constexpr int kFirstInFlight = 8;  // rows of M loads in flight per thread

template <typename T, int VEC>
__device__ __forceinline__ void first_load(const T* p, T (&v)[VEC])
{
    if constexpr (VEC * sizeof(T) == 16) {
        const float4 x = *reinterpret_cast<const float4*>(p);
        __builtin_memcpy(v, &x, 16);
    } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) v[e] = p[e];
    }
}

template <typename T, int R, int VEC>
__global__ void __launch_bounds__(256) first_sweep_kernel(SweepArgs<T> a, int rows)
{
    const DevState* st = a.st;
    if (st->done) return;
    const T* __restrict__ M = static_cast<const T*>(st->M);
    const int64_t ldm = st->ldm;
    const int m = a.m, n = a.n, r = st->r;
    const int tid = threadIdx.x;
    const int grp = blockIdx.y;
    const int i0 = grp * rows, i1 = min(m, i0 + rows);
    const int j = (blockIdx.x * 256 + tid) * VEC;
    const bool jok = j < n;   // n is a multiple of VEC: the vector is all in range or all out
    __shared__ T pch[kFirstChunk * R];
    T q[VEC][R];
#pragma unroll
    for (int e = 0; e < VEC; ++e)
#pragma unroll
        for (int k = 0; k < R; ++k) q[e][k] = T(0);
    double sq = 0.0;
    for (int c0 = i0; c0 < i1; c0 += kFirstChunk) {
        const int cnt = min(kFirstChunk, i1 - c0);
        // P rows of the chunk: M_i[0:r], zero on the padded ranks
        for (int e = tid; e < cnt * R; e += 256) {
            const int row = e / R, k = e % R;
            pch[e] = (k < r) ? M[(int64_t)(c0 + row) * ldm + k] : T(0);
        }
        __syncthreads();
        if (blockIdx.x == 0)
            for (int e = tid; e < cnt * R; e += 256) a.Pnext[(int64_t)c0 * R + e] = pch[e];
        if (jok) {
            for (int b = 0; b < cnt; b += kFirstInFlight) {
                T mv[kFirstInFlight][VEC];
#pragma unroll
                for (int u = 0; u < kFirstInFlight; ++u) {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) mv[u][e] = T(0);
                    if (b + u < cnt) first_load<T, VEC>(M + (int64_t)(c0 + b + u) * ldm + j, mv[u]);
                }
#pragma unroll
                for (int u = 0; u < kFirstInFlight; ++u) {
                    if (b + u >= cnt) break;
                    const T* pr = pch + (b + u) * R;
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        sq = fma((double)mv[u][e], (double)mv[u][e], sq);
#pragma unroll
                        for (int k = 0; k < R; ++k) q[e][k] = fma(mv[u][e], pr[k], q[e][k]);
                    }
                }
            }
        }
        __syncthreads();
    }
    if (jok) {
#pragma unroll
        for (int e = 0; e < VEC; ++e)
#pragma unroll
            for (int k = 0; k < R; ++k) a.Qpart[((size_t)grp * n + j + e) * R + k] = q[e][k];
    }
    // ||M||_F^2 partial of the workgroup: wavefronts by shuffles, then the
    // four wavefront sums in order
    __shared__ double red[4];
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = sq;
    __syncthreads();
    if (tid == 0) a.dy2part[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// Narrow rows (fewer than 256 vectors): thread t takes column vector
// t mod CPV (CPV = n / VEC) of every RPP-th row of the chunk (RPP = 256 div
// CPV rows at a time), as the row-packed returned-S pass does.  The thread
// sums of a column vector are then added across its RPP row subgroups in
// subgroup order, eight ranks at a time through LDS, and one workgroup writes
// one Q partial.
template <typename T, int R, int VEC>
__global__ void __launch_bounds__(256) first_narrow_kernel(SweepArgs<T> a, int rows)
{
    const DevState* st = a.st;
    if (st->done) return;
    const T* __restrict__ M = static_cast<const T*>(st->M);
    const int64_t ldm = st->ldm;
    const int m = a.m, n = a.n, r = st->r;
    const int tid = threadIdx.x;
    const int cpv = n / VEC, rpp = 256 / cpv;
    const int cv = tid % cpv, rr = tid / cpv;
    const bool tact = rr < rpp;
    const int j = cv * VEC;
    const int grp = blockIdx.y;
    const int i0 = grp * rows, i1 = min(m, i0 + rows);
    __shared__ T pch[kFirstChunk * R];
    T q[VEC][R];
#pragma unroll
    for (int e = 0; e < VEC; ++e)
#pragma unroll
        for (int k = 0; k < R; ++k) q[e][k] = T(0);
    double sq = 0.0;
    for (int c0 = i0; c0 < i1; c0 += kFirstChunk) {
        const int cnt = min(kFirstChunk, i1 - c0);
        for (int e = tid; e < cnt * R; e += 256) {
            const int row = e / R, k = e % R;
            pch[e] = (k < r) ? M[(int64_t)(c0 + row) * ldm + k] : T(0);
        }
        __syncthreads();
        for (int e = tid; e < cnt * R; e += 256) a.Pnext[(int64_t)c0 * R + e] = pch[e];
        if (tact) {
            for (int b = rr; b < cnt; b += kFirstInFlight * rpp) {
                T mv[kFirstInFlight][VEC];
#pragma unroll
                for (int u = 0; u < kFirstInFlight; ++u) {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) mv[u][e] = T(0);
                    const int row = b + u * rpp;
                    if (row < cnt) first_load<T, VEC>(M + (int64_t)(c0 + row) * ldm + j, mv[u]);
                }
#pragma unroll
                for (int u = 0; u < kFirstInFlight; ++u) {
                    const int row = b + u * rpp;
                    if (row >= cnt) break;
                    const T* pr = pch + row * R;
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        sq = fma((double)mv[u][e], (double)mv[u][e], sq);
#pragma unroll
                        for (int k = 0; k < R; ++k) q[e][k] = fma(mv[u][e], pr[k], q[e][k]);
                    }
                }
            }
        }
        __syncthreads();
    }
    // the RPP subgroup sums of each column vector, added in subgroup order
    constexpr int KC = 8;
    __shared__ T qs[256 * VEC * KC];
#pragma unroll
    for (int k0 = 0; k0 < R; k0 += KC) {
        if (tact) {
#pragma unroll
            for (int e = 0; e < VEC; ++e)
#pragma unroll
                for (int kk = 0; kk < KC; ++kk)
                    if (k0 + kk < R) qs[(tid * VEC + e) * KC + kk] = q[e][k0 + kk];
        }
        __syncthreads();
        if (tid < cpv) {
#pragma unroll
            for (int e = 0; e < VEC; ++e)
#pragma unroll
                for (int kk = 0; kk < KC; ++kk) {
                    if (k0 + kk >= R) continue;
                    T sum = T(0);
                    for (int g = 0; g < rpp; ++g) sum += qs[((g * cpv + tid) * VEC + e) * KC + kk];
                    a.Qpart[((size_t)grp * n + tid * VEC + e) * R + k0 + kk] = sum;
                }
        }
        __syncthreads();
    }
    __shared__ double red[4];
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = sq;
    __syncthreads();
    if (tid == 0) a.dy2part[blockIdx.y] = (red[0] + red[1]) + (red[2] + red[3]);
}

// About kFirstGroups workgroups in all, at most kFirstMaxGroups row groups
// (each one a Q partial the Gram kernel adds), at least 8 rows a group.
constexpr int kFirstGroups = 1024;
constexpr int kFirstMaxGroups = 64;

FirstPlan first_sweep_plan(const Engine& e)
{
    FirstPlan f;
    const int vec = e.vec;
    if (e.ne < 256 * vec) {
        // narrow rows: one workgroup per row group, rows packed (at least 8 a group)
        f.narrow = true;
        f.gx = 1;
        const int gy = std::max(1, std::min(kFirstGroups, (e.m + 7) / 8));
        f.rows = (e.m + gy - 1) / gy;
        f.gy = (e.m + f.rows - 1) / f.rows;
        f.ok = f.gy <= kMaxDyPartials;
        return f;
    }
    f.gx = (e.ne + 256 * vec - 1) / (256 * vec);
    int gy = std::max(1, std::min(kFirstMaxGroups, (kFirstGroups + f.gx - 1) / f.gx));
    gy = std::max(1, std::min(gy, (e.m + 7) / 8));
    f.rows = (e.m + gy - 1) / gy;
    f.gy = (e.m + f.rows - 1) / f.rows;
    f.ok = f.gx * f.gy <= kMaxDyPartials;
    return f;
}

template <typename T>
hipError_t launch_first_sweep(const SweepArgs<T>& a, int R, const FirstPlan& f, hipStream_t s)
{
    constexpr int V = 16 / sizeof(T);
    const dim3 grid((unsigned)f.gx, (unsigned)f.gy);
    switch (R) {
#define CASE(rr)                                                                                      \
    case rr:                                                                                          \
        if (f.narrow) hipLaunchKernelGGL((first_narrow_kernel<T, rr, V>), grid, dim3(256), 0, s, a, f.rows); \
        else hipLaunchKernelGGL((first_sweep_kernel<T, rr, V>), grid, dim3(256), 0, s, a, f.rows);  \
        break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(8) CASE(10) CASE(12) CASE(16) CASE(20) CASE(24)
        CASE(32)
#undef CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template hipError_t launch_first_sweep<float>(const SweepArgs<float>&, int, const FirstPlan&, hipStream_t);
template hipError_t launch_first_sweep<double>(const SweepArgs<double>&, int, const FirstPlan&, hipStream_t);

}  // namespace sfr
