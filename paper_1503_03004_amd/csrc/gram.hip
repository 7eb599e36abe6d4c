// Gram matrices of one FR-ADM iteration: the cluster partials of Q summed
// into Q, and the FP64 upper triangles of G_Q = Q^T Q and G_P = P^T P per
// workgroup, then (large r x r problems) the partials summed per entry.
#include "sfr_internal.hpp"

namespace sfr {

// Sum the cluster partials of Q (fixed order), write Q, and form the
// upper triangles of G_Q = Q^T Q and G_P = P^T P in FP64 per workgroup.
//
// A workgroup takes its rows in segments held in LDS as FP64.  P is m x R
// row-major, so a P segment is one contiguous run that each thread reads
// with kGramU coalesced loads, all in flight together.  A Q entry is the
// sum of its ncl cluster partials: the clusters of an entry are cut into NS
// contiguous slots, one thread per (entry, slot) with the loads of a slot
// in flight together, and the slot sums are added in slot order.  The Gram
// entries are then split over G row classes (rows jl = g mod G, G threads
// per entry) whose sums are added in class order.  Every sum has a fixed
// order, so results are bitwise repeatable.
template <typename T, int R>
__global__ void __launch_bounds__(kTPB) gram_kernel(GramArgs<T> a)
{
    if (a.st->done) return;
    constexpr int E = R * (R + 1) / 2;
    constexpr int SEGP = (kGramU * kTPB) / R;       // P rows per segment
    constexpr int SEGQ = kTPB / R;                  // Q rows per segment
    constexpr int G = (E >= kTPB) ? 1 : kTPB / E;   // threads per Gram entry
    constexpr int EU = (E + kTPB - 1) / kTPB;       // Gram entries per thread (G == 1)
    constexpr int CH = 32;                          // cluster partials in flight per thread
    __shared__ double tile[SEGP * R];
    __shared__ T qslot[kTPB];
    __shared__ double gred[kTPB];
    const int tid = threadIdx.x;
    const int blk = blockIdx.x;
    const bool isq = blk < a.nqb;
    const int nrows = isq ? a.n : a.m;
    const int per = isq ? a.rows_q : a.rows_p;
    const int r0 = (isq ? blk : blk - a.nqb) * per;
    const int r1 = min(nrows, r0 + per);
    const int seg = isq ? SEGQ : SEGP;

    // Gram entries of this thread: (x, y), x <= y, of entry e
    const int g = (G > 1) ? tid / E : 0;
    const bool gact = (G > 1) ? (tid < E * G) : true;
    int ex[EU], ey[EU];
    double acc[EU];
#pragma unroll
    for (int u = 0; u < EU; ++u) {
        int e = (G > 1) ? tid % E : tid + u * kTPB;
        if (e >= E) e = E - 1;
        int x = 0, rem = e;
        while (rem >= R - x) { rem -= R - x; ++x; }
        ex[u] = x;
        ey[u] = x + rem;
        acc[u] = 0.0;
    }

    for (int base = r0; base < r1; base += seg) {
        const int nr = min(seg, r1 - base);
        const int ne = nr * R;
        if (isq) {
            const int ns = kTPB / ne;                   // slots per entry (ne <= kTPB)
            const int cps = (a.ncl + ns - 1) / ns;      // clusters per slot
            if (tid < ne * ns) {
                const int e = tid % ne, sl = tid / ne;
                const int j = base + e / R, k = e % R;
                const int c0 = sl * cps, c1 = min(a.ncl, c0 + cps);
                T sum = 0;
                for (int cb = c0; cb < c1; cb += CH) {
                    T w[CH];
#pragma unroll
                    for (int u = 0; u < CH; ++u)
                        w[u] = a.Qpart[((size_t)min(cb + u, a.ncl - 1) * a.n + j) * R + k];
#pragma unroll
                    for (int u = 0; u < CH; ++u) sum += (cb + u < c1) ? w[u] : T(0);
                }
                qslot[tid] = sum;
            }
            __syncthreads();
            if (tid < ne) {
                T sum = 0;
                for (int sl = 0; sl < ns; ++sl) sum += qslot[sl * ne + tid];
                a.Qnext[(int64_t)base * R + tid] = sum;
                tile[tid] = (double)sum;
            }
        } else {
            const T* src = a.Pnext + (int64_t)base * R;
            T v[kGramU];
#pragma unroll
            for (int u = 0; u < kGramU; ++u) v[u] = src[min(tid + u * kTPB, ne - 1)];
#pragma unroll
            for (int u = 0; u < kGramU; ++u)
                if (tid + u * kTPB < ne) tile[tid + u * kTPB] = (double)v[u];
        }
        __syncthreads();
        if (G > 1) {
            if (gact) {
                const int x = ex[0], y = ey[0];
                double sum = 0.0;
                for (int jl = g; jl < nr; jl += G) sum = fma(tile[jl * R + x], tile[jl * R + y], sum);
                acc[0] += sum;
            }
        } else {
#pragma unroll
            for (int u = 0; u < EU; ++u) {
                if (tid + u * kTPB < E) {
                    const int x = ex[u], y = ey[u];
                    double sum = 0.0;
                    for (int jl = 0; jl < nr; ++jl) sum = fma(tile[jl * R + x], tile[jl * R + y], sum);
                    acc[u] += sum;
                }
            }
        }
        __syncthreads();
    }
    double* out = isq ? (a.GQpart + (size_t)blk * E) : (a.GPpart + (size_t)(blk - a.nqb) * E);
    if (G > 1) {
        if (gact) gred[tid] = acc[0];                   // tid = g * E + e
        __syncthreads();
        if (tid < E) {
            double sum = 0.0;
            for (int gg = 0; gg < G; ++gg) sum += gred[gg * E + tid];
            out[tid] = sum;
        }
    } else {
#pragma unroll
        for (int u = 0; u < EU; ++u)
            if (tid + u * kTPB < E) out[tid + u * kTPB] = acc[u];
    }

}

// Sum of the Gram partials: entry e of G_Q (e < E) or G_P (E <= e < 2E)
// becomes the sum of its nqb or npb partials, added in a fixed order
// (kGramSlices contiguous slices, the slice sums in slice order), written
// over partial 0.  One workgroup per kGramRedEntries entries, every thread
// with its (at most kMaxGramPartials / kGramSlices) loads in flight
// together: the step kernel then reads one value per entry.
constexpr int kGramRedEntries = 16;
constexpr int kGramSlices = kTPB / kGramRedEntries;

__global__ void __launch_bounds__(kTPB) gram_reduce_kernel(const DevState* st, double* GQpart, int nqb,
                                                           double* GPpart, int npb, int E)
{
    if (st->done) return;
    __shared__ double part[kGramSlices][kGramRedEntries];
    const int tid = threadIdx.x;
    const int el = tid % kGramRedEntries, sl = tid / kGramRedEntries;
    const int w = blockIdx.x * kGramRedEntries + el;
    const bool ok = w < 2 * E;
    const bool isq = w < E;
    double* base = isq ? GQpart : GPpart;
    const int cnt = isq ? nqb : npb;
    const int e = ok ? (isq ? w : w - E) : 0;
    const int per = (cnt + kGramSlices - 1) / kGramSlices;
    const int q0 = sl * per, q1 = min(cnt, q0 + per);
    constexpr int CH = (kMaxGramPartials + kGramSlices - 1) / kGramSlices;
    double s = 0.0;
    for (int qb = q0; qb < q1; qb += CH) {
        double v[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) v[u] = base[(size_t)min(qb + u, cnt - 1) * E + e];
#pragma unroll
        for (int u = 0; u < CH; ++u) s += (qb + u < q1) ? v[u] : 0.0;
    }
    part[sl][el] = s;
    __syncthreads();
    if (sl == 0 && ok) {
        double t = 0.0;
#pragma unroll
        for (int g = 0; g < kGramSlices; ++g) t += part[g][el];
        base[e] = t;
    }
}

hipError_t launch_gram_reduce(const DevState* st, double* GQpart, int nqb, double* GPpart, int npb, int E,
                              hipStream_t s)
{
    const int grid = (2 * E + kGramRedEntries - 1) / kGramRedEntries;
    hipLaunchKernelGGL(gram_reduce_kernel, dim3(grid), dim3(kTPB), 0, s, st, GQpart, nqb, GPpart, npb, E);
    return hipGetLastError();
}

#define SFR_R_LIST(X) X(1) X(2) X(3) X(4) X(5) X(6) X(8) X(10) X(12) X(16) X(20) X(24) X(32)

template <typename T>
hipError_t launch_gram(const GramArgs<T>& a, int R, hipStream_t s)
{
    const int grid = a.nqb + a.npb;
    switch (R) {
#define CASE(r)                                                                     \
    case r:                                                                         \
        hipLaunchKernelGGL((gram_kernel<T, r>), dim3(grid), dim3(kTPB), 0, s, a); \
        return hipGetLastError();
        SFR_R_LIST(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_gram<float>(const GramArgs<float>&, int, hipStream_t);
template hipError_t launch_gram<double>(const GramArgs<double>&, int, hipStream_t);

}  // namespace sfr
