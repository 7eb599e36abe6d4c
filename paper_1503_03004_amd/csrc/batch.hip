// Batched FR-ADM for many small independent problems (FP32 data, FP64 r x r
// algebra): one workgroup solves one problem from start to finish.
//
// For small m x n (n <= 512) a solve through the single-problem engine is
// dominated by launches and host waits (three kernels per iteration).  Here
// a workgroup of 8 wavefronts keeps the whole iteration on one CU:
//   * sweep k (Alg. 1 with the one-pass Alg. 2 products, as sweep.hip):
//     bands of 8 rows, one row per wavefront, lanes over the columns; l_ij
//     from a_i = P_i T_U and V_j (LDS); the S/dual step writes Y_k; x goes to
//     LDS; p_i by a wavefront reduction; thread j accumulates
//     Q_j += x_ij p_i in registers; G_P accumulates in FP64 per band;
//   * then G_Q, the stopping test of iteration k - 1 and the FP64 step
//     (lstep_algebra, the whole workgroup), V_{k+1} = Q T_V into LDS;
//   * after the last iteration the factors U, B, V and S are written.
// Y (two buffers), P and Q (two buffers each) live in a per-slot workspace
// in HBM; nothing leaves the CU between iterations except those streams.
// The iteration, its stopping rule and its outputs are those of the
// single-problem engine (same kernels' arithmetic, FP32 streams).
#include "sfr_internal.hpp"
#include "small_la.hpp"

namespace sfr {

constexpr int kBNW = 8;               // wavefronts per workgroup
constexpr int kBTPB = 64 * kBNW;      // threads per workgroup
constexpr int kBNMax = 512;           // widest problem (columns)
constexpr int kBNV = kBNMax / 64;     // columns per lane per row

template <int R>
__global__ void __launch_bounds__(kBTPB, 1) batch_kernel(BatchItemDev* items, BatchParams bp)
{
    static_assert(R <= 16, "batched solver: r <= 16");
    constexpr int E = R * (R + 1) / 2;
    constexpr int NT = kBTPB;
    BatchItemDev* it = items + blockIdx.x;
    const int m = it->m, n = it->n, r = it->r, ldy = it->ldy;
    const int64_t ldm = it->ldm;
    const float* __restrict__ M = it->M;
    const float lam = (float)it->lambda;

    __shared__ float Vs[R * kBNMax];          // V_k, k-major (Vs[k n + j]); Q staging between iterations
    __shared__ float Xs[kBNW * kBNMax];       // x of the band
    __shared__ float Ps[kBNW * 16];           // p of the band's rows
    __shared__ float TUs[R * R];              // row factor transform (FP32)
    __shared__ double Gp[R * LDP], Gq[R * LDP], Bm[R * LDP], C1[R * LDP], C2[R * LDP];
    __shared__ double Km[R * LDP], T1[R * LDP], T2[R * LDP], Ev[R * LDP], Ev2[R * LDP];
    __shared__ double TUb[R * LDP], TVd[R * LDP];   // U and V transforms of the last step
    __shared__ double tri[2][E];
    __shared__ double red[kBNW];
    __shared__ __align__(16) double cs[2 * 16];
    __shared__ double wbuf[kMaxR];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    // ---- initial state of Alg. 1: V_1 = I_{n x r}, B_0 = I, warm bases I
    for (int e = tid; e < R * n; e += NT) {
        const int k = e / n, j = e % n;
        Vs[e] = (j == k && k < r) ? 1.f : 0.f;
    }
    for (int e = tid; e < R * R; e += NT) {
        const int i = e / R, j = e % R;
        const double id = (i == j) ? 1.0 : 0.0;
        Bm[i * LDP + j] = id;
        Ev[i * LDP + j] = id;
        Ev2[i * LDP + j] = id;
        TUb[i * LDP + j] = 0.0;
        TVd[i * LDP + j] = id;
        TUs[e] = 0.f;
    }
    __syncthreads();

    double mu = it->mu0, mu_prev = it->mu0, nrmM = 0.0, res = 0.0;
    int32_t status = kOK, iters = 0;
    const int nbands = (m + kBNW - 1) / kBNW;
    for (int k = 1;; ++k) {
        const int mode = (k == 1) ? 0 : (k == 2 ? 1 : 2);
        const float* Yp = ((k - 1) & 1) ? it->Y1 : it->Y0;
        float* Yn = (k & 1) ? it->Y1 : it->Y0;
        const float* Pp = ((k - 1) & 1) ? it->P1 : it->P0;
        float* Pn = (k & 1) ? it->P1 : it->P0;
        float* Qn = (k & 1) ? it->Q1 : it->Q0;
        const float mup = (float)mu_prev;
        const float imup = (mode != 0) ? (float)(1.0 / mu_prev) : 0.f;
        const float imuc = (float)(1.0 / mu);

        // ---------------- sweep k ----------------
        float q[R];
#pragma unroll
        for (int kk = 0; kk < R; ++kk) q[kk] = 0.f;
        double gp = 0.0;      // G_P entry `tid` (tid < E)
        int gx = 0, gy = 0;
        if (tid < E) {
            int rem = tid;
            while (rem >= R - gx) { rem -= R - gx; ++gx; }
            gy = gx + rem;
        }
        double acc2 = 0.0;
        for (int b = 0; b < nbands; ++b) {
            const int i = b * kBNW + wave;
            const bool row_ok = i < m;
            float av[R];
            if (mode != 0) {
                float s = 0.f;
                if (lane < R && row_ok) {
#pragma unroll
                    for (int t = 0; t < R; ++t) s = fmaf(Pp[(int64_t)i * R + t], TUs[t * R + lane], s);
                }
#pragma unroll
                for (int kk = 0; kk < R; ++kk) av[kk] = __shfl(s, kk, 64);
            }
            float p[R];
#pragma unroll
            for (int kk = 0; kk < R; ++kk) p[kk] = 0.f;
            float rowacc = 0.f;
#pragma unroll 2
            for (int v = 0; v < kBNV; ++v) {
                const int j = lane + 64 * v;
                const bool jok = j < n;
                const bool ok = row_ok && jok;
                const float mv = ok ? M[(int64_t)i * ldm + j] : 0.f;
                float x;
                if (mode == 0) {
                    x = mv;
                    rowacc = fmaf(mv, mv, rowacc);
                } else {
                    const float yp = (ok && mode == 2) ? Yp[(int64_t)i * ldy + j] : 0.f;
                    float l = 0.f;
                    if (jok) {
#pragma unroll
                        for (int kk = 0; kk < R; ++kk) l = fmaf(av[kk], Vs[kk * n + j], l);
                    }
                    const float Rr = mv - l + yp * imup;
                    const float y = fminf(fmaxf(mup * Rr, -lam), lam);
                    const float dy = y - yp;
                    rowacc = fmaf(dy, dy, rowacc);
                    x = l + dy * imup + y * imuc;
                    if (ok) Yn[(int64_t)i * ldy + j] = y;
                }
                x = ok ? x : 0.f;
                Xs[wave * kBNMax + j] = x;
                if (jok) {
#pragma unroll
                    for (int kk = 0; kk < R; ++kk) p[kk] = fmaf(x, Vs[kk * n + j], p[kk]);
                }
            }
            acc2 += (double)rowacc;
#pragma unroll
            for (int kk = 0; kk < R; ++kk)
                for (int off = 32; off > 0; off >>= 1) p[kk] += __shfl_xor(p[kk], off, 64);
            if (lane < 16) {
                float mine = 0.f;
#pragma unroll
                for (int kk = 0; kk < R; ++kk) mine = (kk == lane) ? p[kk] : mine;
                Ps[wave * 16 + lane] = row_ok ? mine : 0.f;
                if (row_ok && lane < R) Pn[(int64_t)i * R + lane] = mine;
            }
            __syncthreads();
            // column pass: thread j owns column j; FP64 G_P of the band's rows
            if (tid < n) {
#pragma unroll 2
                for (int h = 0; h < kBNW; ++h) {
                    const float xv = Xs[h * kBNMax + tid];
#pragma unroll
                    for (int kk = 0; kk < R; ++kk) q[kk] = fmaf(xv, Ps[h * 16 + kk], q[kk]);
                }
            }
            if (tid < E) {
                for (int h = 0; h < kBNW; ++h) gp = fma((double)Ps[h * 16 + gx], (double)Ps[h * 16 + gy], gp);
            }
            __syncthreads();
        }
        // Q_k: to the workspace (the returned factors read it) and to LDS
        if (tid < n) {
#pragma unroll
            for (int kk = 0; kk < R; ++kk) {
                Qn[(int64_t)tid * R + kk] = q[kk];
                Vs[tid * R + kk] = q[kk];
            }
        }
        // ||Y_k - Y_{k-1}||^2 (mode 0: ||M||^2)
        for (int off = 32; off > 0; off >>= 1) acc2 += __shfl_xor(acc2, off, 64);
        if (lane == 0) red[wave] = acc2;
        __syncthreads();
        double total = 0.0;
#pragma unroll
        for (int w = 0; w < kBNW; ++w) total += red[w];

        // ---------------- stopping test of iteration k - 1 ----------------
        bool stop = false;
        if (k == 1) {
            nrmM = sqrt(total);
            if (!(nrmM > 0.0) || !isfinite(nrmM)) { status = kErrNonFinite; iters = 0; stop = true; }
        } else {
            res = sqrt(total) / (mu_prev * nrmM);
            const int kdone = k - 1;
            if (!isfinite(res)) { stop = true; status = kErrNonFinite; }
            else if (bp.fixed_iters > 0) { stop = kdone >= bp.fixed_iters; }
            else if (res <= it->tol) { stop = true; }
            else if (kdone >= bp.max_iter) { stop = true; status = kWarnMaxIter; }
            if (stop) iters = kdone;
        }
        if (stop) break;

        // ---------------- FP64 step: Grams, Alg. 2 projectors ----------------
        if (tid < E) {
            double gq = 0.0;
            for (int j = 0; j < n; ++j) gq = fma((double)Vs[j * R + gx], (double)Vs[j * R + gy], gq);
            tri[0][tid] = gp;
            tri[1][tid] = gq;
        }
        __syncthreads();
        for (int e = tid; e < R * R; e += NT) {
            const int i = e / R, j = e % R;
            const int x = i < j ? i : j, y = i < j ? j : i;
            const int t = x * R - x * (x - 1) / 2 + (y - x);
            const bool pad = (i >= r) || (j >= r);
            Gp[i * LDP + j] = pad ? (i == j ? 1.0 : 0.0) : tri[0][t];
            Gq[i * LDP + j] = pad ? (i == j ? 1.0 : 0.0) : tri[1][t];
        }
        __syncthreads();
        if (!lstep_algebra<R, NT>(Gp, Gq, Bm, C1, C2, Km, T1, T2, Ev, Ev2, cs, wbuf, r)) {
            status = kErrRank;
            iters = k - 1;
            break;
        }
        // the step's transforms (padded block dropped), B_k, and V_{k+1} = Q_k T_V
        float vn[R];
        if (tid < n) {
#pragma unroll
            for (int kk = 0; kk < R; ++kk) {
                float s = 0.f;
                if (kk < r) {
#pragma unroll
                    for (int t = 0; t < R; ++t)
                        if (t < r) s = fmaf(Vs[tid * R + t], (float)Gp[t * LDP + kk], s);
                }
                vn[kk] = s;
            }
        }
        for (int e = tid; e < R * R; e += NT) {
            const int i = e / R, j = e % R;
            const bool in = (i < r) && (j < r);
            TUs[e] = in ? (float)Km[i * LDP + j] : 0.f;
            TUb[i * LDP + j] = in ? T1[i * LDP + j] : 0.0;
            TVd[i * LDP + j] = in ? Gp[i * LDP + j] : 0.0;
            Bm[i * LDP + j] = in ? T2[i * LDP + j] : (i == j ? 1.0 : 0.0);
        }
        __syncthreads();
        if (tid < n) {
#pragma unroll
            for (int kk = 0; kk < R; ++kk) Vs[kk * n + tid] = vn[kk];
        }
        mu_prev = mu;
        const double nm = bp.rho * mu;
        mu = nm < bp.mu_bar ? nm : bp.mu_bar;
        __syncthreads();
    }
    __syncthreads();

    // ---------------- outputs of the returned iterate K = iters ----------------
    double min_eig = 0.0;
    if (status >= 0) {
        const int K = iters;
        const float* PK = (K & 1) ? it->P1 : it->P0;
        const float* QK = (K & 1) ? it->Q1 : it->Q0;
        const float* YK = (K >= 2) ? ((K & 1) ? it->Y1 : it->Y0) : nullptr;
        // U = P TUbar, V = Q TV (FP64 accumulation), B
        for (int e = tid; e < m * r; e += NT) {
            const int i = e / r, kk = e % r;
            double s = 0.0;
            for (int t = 0; t < r; ++t) s = fma((double)PK[(int64_t)i * R + t], TUb[t * LDP + kk], s);
            it->U[(int64_t)i * r + kk] = (float)s;
        }
        // V_K for the S pass (FP32, k-major in Vs) and the returned V
        for (int e = tid; e < n * R; e += NT) {
            const int j = e / R, kk = e % R;
            double s = 0.0;
            if (kk < r) {
                for (int t = 0; t < r; ++t) s = fma((double)QK[(int64_t)j * R + t], TVd[t * LDP + kk], s);
                it->V[(int64_t)j * r + kk] = (float)s;
            }
            Vs[kk * n + j] = (float)s;
        }
        for (int e = tid; e < r * r; e += NT) it->B[e] = Bm[(e / r) * LDP + e % r];
        __syncthreads();
        if (it->S) {
            const float t = (float)(it->lambda / mu_prev), imu = (float)(1.0 / mu_prev);
            for (int i = wave; i < m; i += kBNW) {
                float s = 0.f;
                if (lane < R) {
                    for (int tt = 0; tt < R; ++tt) s = fmaf(PK[(int64_t)i * R + tt], TUs[tt * R + lane], s);
                }
                float av[R];
#pragma unroll
                for (int kk = 0; kk < R; ++kk) av[kk] = __shfl(s, kk, 64);
                for (int j = lane; j < n; j += 64) {
                    float l = 0.f;
#pragma unroll
                    for (int kk = 0; kk < R; ++kk) l = fmaf(av[kk], Vs[kk * n + j], l);
                    const float yv = YK ? YK[(int64_t)i * ldy + j] : 0.f;
                    const float Rr = M[(int64_t)i * ldm + j] - l + yv * imu;
                    const float a1 = Rr - t, b1 = Rr + t;
                    it->S[(int64_t)i * it->lds + j] = (a1 > 0.f ? a1 : 0.f) + (b1 < 0.f ? b1 : 0.f);
                }
            }
        }
        // smallest eigenvalue of the returned B (Appendix, Lemma 2)
        min_eig = wmin_eig<R, NT>(Bm, LDP, r, C1, C2, cs);
    }
    if (tid == 0) {
        it->iters = iters;
        it->status = status;
        it->res = res;
        it->min_eig_B = min_eig;
        it->mu_final = mu_prev;
    }
}

#define SFR_BATCH_R_LIST(X) X(1) X(2) X(3) X(4) X(5) X(6) X(8) X(10) X(12) X(16)

hipError_t launch_batch(BatchItemDev* items, int count, int R, const BatchParams& bp, hipStream_t s)
{
    switch (R) {
#define CASE(rr)                                                                                \
    case rr: hipLaunchKernelGGL(batch_kernel<rr>, dim3(count), dim3(kBTPB), 0, s, items, bp); \
        return hipGetLastError();
        SFR_BATCH_R_LIST(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sfr
