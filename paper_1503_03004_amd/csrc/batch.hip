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
#include "mfma_bf16.hpp"
#include "sfr_internal.hpp"
#include "small_la.hpp"

#include <stdlib.h>

namespace sfr {

constexpr int kBNW = 8;               // wavefronts per workgroup
constexpr int kBTPB = 64 * kBNW;      // threads per workgroup
constexpr int kBNMax = 512;           // widest problem (columns)
constexpr int kBNV = kBNMax / 64;     // columns per lane per row

// Global-memory views of the descriptor's pointers.  Loaded from memory,
// the pointers would otherwise be generic (flat) ones: flat accesses also
// count against the LDS wait counter, so every LDS wait of the band loop
// would wait for the in-flight HBM loads and stores as well.
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) double gdouble;
template <typename T>
__device__ inline __attribute__((address_space(1))) T* as_global(T* p)
{
    return (__attribute__((address_space(1))) T*)p;
}

template <bool B> struct BoolTag { static constexpr bool value = B; };

typedef float bf32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf32x4 bmfma4(float a, float b, bf32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Matrix-core form of the band loop (wide problems, R = 8..16): bands of 16
// rows; wavefront w owns the 16-column tiles w, w + 8, w + 16, w + 24.  The
// contractions run on v_mfma_f32_16x16x4_f32 with the single-problem
// matrix-core sweep's lane layout (lane l: lr = l % 16, lq = l / 16 supplies
// A[lr][lq], B[lq][lr] and receives D[4 lq + e][lr]):
//   l   (16 columns x 16 rows of a tile) = V_tile . a_band^T      K = R
//   p   (R x 16 rows)                   += V_tile^T-slices . x    K = 16 columns
//   Q   (16 columns x R)                += x_tile^T . P_band      K = 16 rows
// so lane (lr, lq) holds row lr, columns 4 lq .. 4 lq + 3 of each tile.
constexpr int kMB = 16;                 // rows per band
constexpr int kMXP = 4 * 16 + 16;       // LDS pitch of a wavefront's x rows (4 tiles + pad)

__device__ inline float lane_bcast(float v, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}

// RW rows per wavefront per band (a band is 8 RW rows): two rows share each
// V column read; one row keeps the larger ranks' band loop within registers.
template <int R, int RW, bool NARROW, bool MF>
__device__ __forceinline__ void batch_solve(BatchItemDev* it, const BatchParams& bp)
{
    static_assert(R <= 16, "batched solver: r <= 16");
    static_assert(!MF || (!NARROW && R >= 8), "matrix-core form: wide problems, R >= 8");
    constexpr int kBRW = RW;
    constexpr int kBH = kBNW * RW;        // rows per band
    constexpr int E = R * (R + 1) / 2;
    constexpr int NT = kBTPB;
    constexpr int RP = (R + 3) / 4 * 4;   // rank padded to whole float4 groups
    constexpr int RC = RP / 4;
    constexpr int GS = NT / E;            // threads per G_Q entry
    // the descriptor is read once (uniform: scalar loads) and its pointers
    // are held in registers for the whole solve
    const BatchItemDev d = *it;
    const int m = d.m, n = d.n, r = d.r, ldy = d.ldy;
    const int64_t ldm = d.ldm;
    const gfloat* __restrict__ M = as_global(d.M);
    const float lam = (float)d.lambda;
    gfloat* const Y0 = as_global(d.Y0);
    gfloat* const Y1 = as_global(d.Y1);
    gfloat* const P0 = as_global(d.P0);
    gfloat* const P1 = as_global(d.P1);
    gfloat* const Q0 = as_global(d.Q0);
    gfloat* const Q1 = as_global(d.Q1);

    // V_k in float4 groups of 4 rank entries: (k, j) at ((k/4) kBNMax + j) 4 + k%4,
    // so a lane reads the R entries of its column with R/4 128-bit reads.
    // Between the sweep and the step the same space stages Q_k (Vs[j R + k]).
    __shared__ __align__(16) float Vs[RP * kBNMax];
    __shared__ __align__(16) float Xs[MF ? 1024 : kBH * kBNMax];   // x of the band; FP64 G_Q partials in the step
    __shared__ __align__(16) float Ps[MF ? 16 : kBH * 8 * 16];     // p of the band's rows (up to 8 rows per wavefront step)
    // matrix-core form: per-wavefront x tiles, per-wavefront p partials, the band's p
    __shared__ __align__(16) float XwA[MF ? kBNW * kMB * kMXP : 1];
    __shared__ __align__(16) float PWA[MF ? kBNW * 256 : 1];
    __shared__ __align__(16) float PSA[MF ? 256 : 1];
    __shared__ __align__(16) float TUt[R * RP];        // T_U transposed: TUt[k RP + t] = T_U[t][k]
    __shared__ __align__(16) float TVt[R * RP];        // T_V transposed (FP32)
    __shared__ double Gp[R * LDP], Gq[R * LDP], Bm[R * LDP], C1[R * LDP], C2[R * LDP];
    __shared__ double Km[R * LDP], T1[R * LDP], T2[R * LDP], Ev[R * LDP], Ev2[R * LDP];
    __shared__ double TUb[R * LDP], TVd[R * LDP];   // U and V transforms of the last step
    __shared__ double tri[2][E];
    __shared__ double red[kBNW];
    __shared__ __align__(16) double cs[2 * 16];
    __shared__ double wbuf[kMaxR];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    auto vat = [](int kk, int j) { return ((kk >> 2) * kBNMax + j) * 4 + (kk & 3); };

    // ---- initial state of Alg. 1: V_1 = I_{n x r}, B_0 = I, warm bases I
    for (int e = tid; e < RP * n; e += NT) {
        const int kk = e / n, j = e % n;
        Vs[vat(kk, j)] = (j == kk && kk < r) ? 1.f : 0.f;
    }
    for (int e = tid; e < R * R; e += NT) {
        const int i = e / R, j = e % R;
        const double id = (i == j) ? 1.0 : 0.0;
        Bm[i * LDP + j] = id;
        Ev[i * LDP + j] = id;
        Ev2[i * LDP + j] = id;
        TUb[i * LDP + j] = 0.0;
        TVd[i * LDP + j] = id;
    }
    for (int e = tid; e < R * RP; e += NT) TUt[e] = 0.f;
    __syncthreads();

    // G_P entry of thread tid (tid < E) and G_Q entry of thread tid (tid < GS E)
    int gx = 0, gy = 0, qx = 0, qy = 0;
    if (tid < E) {
        int rem = tid;
        while (rem >= R - gx) { rem -= R - gx; ++gx; }
        gy = gx + rem;
    }
    if (tid < GS * E) {
        int rem = tid % E;
        while (rem >= R - qx) { rem -= R - qx; ++qx; }
        qy = qx + rem;
    }

    double mu = d.mu0, mu_prev = d.mu0, nrmM = 0.0, res = 0.0;
    int32_t status = kOK, iters = 0;
    // lanes per row: the fewest (8 .. 64) that cover n with 8 columns per
    // lane, and at least R (a group's lanes form the entries of a_i)
    int lpr = 8;
    while (lpr * kBNV < n) lpr <<= 1;
    if (lpr < (R <= 8 ? 8 : 16)) lpr = (R <= 8 ? 8 : 16);
    for (int k = 1;; ++k) {
        const int mode = (k == 1) ? 0 : (k == 2 ? 1 : 2);
        const gfloat* Yp = ((k - 1) & 1) ? Y1 : Y0;
        gfloat* Yn = (k & 1) ? Y1 : Y0;
        const gfloat* Pp = ((k - 1) & 1) ? P1 : P0;
        gfloat* Pn = (k & 1) ? P1 : P0;
        gfloat* Qn = (k & 1) ? Q1 : Q0;
        const float mup = (float)mu_prev;
        const float imup = (mode != 0) ? (float)(1.0 / mu_prev) : 0.f;
        const float imuc = (float)(1.0 / mu);
        // BF16 operands for the p and Q products of this sweep (matrix-core
        // form only): every sweep while the BF16 phase lasts, i.e. up to
        // bf16_iters iterations and while the last residual is above bf16_tol
        // (either 0: no limit of that kind)
        const bool bfk = MF && bp.bf16 && (bp.bf16_iters <= 0 || k <= bp.bf16_iters) &&
                         (bp.bf16_tol <= 0.0 || k <= 2 || res > bp.bf16_tol);

        // ---------------- sweep k ----------------
        float q[R];
#pragma unroll
        for (int kk = 0; kk < R; ++kk) q[kk] = 0.f;
        double gp = 0.0;      // G_P entry `tid` (tid < E)
        double acc2 = 0.0;
        // NARROW: lpr < 64 lanes per row, 64 / lpr rows per wavefront at once
        // (broadcasts and reductions within lane groups); otherwise one row
        // per wavefront, broadcasts through scalar registers.
        auto sweep_bands = [&](auto tag) __attribute__((always_inline)) {
            const int L = NARROW ? lpr : 64;          // lanes per row
            const int RPW = NARROW ? 64 / lpr : 1;    // rows per wavefront and step
            const int g = NARROW ? lane / lpr : 0;    // row group of this lane
            const int li = NARROW ? (lane & (lpr - 1)) : lane;
            const int HB = kBH * RPW;                 // rows per band
            const int nx = kBNMax / RPW;              // row pitch of Xs
            const int nb = (m + HB - 1) / HB;
            auto row_of = [&](int b, int h) { return b * HB + (h * kBNW + wave) * RPW + g; };
            // The loads of band b + 1 (M, Y_{k-1} and the P rows) are issued
            // before band b is computed, so one band's loads are always in
            // flight behind the arithmetic of the other.
            auto load_band = [&](int b, float* mv, float* yv, float* pr) {
#pragma unroll
                for (int h = 0; h < kBRW; ++h) {
                    const int i = row_of(b, h);
                    const bool row_ok = i < m;
#pragma unroll
                    for (int v = 0; v < kBNV; ++v) {
                        const int j = li + L * v;
                        const bool ok = row_ok && j < n;
                        mv[h * kBNV + v] = ok ? M[(int64_t)i * ldm + j] : 0.f;
                        yv[h * kBNV + v] = (ok && mode == 2) ? Yp[(int64_t)i * ldy + j] : 0.f;
                    }
                    // lane t < R of the row's group holds P_{i,t}
                    pr[h] = (row_ok && mode != 0 && li < R) ? Pp[(int64_t)i * R + li] : 0.f;
                }
            };
            float cm[kBRW * kBNV], cy[kBRW * kBNV], cp[kBRW];
            load_band(0, cm, cy, cp);
            for (int b = 0; b < nb; ++b) {
                float nm[kBRW * kBNV], ny[kBRW * kBNV], np[kBRW];
#pragma unroll
                for (int e = 0; e < kBRW * kBNV; ++e) { nm[e] = 0.f; ny[e] = 0.f; }
#pragma unroll
                for (int e = 0; e < kBRW; ++e) np[e] = 0.f;
                if (b + 1 < nb) load_band(b + 1, nm, ny, np);
                // a_i = P_i T_U for the wavefront's rows
                float av[kBRW][R];
                if (mode != 0) {
#pragma unroll
                    for (int h = 0; h < kBRW; ++h) {
                        float s = 0.f;
                        if constexpr (!NARROW) {
                            // one row: uniform over the wavefront (scalar registers)
                            float pt[R];
#pragma unroll
                            for (int t = 0; t < R; ++t) pt[t] = lane_bcast(cp[h], t);
                            if (lane < R) {
#pragma unroll
                                for (int c = 0; c < RC; ++c) {
                                    const float4 tu = *reinterpret_cast<const float4*>(&TUt[lane * RP + 4 * c]);
                                    s = fmaf(pt[4 * c], tu.x, s);
                                    if (4 * c + 1 < R) s = fmaf(pt[4 * c + 1], tu.y, s);
                                    if (4 * c + 2 < R) s = fmaf(pt[4 * c + 2], tu.z, s);
                                    if (4 * c + 3 < R) s = fmaf(pt[4 * c + 3], tu.w, s);
                                }
                            }
#pragma unroll
                            for (int kk = 0; kk < R; ++kk) av[h][kk] = lane_bcast(s, kk);
                        } else {
                            // one row per lane group: broadcasts within the group
                            const int base = g * L;
                            const int kc = li < R ? li : 0;
#pragma unroll
                            for (int c = 0; c < RC; ++c) {
                                const float4 tu = *reinterpret_cast<const float4*>(&TUt[kc * RP + 4 * c]);
                                s = fmaf(__shfl(cp[h], base + 4 * c, 64), tu.x, s);
                                if (4 * c + 1 < R) s = fmaf(__shfl(cp[h], base + 4 * c + 1, 64), tu.y, s);
                                if (4 * c + 2 < R) s = fmaf(__shfl(cp[h], base + 4 * c + 2, 64), tu.z, s);
                                if (4 * c + 3 < R) s = fmaf(__shfl(cp[h], base + 4 * c + 3, 64), tu.w, s);
                            }
#pragma unroll
                            for (int kk = 0; kk < R; ++kk) av[h][kk] = __shfl(s, base + kk, 64);
                        }
                    }
                }
                float p[kBRW][R];
#pragma unroll
                for (int h = 0; h < kBRW; ++h)
#pragma unroll
                    for (int kk = 0; kk < R; ++kk) p[h][kk] = 0.f;
                float rowacc = 0.f;
#pragma unroll
                for (int v = 0; v < kBNV; ++v) {
                    const int j = li + L * v;
                    const bool jok = j < n;
                    // column j of V_k, read once for the wavefront's rows
                    float vv[RP];
                    if (jok) {
#pragma unroll
                        for (int c = 0; c < RC; ++c) {
                            const float4 t4 = *reinterpret_cast<const float4*>(&Vs[(c * kBNMax + j) * 4]);
                            vv[4 * c] = t4.x; vv[4 * c + 1] = t4.y; vv[4 * c + 2] = t4.z; vv[4 * c + 3] = t4.w;
                        }
                    } else {
#pragma unroll
                        for (int kk = 0; kk < RP; ++kk) vv[kk] = 0.f;
                    }
#pragma unroll
                    for (int h = 0; h < kBRW; ++h) {
                        const int lrow = (h * kBNW + wave) * RPW + g;
                        const int i = b * HB + lrow;
                        const bool ok = (i < m) && jok;
                        const float mv = cm[h * kBNV + v];
                        float x;
                        if (mode == 0) {
                            x = mv;
                            rowacc = fmaf(mv, mv, rowacc);
                        } else {
                            const float yp = cy[h * kBNV + v];
                            float l = 0.f;
#pragma unroll
                            for (int kk = 0; kk < R; ++kk) l = fmaf(av[h][kk], vv[kk], l);
                            const float Rr = mv - l + yp * imup;
                            const float y = fminf(fmaxf(mup * Rr, -lam), lam);
                            const float dy = y - yp;
                            rowacc = ok ? fmaf(dy, dy, rowacc) : rowacc;
                            x = l + dy * imup + y * imuc;
                            if (ok) Yn[(int64_t)i * ldy + j] = y;
                        }
                        x = ok ? x : 0.f;
                        Xs[lrow * nx + j] = x;
#pragma unroll
                        for (int kk = 0; kk < R; ++kk) p[h][kk] = fmaf(x, vv[kk], p[h][kk]);
                    }
                }
                acc2 += (double)rowacc;
#pragma unroll
                for (int h = 0; h < kBRW; ++h) {
                    const int lrow = (h * kBNW + wave) * RPW + g;
                    const int i = b * HB + lrow;
                    const bool row_ok = i < m;
#pragma unroll
                    for (int kk = 0; kk < R; ++kk)
                        for (int off = L >> 1; off > 0; off >>= 1) p[h][kk] += __shfl_xor(p[h][kk], off, 64);
                    if (li < 16) {
                        float mine = 0.f;
#pragma unroll
                        for (int kk = 0; kk < R; ++kk) mine = (kk == li) ? p[h][kk] : mine;
                        Ps[lrow * 16 + li] = row_ok ? mine : 0.f;
                        if (row_ok && li < R) Pn[(int64_t)i * R + li] = mine;
                    }
                }
                __syncthreads();
                // column pass: thread j owns column j; FP64 G_P of the band's rows
                if (tid < n) {
#pragma unroll 4
                    for (int h = 0; h < HB; ++h) {
                        const float xv = Xs[h * nx + tid];
#pragma unroll
                        for (int c = 0; c < RC; ++c) {
                            const float4 pp = *reinterpret_cast<const float4*>(&Ps[h * 16 + 4 * c]);
                            q[4 * c] = fmaf(xv, pp.x, q[4 * c]);
                            if (4 * c + 1 < R) q[4 * c + 1] = fmaf(xv, pp.y, q[4 * c + 1]);
                            if (4 * c + 2 < R) q[4 * c + 2] = fmaf(xv, pp.z, q[4 * c + 2]);
                            if (4 * c + 3 < R) q[4 * c + 3] = fmaf(xv, pp.w, q[4 * c + 3]);
                        }
                    }
                }
                if (tid < E) {
                    for (int h = 0; h < HB; ++h) gp = fma((double)Ps[h * 16 + gx], (double)Ps[h * 16 + gy], gp);
                }
                __syncthreads();
#pragma unroll
                for (int e = 0; e < kBRW * kBNV; ++e) { cm[e] = nm[e]; cy[e] = ny[e]; }
#pragma unroll
                for (int e = 0; e < kBRW; ++e) cp[e] = np[e];
            }
        };
        if constexpr (MF) {
            constexpr int S1 = (R + 3) / 4;
            const int lr = lane & 15, lq = lane >> 4;
            const int ntile = (n + 15) / 16;
            // this lane's V operands for its tiles: l product A[lr][lq] = V[col 16 tg + lr][rank 4 s + lq],
            // p product A[lr][lq] = V[col 16 tg + 4 lq + e][rank lr]
            float va1[4][S1], va2[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int c0 = 16 * (wave + 8 * u);
#pragma unroll
                for (int s2 = 0; s2 < S1; ++s2) {
                    const int kk = 4 * s2 + lq, j = c0 + lr;
                    va1[u][s2] = (kk < R && j < n) ? Vs[vat(kk, j)] : 0.f;
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int j = c0 + 4 * lq + e;
                    va2[u][e] = (lr < R && j < n) ? Vs[vat(lr, j)] : 0.f;
                }
            }
            bf32x4 qacc[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) qacc[u] = bf32x4{0.f, 0.f, 0.f, 0.f};
            float* Xw = XwA + wave * kMB * kMXP;
            const int nb = (m + kMB - 1) / kMB;
            for (int b = 0; b < nb; ++b) {
                const int i = b * kMB + lr;
                const bool row_ok = i < m;
                // a_i = P_i T_U for entries 4 s + lq
                float aop[S1];
                if (mode != 0) {
                    float prow[R];
#pragma unroll
                    for (int t = 0; t < R; ++t) prow[t] = row_ok ? Pp[(int64_t)i * R + t] : 0.f;
#pragma unroll
                    for (int s2 = 0; s2 < S1; ++s2) {
                        const int kk = 4 * s2 + lq;
                        float v = 0.f;
                        if (kk < R) {
#pragma unroll
                            for (int t = 0; t < R; ++t) v = fmaf(prow[t], TUt[kk * RP + t], v);
                        }
                        aop[s2] = v;
                    }
                }
                bf32x4 pacc = {0.f, 0.f, 0.f, 0.f};
                float rowacc = 0.f;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int tg = wave + 8 * u;
                    if (tg < ntile) {     // uniform over the wavefront
                        const int col = 16 * tg + 4 * lq;
                        float mv[4], yp[4] = {0.f, 0.f, 0.f, 0.f}, x[4];
                        bool okv[4];
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            okv[e] = row_ok && (col + e < n);
                            mv[e] = okv[e] ? M[(int64_t)i * ldm + col + e] : 0.f;
                        }
                        if (mode == 0) {
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                x[e] = mv[e];
                                rowacc = fmaf(mv[e], mv[e], rowacc);
                            }
                        } else {
                            bf32x4 lv = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                            for (int s2 = 0; s2 < S1; ++s2) lv = bmfma4(va1[u][s2], aop[s2], lv);
                            if (mode == 2 && row_ok && col < n) {
                                const bf32x4 y4 = *reinterpret_cast<const __attribute__((address_space(1))) bf32x4*>(
                                    Yp + (int64_t)i * ldy + col);
                                yp[0] = y4[0]; yp[1] = y4[1]; yp[2] = y4[2]; yp[3] = y4[3];
                            }
                            float yn[4];
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                const float ype = okv[e] ? yp[e] : 0.f;
                                const float Rr = mv[e] - lv[e] + ype * imup;
                                const float y = fminf(fmaxf(mup * Rr, -lam), lam);
                                const float dy = y - ype;
                                rowacc = okv[e] ? fmaf(dy, dy, rowacc) : rowacc;
                                x[e] = okv[e] ? (lv[e] + dy * imup + y * imuc) : 0.f;
                                yn[e] = y;
                            }
                            // col < n and col % 4 == 0: the vector stays inside the row's ldy >= n (rounded up to 4)
                            if (row_ok && col < n)
                                *reinterpret_cast<__attribute__((address_space(1))) bf32x4*>(Yn + (int64_t)i * ldy + col) =
                                    bf32x4{yn[0], yn[1], yn[2], yn[3]};
                        }
                        *reinterpret_cast<float4*>(Xw + lr * kMXP + 16 * u + 4 * lq) = make_float4(x[0], x[1], x[2], x[3]);
                        if (bfk) {
                            pacc = mfma_bf16(va2[u], x, pacc);
                        } else {
#pragma unroll
                            for (int e = 0; e < 4; ++e) pacc = bmfma4(va2[u][e], x[e], pacc);
                        }
                    }
                }
                acc2 += (double)rowacc;
                // lane (lr, lq) holds p[row lr][rank 4 lq + e] of this wavefront's columns
#pragma unroll
                for (int e = 0; e < 4; ++e) PWA[wave * 256 + lr * 16 + 4 * lq + e] = pacc[e];
                __syncthreads();
                if (tid < 256) {
                    float sum = 0.f;
#pragma unroll
                    for (int w = 0; w < kBNW; ++w) sum += PWA[w * 256 + tid];
                    PSA[tid] = sum;
                    const int hh = tid >> 4, kk = tid & 15;
                    if (kk < R && b * kMB + hh < m) Pn[(int64_t)(b * kMB + hh) * R + kk] = sum;
                }
                __syncthreads();
                // column pass: Q[col 16 tg + 4 lq + e][rank lr] += x^T p over the band's rows
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (wave + 8 * u < ntile) {
                        if (bfk) {
                            float a3[4], b3[4];
#pragma unroll
                            for (int s2 = 0; s2 < 4; ++s2) {
                                a3[s2] = Xw[(4 * s2 + lq) * kMXP + 16 * u + lr];
                                b3[s2] = PSA[(4 * s2 + lq) * 16 + lr];
                            }
                            qacc[u] = mfma_bf16(a3, b3, qacc[u]);
                        } else {
#pragma unroll
                            for (int s2 = 0; s2 < 4; ++s2) {
                                const float a3 = Xw[(4 * s2 + lq) * kMXP + 16 * u + lr];
                                const float b3 = PSA[(4 * s2 + lq) * 16 + lr];
                                qacc[u] = bmfma4(a3, b3, qacc[u]);
                            }
                        }
                    }
                }
                if (tid < E) {
#pragma unroll 4
                    for (int h = 0; h < kMB; ++h) gp = fma((double)PSA[h * 16 + gx], (double)PSA[h * 16 + gy], gp);
                }
                __syncthreads();
            }
            // Q_k from the MFMA layout to the staging rows (Vs[j R + k]), then
            // into each column thread's registers
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int c0 = 16 * (wave + 8 * u) + 4 * lq;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (lr < R && c0 + e < n) Vs[(c0 + e) * R + lr] = qacc[u][e];
            }
            __syncthreads();
            if (tid < n) {
#pragma unroll
                for (int kk = 0; kk < R; ++kk) q[kk] = Vs[tid * R + kk];
            }
            __syncthreads();
        } else {
            sweep_bands(BoolTag<NARROW>{});
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
            else if (res <= d.tol) { stop = true; }
            else if (kdone >= bp.max_iter) { stop = true; status = kWarnMaxIter; }
            if (stop) iters = kdone;
        }
        if (stop) break;

        // ---------------- FP64 step: Grams, Alg. 2 projectors ----------------
        // G_Q = Q^T Q: GS threads per entry, each over every GS-th column
        double* gsum = reinterpret_cast<double*>(Xs);
        if (tid < GS * E) {
            const int sl = tid / E;
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            int j = sl;
            for (; j + 3 * GS < n; j += 4 * GS) {
                a0 = fma((double)Vs[j * R + qx], (double)Vs[j * R + qy], a0);
                a1 = fma((double)Vs[(j + GS) * R + qx], (double)Vs[(j + GS) * R + qy], a1);
                a2 = fma((double)Vs[(j + 2 * GS) * R + qx], (double)Vs[(j + 2 * GS) * R + qy], a2);
                a3 = fma((double)Vs[(j + 3 * GS) * R + qx], (double)Vs[(j + 3 * GS) * R + qy], a3);
            }
            for (; j < n; j += GS) a0 = fma((double)Vs[j * R + qx], (double)Vs[j * R + qy], a0);
            gsum[tid] = (a0 + a1) + (a2 + a3);
        }
        __syncthreads();
        if (tid < E) {
            double gq = 0.0;
            for (int sl = 0; sl < GS; ++sl) gq += gsum[sl * E + tid];
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
        if (!lstep_algebra<R, NT>(Gp, Gq, Bm, C1, C2, Km, T1, T2, Ev, Ev2, cs, wbuf, r, kDkTauF32)) {
            status = kErrRank;
            iters = k - 1;
            break;
        }
        // the step's transforms (padded block dropped) and B_k
        for (int e = tid; e < R * R; e += NT) {
            const int i = e / R, j = e % R;
            const bool in = (i < r) && (j < r);
            TUt[j * RP + i] = in ? (float)Km[i * LDP + j] : 0.f;
            TVt[j * RP + i] = in ? (float)Gp[i * LDP + j] : 0.f;
            TUb[i * LDP + j] = in ? T1[i * LDP + j] : 0.0;
            TVd[i * LDP + j] = in ? Gp[i * LDP + j] : 0.0;
            Bm[i * LDP + j] = in ? T2[i * LDP + j] : (i == j ? 1.0 : 0.0);
        }
        if (RP > R) {
            constexpr int PW = RP > R ? RP - R : 1;
            for (int e = tid; e < R * PW; e += NT) {
                const int j = e / PW, i = R + e % PW;
                TUt[j * RP + i] = 0.f;
                TVt[j * RP + i] = 0.f;
            }
        }
        __syncthreads();
        // V_{k+1} = Q_k T_V from the column's own Q row (registers)
        if (tid < n) {
            float vn[RP];
#pragma unroll
            for (int kk = 0; kk < RP; ++kk) vn[kk] = 0.f;
#pragma unroll
            for (int kk = 0; kk < R; ++kk) {
                float s = 0.f;
#pragma unroll
                for (int c = 0; c < RC; ++c) {
                    const float4 tv = *reinterpret_cast<const float4*>(&TVt[kk * RP + 4 * c]);
                    s = fmaf(q[4 * c], tv.x, s);
                    if (4 * c + 1 < R) s = fmaf(q[4 * c + 1], tv.y, s);
                    if (4 * c + 2 < R) s = fmaf(q[4 * c + 2], tv.z, s);
                    if (4 * c + 3 < R) s = fmaf(q[4 * c + 3], tv.w, s);
                }
                vn[kk] = s;
            }
#pragma unroll
            for (int c = 0; c < RC; ++c)
                *reinterpret_cast<float4*>(&Vs[(c * kBNMax + tid) * 4]) =
                    make_float4(vn[4 * c], vn[4 * c + 1], vn[4 * c + 2], vn[4 * c + 3]);
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
        const gfloat* PK = (K & 1) ? P1 : P0;
        const gfloat* QK = (K & 1) ? Q1 : Q0;
        const gfloat* YK = (K & 1) ? Y1 : Y0;     // Y_K (K >= 2); Y_1 = 0
        const bool haveY = K >= 2;
        gfloat* const U = as_global(d.U);
        gfloat* const V = as_global(d.V);
        gdouble* const Bo = as_global(d.B);
        gfloat* const S = as_global(d.S);
        // U = P TUbar, V = Q TV (FP64 accumulation), B; one row per thread
        for (int i = tid; i < m; i += NT) {
            float pr[R];
#pragma unroll
            for (int t = 0; t < R; ++t) pr[t] = PK[(int64_t)i * R + t];
#pragma unroll 1
            for (int kk = 0; kk < r; ++kk) {
                double s = 0.0;
#pragma unroll
                for (int t = 0; t < R; ++t)
                    if (t < r) s = fma((double)pr[t], TUb[t * LDP + kk], s);
                U[(int64_t)i * r + kk] = (float)s;
            }
        }
        // V_K for the S pass (FP32, grouped layout in Vs) and the returned V
        for (int j = tid; j < n; j += NT) {
            float qr[R];
#pragma unroll
            for (int t = 0; t < R; ++t) qr[t] = QK[(int64_t)j * R + t];
#pragma unroll 1
            for (int kk = 0; kk < RP; ++kk) {
                double s = 0.0;
                if (kk < r) {
#pragma unroll
                    for (int t = 0; t < R; ++t)
                        if (t < r) s = fma((double)qr[t], TVd[t * LDP + kk], s);
                    V[(int64_t)j * r + kk] = (float)s;
                }
                Vs[vat(kk, j)] = (float)s;
            }
        }
        for (int e = tid; e < r * r; e += NT) Bo[e] = Bm[(e / r) * LDP + e % r];
        __syncthreads();
        if (d.S) {
            const float t = (float)(d.lambda / mu_prev), imu = (float)(1.0 / mu_prev);
            // one row per wavefront; the next row's loads are issued first
            auto load_row = [&](int i, float* mv, float* yv, float& pr) {
#pragma unroll
                for (int v = 0; v < kBNV; ++v) {
                    const int j = lane + 64 * v;
                    const bool ok = j < n;
                    mv[v] = ok ? M[(int64_t)i * ldm + j] : 0.f;
                    yv[v] = (ok && haveY) ? YK[(int64_t)i * ldy + j] : 0.f;
                }
                pr = (lane < R) ? PK[(int64_t)i * R + lane] : 0.f;
            };
            float cm[kBNV], cy[kBNV], cp = 0.f;
            if (wave < m) load_row(wave, cm, cy, cp);
            for (int i = wave; i < m; i += kBNW) {
                float nm[kBNV], ny[kBNV], np = 0.f;
#pragma unroll
                for (int v = 0; v < kBNV; ++v) { nm[v] = 0.f; ny[v] = 0.f; }
                if (i + kBNW < m) load_row(i + kBNW, nm, ny, np);
                float pt[R];
#pragma unroll
                for (int tt = 0; tt < R; ++tt) pt[tt] = lane_bcast(cp, tt);
                float s = 0.f;
                if (lane < R) {
#pragma unroll
                    for (int c = 0; c < RC; ++c) {
                        const float4 tu = *reinterpret_cast<const float4*>(&TUt[lane * RP + 4 * c]);
                        s = fmaf(pt[4 * c], tu.x, s);
                        if (4 * c + 1 < R) s = fmaf(pt[4 * c + 1], tu.y, s);
                        if (4 * c + 2 < R) s = fmaf(pt[4 * c + 2], tu.z, s);
                        if (4 * c + 3 < R) s = fmaf(pt[4 * c + 3], tu.w, s);
                    }
                }
                float av[R];
#pragma unroll
                for (int kk = 0; kk < R; ++kk) av[kk] = lane_bcast(s, kk);
#pragma unroll
                for (int v = 0; v < kBNV; ++v) {
                    const int j = lane + 64 * v;
                    if (j < n) {
                        float vv[RP];
#pragma unroll
                        for (int c = 0; c < RC; ++c) {
                            const float4 t4 = *reinterpret_cast<const float4*>(&Vs[(c * kBNMax + j) * 4]);
                            vv[4 * c] = t4.x; vv[4 * c + 1] = t4.y; vv[4 * c + 2] = t4.z; vv[4 * c + 3] = t4.w;
                        }
                        float l = 0.f;
#pragma unroll
                        for (int kk = 0; kk < R; ++kk) l = fmaf(av[kk], vv[kk], l);
                        const float Rr = cm[v] - l + cy[v] * imu;
                        const float a1 = Rr - t, b1 = Rr + t;
                        S[(int64_t)i * d.lds + j] = (a1 > 0.f ? a1 : 0.f) + (b1 < 0.f ? b1 : 0.f);
                    }
                }
#pragma unroll
                for (int v = 0; v < kBNV; ++v) { cm[v] = nm[v]; cy[v] = ny[v]; }
                cp = np;
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

// One problem per workgroup (sfr_solve_batch).
template <int R, int RW, bool NARROW, bool MF>
__global__ void __launch_bounds__(kBTPB, 1) batch_kernel(BatchItemDev* items, BatchParams bp)
{
    batch_solve<R, RW, NARROW, MF>(items + blockIdx.x, bp);
}

// orth_err of one item: ||U^T U - I_r||_F and ||V^T V - I_r||_F of the
// factors it wrote (FP64 sums over 64-row tiles staged in LDS, each Gram
// entry owned by one thread and summed in row order).
constexpr int kOrthRows = 64;

__device__ void batch_orth_item(BatchItemDev* it)
{
    if (it->status < 0) return;
    __shared__ float tile[kOrthRows * 16];
    __shared__ double red[256];
    const int r = it->r, E = r * (r + 1) / 2, tid = threadIdx.x;
    const int NT = blockDim.x;   // 256 or 512; entries and reductions use the first 256 threads
    int p = 0, q = 0;
    if (tid < E) {
        int e = tid;
        while (e >= r - p) { e -= r - p; ++p; }
        q = p + e;
    }
    double dist[2];
    for (int f = 0; f < 2; ++f) {
        const float* X = f == 0 ? it->U : it->V;
        const int rows = f == 0 ? it->m : it->n;
        double g = 0.0;
        for (int i0 = 0; i0 < rows; i0 += kOrthRows) {
            const int nr = min(kOrthRows, rows - i0);
            __syncthreads();
            for (int e = tid; e < nr * r; e += NT) tile[e] = X[(int64_t)i0 * r + e];
            __syncthreads();
            if (tid < E)
                for (int i = 0; i < nr; ++i) g = fma((double)tile[i * r + p], (double)tile[i * r + q], g);
        }
        const double d = g - (p == q ? 1.0 : 0.0);
        if (tid < 256) red[tid] = (tid < E) ? ((p == q) ? 1.0 : 2.0) * d * d : 0.0;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (tid < h) red[tid] += red[tid + h];
            __syncthreads();
        }
        dist[f] = sqrt(red[0]);
        __syncthreads();
    }
    if (tid == 0) it->orth_err = fmax(dist[0], dist[1]);
}

__global__ void __launch_bounds__(256) batch_orth_kernel(BatchItemDev* items)
{
    batch_orth_item(items + blockIdx.x);
}

// Persistent form: the workgroups of one launch take problems one by one
// from a queue that the host appends to while the kernel runs, and retire
// each as soon as it is solved.  The host side (pinned, coherent memory):
// the descriptors, the queue entries (entry -> slot) and `tail`; `closed`
// asks the workgroups to leave once the queue is drained.  The device side:
// `head`, the next entry to claim (compare-and-swap).  A workgroup that finds
// no work for kQueueIdle polls leaves as well (the host relaunches when work
// is pending and the kernel has ended), so every workgroup exits.
constexpr uint32_t kQueueIdle = 1u << 18;

template <int R, int RW, bool NARROW, bool MF>
__global__ void __launch_bounds__(kBTPB, 1) batch_queue_kernel(BatchItemDev* items, BatchParams bp,
                                                               BatchQueueDev* q, BatchQueueHost* hq, int32_t* done,
                                                               int cap)
{
    __shared__ int s_slot;
    __shared__ BatchItemDev sdesc;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) {
            int slot = -1;
            uint32_t polls = 0;
            for (;;) {
                const int tail = __hip_atomic_load(&hq->tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
                int h = __hip_atomic_load(&q->head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (h < tail) {
                    if (__hip_atomic_compare_exchange_strong(&q->head, &h, h + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT)) {
                        slot = __hip_atomic_load(&hq->order[h % cap], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                        break;
                    }
                    continue;
                }
                if (__hip_atomic_load(&hq->closed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) break;
                if (++polls >= kQueueIdle) break;
                __builtin_amdgcn_s_sleep(127);
            }
            s_slot = slot;
        }
        __syncthreads();
        const int slot = s_slot;
        __syncthreads();
        if (slot < 0 || slot >= cap) break;
        // The host rewrites a slot's descriptor between uses: it is read here
        // word by word with system-scope loads into an LDS copy, solved from
        // that copy, and the results are written back to the slot.
        BatchItemDev* it = items + slot;
        constexpr int DW = sizeof(BatchItemDev) / 4;
        static_assert(DW <= kBTPB, "descriptor words per thread");
        if (tid < DW)
            reinterpret_cast<int32_t*>(&sdesc)[tid] =
                __hip_atomic_load(reinterpret_cast<int32_t*>(it) + tid, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __syncthreads();
        batch_solve<R, RW, NARROW, MF>(&sdesc, bp);
        __syncthreads();
        __threadfence();   // this workgroup's U and V stores are visible to its reads below
        batch_orth_item(&sdesc);
        __syncthreads();
        if (tid == 0) {
            it->iters = sdesc.iters;
            it->status = sdesc.status;
            it->res = sdesc.res;
            it->min_eig_B = sdesc.min_eig_B;
            it->mu_final = sdesc.mu_final;
            it->orth_err = sdesc.orth_err;
            __threadfence_system();
            __hip_atomic_store(&done[slot], sdesc.seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
        __syncthreads();
    }
}

hipError_t launch_batch_queue(BatchItemDev* items, const BatchParams& bp, BatchQueueDev* q, BatchQueueHost* hq,
                              int32_t* done, int cap, int small, int grid, hipStream_t s)
{
    if (small)
        hipLaunchKernelGGL((batch_queue_kernel<6, 2, false, false>), dim3(grid), dim3(kBTPB), 0, s, items, bp, q, hq,
                           done, cap);
    else
        hipLaunchKernelGGL((batch_queue_kernel<16, 1, false, true>), dim3(grid), dim3(kBTPB), 0, s, items, bp, q, hq,
                           done, cap);
    return hipGetLastError();
}

hipError_t launch_batch_orth(BatchItemDev* items, int count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(batch_orth_kernel, dim3((unsigned)count), dim3(256), 0, s, items);
    return hipGetLastError();
}

#define SFR_BATCH_R_LIST(X) X(1) X(2) X(3) X(4) X(5) X(6) X(8) X(10) X(12) X(16)

#ifndef SFR_BATCH_RW
#define SFR_BATCH_RW(R) ((R) <= 12 ? 2 : 1)
#endif

static bool batch_mfma_enabled()
{
    const char* v = getenv("SFR_BATCH_MFMA");
    return !(v && v[0] == '0');
}

int batch_default_variant(int R, bool narrow)
{
    if (narrow) return kBVNarrow;
    if (R >= 8 && batch_mfma_enabled()) return kBVMfma;
    return SFR_BATCH_RW(R) == 2 ? kBVRow2 : kBVRow1;
}

bool batch_variant_valid(int R, int variant)
{
    return variant == kBVNarrow || variant == kBVRow1 || variant == kBVRow2 || (variant == kBVMfma && R >= 8);
}

hipError_t launch_batch(BatchItemDev* items, int count, int R, bool narrow, int variant, const BatchParams& bp,
                        hipStream_t s)
{
    if (variant == kBVAuto) variant = batch_default_variant(R, narrow);
    if (!batch_variant_valid(R, variant)) return hipErrorInvalidValue;
    switch (R) {
#define CASE(rr)                                                                                               \
    case rr:                                                                                                   \
        switch (variant) {                                                                                     \
        case kBVNarrow:                                                                                        \
            hipLaunchKernelGGL((batch_kernel<rr, 1, true, false>), dim3(count), dim3(kBTPB), 0, s, items, bp); \
            break;                                                                                             \
        case kBVMfma:                                                                                          \
            hipLaunchKernelGGL((batch_kernel<rr, 1, false, (rr >= 8)>), dim3(count), dim3(kBTPB), 0, s, items,   \
                               bp);                                                                            \
            break;                                                                                             \
        case kBVRow2:                                                                                          \
            hipLaunchKernelGGL((batch_kernel<rr, 2, false, false>), dim3(count), dim3(kBTPB), 0, s, items, bp); \
            break;                                                                                             \
        default:                                                                                               \
            hipLaunchKernelGGL((batch_kernel<rr, 1, false, false>), dim3(count), dim3(kBTPB), 0, s, items, bp); \
            break;                                                                                             \
        }                                                                                                      \
        return hipGetLastError();
        SFR_BATCH_R_LIST(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sfr
