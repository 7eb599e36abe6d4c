// The fused FR-ADM sweep on the matrix cores (FP32, R <= 32, wide rows).
//
// Same iteration as sweep.hip (Alg. 1 with the Alg. 2 L-step; one pass
// over M and Y per iteration), with its three contractions on
// v_mfma_f32_16x16x4_f32 (exact FP32 products, FP32 accumulation):
//   l  (16 rows x 16 columns)  = A_band (16 x R) . V_tile^T        K = R
//   p  (16 rows x R)          += X_tile (16 x 16) . V_tile (16 x R) K = 16 columns
//   Q  (16 columns x R)       += X_tile^T (16 x 16) . P_band        K = 16 rows
// Lane layout of the instruction (lane l, lr = l % 16, lq = l / 16): it
// supplies A[lr][lq] and B[lq][lr] and receives D[4 lq + e][lr], e = 0..3.
// With l computed as D[column][row], lane l holds row lr, columns
// 4 lq .. 4 lq + 3 of a 16 x 16 tile: exactly one 16-byte vector of M and
// Y.  The p product takes that lane's own x values as its B operand; the Q
// product needs x transposed, which goes through a wave-private LDS tile.
//
// Work decomposition
//   * A band is 16 rows.  A workgroup is 8 wavefronts; wave w owns 16 TPW
//     consecutive columns of its member's slice (TPW = 8 tiles of 16 columns
//     for R <= 12, 4 above; the R = 16 bucket also has a wide form with 8,
//     taken where n holds its 1024-column slices), for every band.  Ranks are padded to 16-wide
//     tiles (one, or two for R > 16).  The V values a lane needs for its
//     tiles are loaded into registers once.
//   * Row pass: per tile, l (ceil(R/4) MFMA), the S/dual step, Y_k, x, the
//     wave's p partial (4 MFMA); each 16-byte load of the next band goes
//     out as soon as its tile has been consumed.
//   * The 8 waves' p partials are added in LDS; with c > 1 members of a
//     cluster exchange them through tagged words (exchange.hpp).  Two forms:
//     all-gather (every member reads every member's partials of a band, one
//     band behind the row pass), and, for wide clusters of the 4-tile form,
//     reduce-then-broadcast: the band's (row, rank) entries are dealt out
//     to the members round-robin, each member adds the c partials of the
//     entries it owns (one band behind) and publishes the sums, and every
//     member reads the sums back (two bands behind).  A member then reads
//     about 16 R + c words a band instead of 16 R c; both forms add the
//     partials in member order, so they give bitwise the same P.
//   * Column pass: Q += X^T P from the wave's own x tile (4 MFMA per tile);
//     Q stays in registers until the end.
// HBM traffic per element: read M, read Y_{k-1}, write Y_k.
#include "exchange.hpp"
#include "mfma_bf16.hpp"
#include "sfr_internal.hpp"

#include <hip/hip_ext.h>

// Non-temporal hints on this sweep's streams measured slower (8000^2: r = 20
// 382 against 378 us, X = M sweeps 113 against 107 us, alternating on one
// device), unlike the vector sweep's: off by default.
#ifndef SFR_NT_MFMA
#define SFR_NT_MFMA 0
#endif

namespace sfr {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMW8 = 8;                  // wavefronts per workgroup
constexpr int kMTPB = 64 * kMW8;         // threads per workgroup
constexpr int kMH = 16;                  // rows per band
constexpr int kGatherBatch = 8;          // exchange words read together per thread

// Compile-time shape for rank bucket R.
template <int R, int TW = 0>
struct MShape {
    static constexpr int RT = (R + 15) / 16;          // 16-wide rank tiles (p, Q)
    static constexpr int S1 = (R + 3) / 4;            // K steps of the l product
    static constexpr int TPW = TW ? TW : ((R <= 12) ? 8 : 4);   // 16-column tiles per wavefront
    static constexpr int COLS = 16 * TPW;             // columns per wavefront
    static constexpr int WIDTH = kMW8 * COLS;         // columns per member slice
    static constexpr int XP = COLS + 16;              // LDS pitch of a row of a wave's x tile (floats)
};

struct MfmaLds {
    size_t tu, xw, pw, ps, rb, red, total;
};

// Largest cluster of the reduce-then-broadcast form (members resident at
// once: at most two workgroups per CU of 256 CUs).
constexpr int kRbMaxC = 512;

// RB: reduce-then-broadcast exchange (column pass two bands behind the row
// pass, three band buffers of x and P); else all-gather (one band behind).
template <int R, int TW = 0, bool RB = false>
__host__ __device__ inline MfmaLds mfma_lds()
{
    using S = MShape<R, TW>;
    constexpr int NBUF = RB ? 3 : 2;
    auto al = [](size_t x) { return (x + 15) & ~size_t(15); };
    MfmaLds L;
    size_t o = 0;
    L.tu = o; o = al(o + sizeof(float) * R * R);
    // x tiles: per wave, NBUF band buffers of 16 rows; the V slice
    // (WIDTH x R floats) is staged here during the prologue
    size_t xw = sizeof(float) * (size_t)kMW8 * NBUF * kMH * S::XP;
    const size_t vst = sizeof(float) * (size_t)S::WIDTH * R;
    L.xw = o; o = al(o + (xw > vst ? xw : vst));
    L.pw = o; o = al(o + sizeof(float) * kMW8 * 256 * S::RT);
    L.ps = o; o = al(o + sizeof(float) * NBUF * 256 * S::RT);
    // partials of the owned entries of a band (at most 16 R + c - 1)
    L.rb = o; o = al(o + (RB ? sizeof(float) * (size_t)(kMH * R + kRbMaxC) : 0));
    L.red = o; o = al(o + sizeof(double) * kMW8);
    L.total = o;
    return L;
}

__device__ __forceinline__ f32x4 mfma4(float a, float b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}


// BF: the p and Q contractions take BF16 operands (FP32 accumulation); the
// l reconstruction, M, Y and every stored value stay FP32.  RB: the
// reduce-then-broadcast exchange (the host takes it only with c > 1).
template <int R, bool BF, int TW = 0, bool RB = false>
__global__ void __launch_bounds__(kMTPB, 1) sweep_mfma_kernel(SweepArgs<float> a)
{
    using SH = MShape<R, TW>;
    constexpr int LAG = RB ? 2 : 1, NBUF = LAG + 1;
    constexpr int RT = SH::RT, S1 = SH::S1, kMTiles = SH::TPW, kMCols = SH::COLS;
    constexpr int kMWidth = SH::WIDTH, kMXP = SH::XP;
    constexpr int PT = 256 * RT;      // (row, padded rank) entries of one band
    DevState* st = const_cast<DevState*>(a.st);
    if (st->done) return;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lq = lane >> 4;
    const int c = a.c;
    const int g = blockIdx.x;
    int q, cl;
    if (a.xcd_local) {
        const int xcd = g % kXCD, loc = g / kXCD;
        q = loc % c;
        cl = xcd * a.cpx + loc / c;
    } else {
        q = g % c;
        cl = g / c;
    }
    const int c0 = q * kMWidth;                 // first column of this member
    const int cw = c0 + wave * kMCols;          // first column of this wave
    const int m = a.m, n = a.n;
    const int64_t ldm = st->ldm, ldy = a.ldy;
    const float* __restrict__ M = static_cast<const float*>(st->M);
    const int mode = a.mode;
    const float lam = (float)st->lambda;
    const float mu_prev = (float)st->mu_prev;
    const float imu_prev = (mode != 0) ? (float)(1.0 / st->mu_prev) : 0.f;
    const float imu_cur = (float)(1.0 / st->mu);
    const uint32_t kiter = (uint32_t)st->k;
    int32_t* tflag = &st->exch_timeout;

    extern __shared__ __align__(16) unsigned char smem[];
    const MfmaLds L = mfma_lds<R, TW, RB>();
    float* TUs = reinterpret_cast<float*>(smem + L.tu);
    float* Xall = reinterpret_cast<float*>(smem + L.xw);
    float* Xw = Xall + (size_t)wave * NBUF * kMH * kMXP;
    float* PW = reinterpret_cast<float*>(smem + L.pw);
    float* PS = reinterpret_cast<float*>(smem + L.ps);
    double* red = reinterpret_cast<double*>(smem + L.red);
    float* RED1 = reinterpret_cast<float*>(smem + L.rb);

    // ---- prologue: TU, and V_j = Q_j TV for this member's columns
    float* Vst = Xall;   // kMWidth x R, row j - c0
    {
        const float* tu = st->TUf;
        const float* tv = st->TVf;
        for (int e = tid; e < R * R; e += kMTPB) TUs[e] = tu[(e / R) * kMaxR + e % R];
        for (int jj = tid; jj < kMWidth; jj += kMTPB) {
            const int j = c0 + jj;
            float qrow[R];
#pragma unroll
            for (int t = 0; t < R; ++t) qrow[t] = (j < n) ? a.Qprev[(int64_t)j * R + t] : 0.f;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                float s = 0.f;
#pragma unroll
                for (int t = 0; t < R; ++t) s = fmaf(qrow[t], tv[t * kMaxR + k], s);
                Vst[(size_t)jj * R + k] = s;
            }
        }
    }
    __syncthreads();
    // this lane's V operands: l product A[lr][lq] = V[col 16t + lr][rank 4s + lq],
    // p product A[lr][lq] = V[col 16t + 4 lq + u][rank 16 rt + lr]
    float va1[kMTiles][S1], va2[kMTiles][RT][4];
#pragma unroll
    for (int t = 0; t < kMTiles; ++t) {
        const int jl = wave * kMCols + 16 * t;
#pragma unroll
        for (int s = 0; s < S1; ++s) {
            const int k = 4 * s + lq;
            va1[t][s] = (k < R) ? Vst[(size_t)(jl + lr) * R + k] : 0.f;
        }
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
            const int k = 16 * rt + lr;
#pragma unroll
            for (int u = 0; u < 4; ++u) va2[t][rt][u] = (k < R) ? Vst[(size_t)(jl + 4 * lq + u) * R + k] : 0.f;
        }
    }
    __syncthreads();   // the staging area becomes the x tiles

    const int nbands = a.nbands, ncl = a.ncl;
    const int nbl = (cl < nbands) ? (nbands - 1 - cl) / ncl + 1 : 0;
    double acc2 = 0.0;
    f32x4 qacc[kMTiles][RT];
#pragma unroll
    for (int t = 0; t < kMTiles; ++t)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) qacc[t][rt] = f32x4{0.f, 0.f, 0.f, 0.f};

    // the row-pass operands of one band: tile t of row lr, columns
    // cw + 16 t + 4 lq .. + 3 (out-of-range vectors read a valid dummy
    // address and are zeroed at use)
    float4 mv[kMTiles], yv[kMTiles];
    auto issue_load = [&](int jb, int t) {
        const int i = (cl + jb * ncl) * kMH + lr;
        const int col = cw + 16 * t + 4 * lq;
        const bool ok = (i < m) && (col < n);
#if SFR_NT_MFMA
        float v4[4];
        load_vec_stream<float>(M + (ok ? (int64_t)i * ldm + col : 0), v4);
        mv[t] = make_float4(v4[0], v4[1], v4[2], v4[3]);
        if (mode == 2) {
            load_vec_stream<float>(a.Yprev + (ok ? (int64_t)i * ldy + col : 0), v4);
            yv[t] = make_float4(v4[0], v4[1], v4[2], v4[3]);
        }
#else
        mv[t] = *reinterpret_cast<const float4*>(M + (ok ? (int64_t)i * ldm + col : 0));
        if (mode == 2) yv[t] = *reinterpret_cast<const float4*>(a.Yprev + (ok ? (int64_t)i * ldy + col : 0));
#endif
    };
    if (nbl > 0) {
#pragma unroll
        for (int t = 0; t < kMTiles; ++t) issue_load(0, t);
    }

    for (int j = 0; j < nbl + LAG; ++j) {
        const int buf = j % NBUF;
        if (j < nbl) {
            // ---------------- row pass over band j ----------------
            const int i = (cl + j * ncl) * kMH + lr;
            const bool row_ok = i < m;
            float aop[S1];
            if (mode != 0) {
                float prow[R];
#pragma unroll
                for (int t = 0; t < R; ++t) prow[t] = row_ok ? a.Pprev[(int64_t)i * R + t] : 0.f;
#pragma unroll
                for (int s = 0; s < S1; ++s) {
                    const int k = 4 * s + lq;
                    float v = 0.f;
                    if (k < R) {
#pragma unroll
                        for (int t = 0; t < R; ++t) v = fmaf(prow[t], TUs[t * R + k], v);
                    }
                    aop[s] = v;
                }
            }
            f32x4 pacc[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) pacc[rt] = f32x4{0.f, 0.f, 0.f, 0.f};
            float rowacc = 0.f;
#pragma unroll
            for (int t = 0; t < kMTiles; ++t) {
                const int col = cw + 16 * t + 4 * lq;
                const bool ok = row_ok && (col < n);
                float x[4];
                const float mvv[4] = {mv[t].x, mv[t].y, mv[t].z, mv[t].w};
                if (mode == 0) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        x[e] = ok ? mvv[e] : 0.f;
                        rowacc = fmaf(x[e], x[e], rowacc);
                    }
                } else {
                    // l stays on FP32 operands in both forms: its rounding
                    // would enter Y_k, S_k and x elementwise, unaveraged
                    f32x4 lv = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int s = 0; s < S1; ++s) lv = mfma4(va1[t][s], aop[s], lv);
                    float ypv[4] = {0.f, 0.f, 0.f, 0.f};
                    if (mode == 2) {
                        ypv[0] = yv[t].x; ypv[1] = yv[t].y; ypv[2] = yv[t].z; ypv[3] = yv[t].w;
                    }
                    float yn[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const float yp = ok ? ypv[e] : 0.f;
                        const float mm = ok ? mvv[e] : 0.f;
                        const float l = lv[e];
                        const float Rr = mm - l + yp * imu_prev;
                        const float y = fminf(fmaxf(mu_prev * Rr, -lam), lam);
                        const float dy = y - yp;
                        rowacc = fmaf(dy, dy, rowacc);
                        x[e] = ok ? (l + dy * imu_prev + y * imu_cur) : 0.f;
                        yn[e] = y;
                    }
#if SFR_NT_MFMA
                    if (ok) store_vec_stream<float>(a.Ynext + (int64_t)i * ldy + col, yn);
#else
                    if (ok) *reinterpret_cast<float4*>(a.Ynext + (int64_t)i * ldy + col) = make_float4(yn[0], yn[1], yn[2], yn[3]);
#endif
                }
                *reinterpret_cast<float4*>(Xw + ((size_t)buf * kMH + lr) * kMXP + 16 * t + 4 * lq) =
                    make_float4(x[0], x[1], x[2], x[3]);
                if constexpr (BF) {
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt) pacc[rt] = mfma_bf16(va2[t][rt], x, pacc[rt]);
                } else {
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                        for (int u = 0; u < 4; ++u) pacc[rt] = mfma4(va2[t][rt][u], x[u], pacc[rt]);
                }
                if (j + 1 < nbl) issue_load(j + 1, t);
            }
            acc2 += (double)rowacc;
            // lane l holds p[row lr][rank 16 rt + 4 lq + e] of this wave's columns
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int e = 0; e < 4; ++e) PW[wave * PT + rt * 256 + lr * 16 + 4 * lq + e] = pacc[rt][e];
        }
        __syncthreads();
        // (row, rank) owned by threads 0..PT-1: tid = 256 rt + 16 row + rank % 16
        const int prow_ = (tid & 255) >> 4, prk = 16 * (tid >> 8) + (tid & 15);
        if (j < nbl && tid < PT) {
            float s = 0.f;
#pragma unroll
            for (int w = 0; w < kMW8; ++w) s += PW[w * PT + tid];
            if (c == 1) {
                PS[buf * PT + tid] = s;
            } else if (prk < R) {
                const uint32_t tag = kiter * (uint32_t)a.nbl_max + (uint32_t)j + 1u;
                const int slot = j & (kExchSlots - 1);
                publish<float>(a.exch + ((((size_t)cl * kExchSlots + slot) * c + q) * kMH + prow_) * R + prk, s, tag);
            }
        }
        if constexpr (RB) {
            // (1) the entries of band j - 1 this member owns: entry
            // e = row * R + rank goes to member e mod c; thread t loads the
            // partial of member t mod c for its owned entry t / c
            const int EN = kMH * R;
            const int nown = (q < EN) ? (EN - q + c - 1) / c : 0;
            const bool red_now = (c > 1) && (j >= 1) && (j - 1 < nbl);
            const int jb1 = j - 1;
            const uint32_t tag1 = kiter * (uint32_t)a.nbl_max + (uint32_t)jb1 + 1u;
            const int slot1 = jb1 & (kExchSlots - 1);
            if (red_now) {
                const unsigned long long* pbase = a.exch + ((size_t)cl * kExchSlots + slot1) * c * EN;
                for (int t = tid; t < nown * c; t += kMTPB) {
                    const int u = t / c, q0 = t - u * c;
                    const unsigned long long* src = pbase + (size_t)q0 * EN + (q + u * c);
                    unsigned long long w = peek_word(src);
                    if ((uint32_t)(w >> 32) != tag1) w = spin_word(src, tag1, tflag);
                    RED1[t] = __uint_as_float((uint32_t)(w & 0xffffffffull));
                }
            }
            __syncthreads();
            unsigned long long* rbase = a.exch + (size_t)a.ncl * kExchSlots * c * EN;
            if (red_now && tid < nown) {
                float sr = 0.f;
                for (int q0 = 0; q0 < c; ++q0) sr += RED1[tid * c + q0];   // member order
                publish<float>(rbase + ((size_t)cl * kExchSlots + slot1) * EN + (q + tid * c), sr, tag1);
            }
            // (2) the sums of band j - 2, from their owners
            if (c > 1 && j >= 2 && tid < PT) {
                const int jb2 = j - 2;
                const uint32_t tag2 = kiter * (uint32_t)a.nbl_max + (uint32_t)jb2 + 1u;
                const int slot2 = jb2 & (kExchSlots - 1);
                float sv = 0.f;
                if (prk < R) {
                    const unsigned long long* src = rbase + ((size_t)cl * kExchSlots + slot2) * EN + prow_ * R + prk;
                    unsigned long long w = peek_word(src);
                    if ((uint32_t)(w >> 32) != tag2) w = spin_word(src, tag2, tflag);
                    sv = __uint_as_float((uint32_t)(w & 0xffffffffull));
                }
                PS[(jb2 % NBUF) * PT + tid] = sv;
            }
        } else if (j >= 1 && c > 1 && tid < PT) {
            // gather the members' partials of band j - 1, added in member order
            const int jb = j - 1;
            const uint32_t tag = kiter * (uint32_t)a.nbl_max + (uint32_t)jb + 1u;
            const int slot = jb & (kExchSlots - 1);
            float s = 0.f;
            if (prk < R) {
                // the words of kGatherBatch members are read together (member
                // indices clamped into range), then those whose tag has not
                // arrived yet are polled: one round trip per batch instead of
                // one per member
                const unsigned long long* base =
                    a.exch + (((size_t)cl * kExchSlots + slot) * c) * kMH * R + (size_t)prow_ * R + prk;
                const size_t qstride = (size_t)kMH * R;
                for (int q0 = 0; q0 < c; q0 += kGatherBatch) {
                    unsigned long long w[kGatherBatch];
#pragma unroll
                    for (int u = 0; u < kGatherBatch; ++u) w[u] = peek_word(base + (size_t)min(q0 + u, c - 1) * qstride);
#pragma unroll
                    for (int u = 0; u < kGatherBatch; ++u) {
                        if (q0 + u < c) {
                            if ((uint32_t)(w[u] >> 32) != tag) w[u] = spin_word(base + (size_t)(q0 + u) * qstride, tag, tflag);
                            s += __uint_as_float((uint32_t)(w[u] & 0xffffffffull));
                        }
                    }
                }
            }
            PS[(jb % NBUF) * PT + tid] = s;
        }
        __syncthreads();
        if (j >= LAG) {
            // ---------------- column pass over band j - LAG ----------------
            const int jb = j - LAG;
            const int bb = jb % NBUF;
            const int i0 = (cl + jb * ncl) * kMH;
            if (q == 0) {
                for (int e = tid; e < kMH * R; e += kMTPB) {
                    const int hh = e / R, k = e % R;
                    if (i0 + hh < m)
                        a.Pnext[(int64_t)(i0 + hh) * R + k] = PS[bb * PT + (k >> 4) * 256 + hh * 16 + (k & 15)];
                }
            }
            // B operand: p[row 4 s + lq][rank 16 rt + lr]; A operand: x[row 4 s + lq][column 16 t + lr]
            float b3[RT][4];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int s = 0; s < 4; ++s) b3[rt][s] = PS[bb * PT + rt * 256 + (4 * s + lq) * 16 + lr];
#pragma unroll
            for (int t = 0; t < kMTiles; ++t) {
                if constexpr (BF) {
                    float a3[4];
#pragma unroll
                    for (int s = 0; s < 4; ++s) a3[s] = Xw[((size_t)bb * kMH + 4 * s + lq) * kMXP + 16 * t + lr];
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt) qacc[t][rt] = mfma_bf16(a3, b3[rt], qacc[t][rt]);
                } else {
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const float a3 = Xw[((size_t)bb * kMH + 4 * s + lq) * kMXP + 16 * t + lr];
#pragma unroll
                        for (int rt = 0; rt < RT; ++rt) qacc[t][rt] = mfma4(a3, b3[rt][s], qacc[t][rt]);
                    }
                }
            }
        }
    }

    // ---------------- write the column partials of this cluster -----------
    // lane l holds Q[column 16 t + 4 lq + e][rank 16 rt + lr]
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int k = 16 * rt + lr;
        if (k < R) {
#pragma unroll
            for (int t = 0; t < kMTiles; ++t) {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int col = cw + 16 * t + 4 * lq + e;
                    if (col < n) a.Qpart[((size_t)cl * n + col) * R + k] = qacc[t][rt][e];
                }
            }
        }
    }
    // ---------------- ||Y_k - Y_{k-1}||^2 (or ||M||^2) partial ------------
    for (int off = 32; off > 0; off >>= 1) acc2 += __shfl_xor(acc2, off, 64);
    if (lane == 0) red[wave] = acc2;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kMW8; ++w) t += red[w];
        a.dy2part[g] = t;
    }
}

#define SFR_MFMA_R_LIST(X) X(1) X(2) X(3) X(4) X(5) X(6) X(8) X(10) X(12) X(16) X(20) X(24) X(32)

bool sweep_mfma_supported(int R)
{
    switch (R) {
#define CASE(r) case r: return true;
        SFR_MFMA_R_LIST(CASE)
#undef CASE
    default: return false;
    }
}

// tiles = 8 selects the wide form of the R = 16 bucket; 0 the default form.
static bool wide16(int R, int tiles) { return R == 16 && tiles == 8; }
// 16-column tiles per wavefront of the default form of bucket R.
static int MShape_tpw(int R) { return R <= 12 ? 8 : 4; }

// The reduce-then-broadcast exchange exists for the 4-tile forms (R > 12;
// the 8-tile forms have no room for a third band buffer in LDS).
#define SFR_MFMA_RB_LIST(X) X(16) X(20) X(24) X(32)

bool sweep_mfma_rb_supported(int R, int tiles)
{
    return !wide16(R, tiles) && MShape_tpw(R) == 4 && sweep_mfma_supported(R);
}

size_t sweep_mfma_lds_bytes(int R, int tiles, bool rb)
{
    if (wide16(R, tiles)) return mfma_lds<16, 8>().total;
    if (rb) {
        switch (R) {
#define CASE(r) case r: return mfma_lds<r, 0, true>().total;
            SFR_MFMA_RB_LIST(CASE)
#undef CASE
        default: return 0;
        }
    }
    switch (R) {
#define CASE(r) case r: return mfma_lds<r>().total;
        SFR_MFMA_R_LIST(CASE)
#undef CASE
    default: return 0;
    }
}

int sweep_mfma_width(int R, int tiles)
{
    if (wide16(R, tiles)) return MShape<16, 8>::WIDTH;
    switch (R) {
#define CASE(r) case r: return MShape<r>::WIDTH;
        SFR_MFMA_R_LIST(CASE)
#undef CASE
    default: return 0;
    }
}

static void* sweep_mfma_fn(int R, int tiles, bool bf16, bool rb)
{
    if (wide16(R, tiles))
        return bf16 ? reinterpret_cast<void*>(&sweep_mfma_kernel<16, true, 8>)
                    : reinterpret_cast<void*>(&sweep_mfma_kernel<16, false, 8>);
    if (rb) {
        switch (R) {
#define CASE(r)                                                                             \
    case r:                                                                                 \
        return bf16 ? reinterpret_cast<void*>(&sweep_mfma_kernel<r, true, 0, true>)         \
                    : reinterpret_cast<void*>(&sweep_mfma_kernel<r, false, 0, true>);
            SFR_MFMA_RB_LIST(CASE)
#undef CASE
        default: return nullptr;
        }
    }
    switch (R) {
#define CASE(r)                                                                             \
    case r:                                                                                 \
        return bf16 ? reinterpret_cast<void*>(&sweep_mfma_kernel<r, true>)                  \
                    : reinterpret_cast<void*>(&sweep_mfma_kernel<r, false>);
        SFR_MFMA_R_LIST(CASE)
#undef CASE
    default: return nullptr;
    }
}

hipError_t sweep_mfma_prepare(int R, int tiles, bool rb, size_t lds, int* blocks_per_cu)
{
    // both operand forms share the launch shape and LDS size
    for (int bf = 1; bf >= 0; --bf) {
        void* fn = sweep_mfma_fn(R, tiles, bf != 0, rb);
        if (!fn) return hipErrorInvalidValue;
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, sweep_mfma_fn(R, tiles, false, rb), kMTPB,
                                                        lds);
}

hipError_t launch_sweep_mfma(const SweepArgs<float>& a, int R, int tiles, bool rb, int grid, size_t lds,
                             hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, bool bf16)
{
#define LAUNCH_TW(r, BF, TW, RBF)                                                                           \
    if (ev0)                                                                                                \
        hipExtLaunchKernelGGL((sweep_mfma_kernel<r, BF, TW, RBF>), dim3(grid), dim3(kMTPB), (uint32_t)lds, s, \
                              ev0, ev1, 0u, a);                                                             \
    else                                                                                                    \
        hipLaunchKernelGGL((sweep_mfma_kernel<r, BF, TW, RBF>), dim3(grid), dim3(kMTPB), lds, s, a);
#define LAUNCH(r, BF) LAUNCH_TW(r, BF, 0, false)
    if (rb) {
        switch (R) {
#define CASE(r)                           \
    case r:                               \
        if (bf16) {                       \
            LAUNCH_TW(r, true, 0, true)   \
        } else {                          \
            LAUNCH_TW(r, false, 0, true)  \
        }                                 \
        return hipGetLastError();
            SFR_MFMA_RB_LIST(CASE)
#undef CASE
        default: return hipErrorInvalidValue;
        }
    }
    if (wide16(R, tiles)) {
        if (bf16) {
            LAUNCH_TW(16, true, 8, false)
        } else {
            LAUNCH_TW(16, false, 8, false)
        }
        return hipGetLastError();
    }
    switch (R) {
#define CASE(r)                 \
    case r:                     \
        if (bf16) {             \
            LAUNCH(r, true)     \
        } else {                \
            LAUNCH(r, false)    \
        }                       \
        return hipGetLastError();
        SFR_MFMA_R_LIST(CASE)
#undef CASE
#undef LAUNCH
#undef LAUNCH_TW
    default: return hipErrorInvalidValue;
    }
}

}  // namespace sfr
