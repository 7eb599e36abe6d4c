// FP64 r x r algebra of one FR-ADM step on the matrix cores
// (v_mfma_f64_16x16x4_f64).
//
// Matrices of up to 32 x 32 live in LDS (row pitch LDP) padded to RT = 16 NB
// (NB = 1 up to r = 16, else 2) with an identity block on the padded
// indices, so every product is block diagonal and exact on the leading
// r x r block.  A product C = A B is computed by NB^2 wavefronts, wavefront w
// forming the 16 x 16 output block (w / NB, w % NB) from 4 NB chained
// matrix-core steps whose operands it reads straight from LDS: lane l
// supplies A[i + l % 16][k + l / 16] and B[k + l / 16][j + l % 16] for each
// 4-wide k chunk and receives C[i + l / 16 + 4 e][j + l % 16], e = 0..3.
//
// Inverse square roots: the coupled Newton-Schulz iteration on A / s
// (s >= lambda_max, so the spectrum lies in (0, 1]):
//   W_k = Z_k Y_k,  T_k = (3 I - W_k) / 2,  Y_{k+1} = Y_k T_k,  Z_{k+1} = T_k Z_k,
// from Y_0 = A / s, Z_0 = I; Y_k -> (A / s)^{1/2} and Z_k -> (A / s)^{-1/2}
// (Higham, Functions of Matrices, Sec. 6.7).  Each eigenvalue w of W moves
// as w -> w (3 - w)^2 / 4, monotonically towards 1 from (0, 1], so
// ||W_k - I||_F decreases at every step; once it is <= kNsTol one more
// update is made (quadratic convergence: error ~ kNsTol^2).  Iterations
// grow as log(cond(A)) (about 2.25x per step for the smallest eigenvalue).
// Its result is accurate to about cond(A) eps: if the iteration stalls,
// grows, runs past kNsCap steps, or the result's norm bounds cond(A) above
// a limit set by the solve's precision, the caller falls back to the
// warm-started Jacobi eigendecompositions (small_la.hpp), which also decide
// rank loss.
#pragma once

#include "small_la.hpp"

namespace sfr {

typedef double f64x4 __attribute__((ext_vector_type(4)));

template <int R> constexpr int ns_nb() { return R <= 16 ? 1 : 2; }

constexpr int kNsCap = 40;        // Newton-Schulz steps before the Jacobi fallback
constexpr double kNsTol = 1e-8;   // ||W - I||_F at which one last update is made

// Threads of the algebra synchronise with a wavefront fence (NB = 1: one
// wavefront) or a workgroup barrier (NB = 2: every thread of the workgroup
// takes part; wavefronts beyond the first four only wait).
template <int NB>
__device__ __forceinline__ void ns_sync()
{
    if constexpr (NB == 1) wsync();
    else __syncthreads();
}

// This lane's four entries of its wavefront's output block.
template <int NB>
struct NsLane {
    int bi, bj, c, g;
    bool act;
    __device__ __forceinline__ NsLane()
    {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        act = wave < NB * NB;
        bi = act ? wave / NB : 0;
        bj = act ? wave % NB : 0;
        c = lane & 15;
        g = lane >> 4;
    }
    __device__ __forceinline__ int row(int e) const { return 16 * bi + g + 4 * e; }
    __device__ __forceinline__ int col() const { return 16 * bj + c; }
};

// The lane's output block of A B (A, B in LDS).
template <int NB>
__device__ __forceinline__ f64x4 ns_mm(const NsLane<NB>& L, const double* A, const double* B)
{
    constexpr int KC = 4 * NB;
    double a[KC], b[KC];
    const int i = 16 * L.bi + L.c, j = 16 * L.bj + L.c;
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
        const int k = 4 * kc + L.g;
        a[kc] = A[i * LDP + k];
        b[kc] = B[k * LDP + j];
    }
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kc], b[kc], acc, 0, 0, 0);
    return acc;
}

template <int NB>
__device__ __forceinline__ void ns_st(const NsLane<NB>& L, double* C, const f64x4& v)
{
#pragma unroll
    for (int e = 0; e < 4; ++e) C[L.row(e) * LDP + L.col()] = v[e];
}

// Sum over the 64 lanes of a wavefront, the same value on every lane: a
// butterfly within rows of 16 lanes by DPP (quad permutations, half-row
// and row mirrors; each step adds two disjoint partial sums, so every lane
// of a row ends with the same row sum), then the four row sums in row order.
template <int CTRL>
__device__ __forceinline__ double ns_dpp(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double ns_readlane(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double ns_wave_sum(double v)
{
    v += ns_dpp<0xB1>(v);    // quad_perm [1,0,3,2]
    v += ns_dpp<0x4E>(v);    // quad_perm [2,3,0,1]
    v += ns_dpp<0x141>(v);   // row_half_mirror
    v += ns_dpp<0x140>(v);   // row_mirror
    return (ns_readlane(v, 0) + ns_readlane(v, 16)) + (ns_readlane(v, 32) + ns_readlane(v, 48));
}

// Sum of v over the algebra's threads.  NB = 2: through red[0..3] and one
// workgroup barrier (a caller alternates red slots between calls that have
// no barrier between them).
template <int NB>
__device__ __forceinline__ double ns_sum(double v, double* red)
{
    v = ns_wave_sum(v);
    if constexpr (NB == 1) {
        return v;
    } else {
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        if (lane == 0 && wave < 4) red[wave] = v;
        __syncthreads();
        return (red[0] + red[1]) + (red[2] + red[3]);
    }
}

// One wavefront (NB = 1): the lane's output block of A B with A read by
// rows from LDS and B held in registers in the output layout (element kc of
// a lane is the B operand of k chunk kc).
__device__ __forceinline__ f64x4 ns_mm_lr(const NsLane<1>& L, const double* A, const f64x4& b)
{
    double a[4];
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) a[kc] = A[L.c * LDP + 4 * kc + L.g];
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[kc], b[kc], acc, 0, 0, 0);
    return acc;
}

// lambda_max(S) <= ||S^4||_F^{1/4} for symmetric S: the scale of the
// Newton-Schulz start (within r^{1/8} of lambda_max, against r^{1/2} for
// ||S||_F), from the lane's block v of S (identity outside the leading
// r x r block) with S2 = S S staged in Sq.  The padded block contributes
// r_pad to ||S^4||_F^2 exactly and is removed.
template <int NB>
__device__ __forceinline__ double ns_scale(const NsLane<NB>& L, const f64x4& v, double* Ss, double* Sq, double* red,
                                           int r)
{
    if (L.act) ns_st<NB>(L, Ss, v);
    ns_sync<NB>();
    if (L.act) ns_st<NB>(L, Sq, ns_mm<NB>(L, Ss, Ss));
    ns_sync<NB>();
    double f = 0.0;
    if (L.act) {
        const f64x4 q = ns_mm<NB>(L, Sq, Sq);
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (L.row(e) < r && L.col() < r) f = fma(q[e], q[e], f);
    }
    f = ns_sum<NB>(f, red);
    return sqrt(sqrt(sqrt(f))) * (1.0 + 1e-12);
}

// C = Sym(A)^{-1/2} on the leading r x r block, identity on the padded
// block, by Newton-Schulz.  A is read only.  Y0, Y1, Z0, Z1, T: scratch;
// red: 12 doubles.  Returns false (C undefined) when the iteration stalls,
// grows, runs past kNsCap steps, or ||Z||_F^2 >= kappa_max, an upper bound
// on cond(A) (with s >= lambda_max, cond(A) <= s / lambda_min = ||Z||_2^2):
// the Newton-Schulz result is accurate to about cond(A) eps, so the caller
// then takes the eigendecomposition.  Uniform over the algebra's threads.
template <int NB>
__device__ bool ns_invsqrt(const double* A, double* C, double* Y0, double* Y1, double* Z0, double* Z1, double* T,
                           double* red, int r, double kappa_max)
{
    const NsLane<NB> L;
    f64x4 w = {0.0, 0.0, 0.0, 0.0};
    if (L.act) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = L.row(e), j = L.col();
            w[e] = (i < r && j < r) ? 0.5 * (A[i * LDP + j] + A[j * LDP + i]) : (i == j ? 1.0 : 0.0);
        }
    }
    const double s = ns_scale<NB>(L, w, Y1, Z1, red, r);
    if (!(s > 0.0) || !isfinite(s)) return false;
    const double is = 1.0 / s;
    // Y_0 = Sym(A) / s (identity on the padded block, a fixed point of the
    // iteration), Z_0 = I, so W_0 = Y_0
    f64x4 y = w, z;
    if (L.act) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = L.row(e), j = L.col();
            if (i < r && j < r) y[e] *= is;
            z[e] = (i == j) ? 1.0 : 0.0;
        }
        ns_st<NB>(L, Y0, y);
        ns_st<NB>(L, Z0, z);
    }
    w = y;
    int cur = 0;
    double prev = INFINITY;
    bool ok = false;
    for (int it = 0; it < kNsCap; ++it) {
        // current and next iterates (pointer selects, no indexed arrays)
        double* Yc = cur ? Y1 : Y0;
        double* Zc = cur ? Z1 : Z0;
        double* Yn = NB == 1 ? Yc : (cur ? Y0 : Y1);
        double* Zn = NB == 1 ? Zc : (cur ? Z0 : Z1);
        if (it > 0 && L.act) {
            if constexpr (NB == 1) w = ns_mm_lr(L, Zc, y);
            else w = ns_mm<NB>(L, Zc, Yc);
        }
        double d2 = 0.0;
        f64x4 t;
        if (L.act) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = L.row(e), j = L.col();
                const double id = (i == j) ? 1.0 : 0.0;
                t[e] = fma(-0.5, w[e], 1.5 * id);
                const double d = w[e] - id;
                if (i < r && j < r) d2 = fma(d, d, d2);
            }
            ns_st<NB>(L, T, t);
        }
        if constexpr (NB == 1) {
            // one wavefront: T's stores before the fence, the update's
            // products overlap the reduction, which decides afterwards
            wsync();
            const f64x4 yn = ns_mm_lr(L, Yc, t);
            const f64x4 zn = ns_mm_lr(L, T, z);
            d2 = ns_wave_sum(d2);
            if (!(d2 < prev)) break;   // not finite, or no longer contracting
            prev = d2;
            // in place: this wavefront's reads of Yc and T are complete
            ns_st<NB>(L, Yn, yn);
            ns_st<NB>(L, Zn, zn);
            wsync();
            y = yn;
            z = zn;
        } else {
            d2 = ns_sum<NB>(d2, red + 4 + 4 * (it & 1));   // its barrier publishes T
            if (!(d2 < prev)) break;
            prev = d2;
            if (L.act) {
                const f64x4 yn = ns_mm<NB>(L, Yc, T);
                const f64x4 zn = ns_mm<NB>(L, T, Zc);
                ns_st<NB>(L, Yn, yn);
                ns_st<NB>(L, Zn, zn);
            }
            ns_sync<NB>();
            cur ^= 1;
        }
        if (prev <= kNsTol * kNsTol) {
            ok = true;
            break;
        }
    }
    if (!ok) return false;
    // C = Sym(Z) / sqrt(s)
    const double rs = sqrt(is);
    const double* Zf = cur ? Z1 : Z0;
    double z2 = 0.0;
    f64x4 cv = {0.0, 0.0, 0.0, 0.0};
    if (L.act) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = L.row(e), j = L.col();
            const bool in = i < r && j < r;
            const double zz = 0.5 * (Zf[i * LDP + j] + Zf[j * LDP + i]);
            if (in) z2 = fma(zz, zz, z2);
            cv[e] = in ? zz * rs : (i == j ? 1.0 : 0.0);
        }
    }
    z2 = ns_sum<NB>(z2, red + 8);
    if (!(z2 < kappa_max)) return false;
    if (L.act) ns_st<NB>(L, C, cv);
    ns_sync<NB>();
    return true;
}

// The r x r algebra of one FixedRankOptStep (Alg. 2) in its one-pass form
// (Sec. 4.1, eqs. (7), (8)) from the Grams G_P = P^T P, G_Q = Q^T Q of the
// products P = X V_0, Q = X^T P and the previous SPD factor B_0:
//   C1 = (B_0 G_P B_0)^{-1/2}               U = P (B_0 C1)
//   K  = B_0 C1 B_0,  C2 = (K G_Q K)^{-1/2}    V = Q (K C2)
//   B  = Sym(C1 B_0 G_Q K C2)               a_i = P_i (B_0 C1 B)
// Buffers (RT x LDP each, identity padded): on entry Bm = B_0, Gp, Gq; on
// success T1 = B_0 C1 (U transform), Gp = K C2 (V transform), Y0 = B and
// Am = B_0 C1 B (row factor transform).  X, Am, C, Y1, Z0, Z1, T, R1, Km:
// scratch.  Returns false if either inverse square root is not trusted
// (ns_invsqrt); Bm, Gp and Gq are then intact.  Uniform.
template <int R>
__device__ bool ns_lstep(double* Bm, double* Gp, double* Gq, double* X, double* Am, double* C, double* Y0,
                         double* Y1, double* Z0, double* Z1, double* T, double* T1, double* R1, double* Km,
                         double* red, int r, double kappa_max)
{
    constexpr int NB = ns_nb<R>();
    const NsLane<NB> L;
    // A = B_0 G_P B_0
    if (L.act) ns_st<NB>(L, X, ns_mm<NB>(L, Gp, Bm));
    ns_sync<NB>();
    if (L.act) ns_st<NB>(L, Am, ns_mm<NB>(L, Bm, X));
    ns_sync<NB>();
    if (!ns_invsqrt<NB>(Am, C, Y0, Y1, Z0, Z1, T, red, r, kappa_max)) return false;
    // T1 = B_0 C1, R1 = C1 B_0 = T1^T
    if (L.act) {
        const f64x4 t1 = ns_mm<NB>(L, Bm, C);
        const f64x4 r1 = ns_mm<NB>(L, C, Bm);
        ns_st<NB>(L, T1, t1);
        ns_st<NB>(L, R1, r1);
    }
    ns_sync<NB>();
    // K = Sym(T1 B_0): (T1 B_0)^T = B_0 R1, both formed for the lane's block
    if (L.act) {
        const f64x4 x = ns_mm<NB>(L, T1, Bm);
        const f64x4 xt = ns_mm<NB>(L, Bm, R1);
        ns_st<NB>(L, Km, 0.5 * (x + xt));
    }
    ns_sync<NB>();
    // A = K G_Q K
    if (L.act) ns_st<NB>(L, X, ns_mm<NB>(L, Gq, Km));
    ns_sync<NB>();
    if (L.act) ns_st<NB>(L, Am, ns_mm<NB>(L, Km, X));
    ns_sync<NB>();
    if (!ns_invsqrt<NB>(Am, C, Y0, Y1, Z0, Z1, T, red, r, kappa_max)) return false;
    // TV = K C2 (into Gp, free since the first product)
    if (L.act) ns_st<NB>(L, Gp, ns_mm<NB>(L, Km, C));
    ns_sync<NB>();
    // B = Sym(C1 B_0 G_Q K C2) = Sym(R1 (G_Q TV))
    if (L.act) ns_st<NB>(L, X, ns_mm<NB>(L, Gq, Gp));
    ns_sync<NB>();
    if (L.act) ns_st<NB>(L, Am, ns_mm<NB>(L, R1, X));
    ns_sync<NB>();
    if (L.act) {
        f64x4 b;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = L.row(e), j = L.col();
            b[e] = 0.5 * (Am[i * LDP + j] + Am[j * LDP + i]);
        }
        ns_st<NB>(L, Y0, b);
    }
    ns_sync<NB>();
    // row factor transform B_0 C1 B = T1 B
    if (L.act) ns_st<NB>(L, Am, ns_mm<NB>(L, T1, Y0));
    ns_sync<NB>();
    return true;
}


// ---- register form for one wavefront (NB = 1, R <= 16) ----------------
// A 16 x 16 matrix X is held as the lane's four entries X[g + 4e][c]
// (c = lane % 16, g = lane / 16): the output layout of the f64 matrix-core
// step.  That layout is also the step's B-operand layout, and read as the A
// operand it gives X^T (chunk kc takes A[c][4 kc + g]).  So ns_tmm(X, Y) =
// X^T Y takes both operands from registers, which is X Y whenever X is
// symmetric: every product of the step is arranged that way (a symmetric
// left factor, or a left factor whose transpose is at hand), and only the
// two symmetrisations of Z pass through LDS.
__device__ __forceinline__ f64x4 ns_tmm(const f64x4& x, const f64x4& y)
{
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x[kc], y[kc], acc, 0, 0, 0);
    return acc;
}

// The lane's entries of V^T, through the LDS scratch S (16 x LDP doubles).
__device__ __forceinline__ f64x4 ns_tile_t(const f64x4& v, double* S)
{
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4;
#pragma unroll
    for (int e = 0; e < 4; ++e) S[(g + 4 * e) * LDP + c] = v[e];
    wsync();
    f64x4 t;
#pragma unroll
    for (int e = 0; e < 4; ++e) t[e] = S[c * LDP + g + 4 * e];
    wsync();
    return t;
}

// C = A^{-1/2} by Newton-Schulz as ns_invsqrt, in registers.  a: the lane's
// entries of the symmetric A (the padded block is taken as identity).
// Returns false under the same conditions as ns_invsqrt.
__device__ inline bool ns1_invsqrt(const f64x4& a, f64x4& cout, double* S, int r, double kappa_max)
{
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4;
    f64x4 w, id;
    bool in[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int i = g + 4 * e;
        in[e] = (i < r) && (c < r);
        id[e] = (i == c) ? 1.0 : 0.0;
        w[e] = in[e] ? a[e] : id[e];
    }
    // s = ||A^4||_F^{1/4} (leading block) >= lambda_max
    const f64x4 s2 = ns_tmm(w, w);
    const f64x4 s4 = ns_tmm(s2, s2);
    double f = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e)
        if (in[e]) f = fma(s4[e], s4[e], f);
    f = ns_wave_sum(f);
    const double s = sqrt(sqrt(sqrt(f))) * (1.0 + 1e-12);
    if (!(s > 0.0) || !isfinite(s)) return false;
    const double is = 1.0 / s;
    // Y_0 = A / s (identity on the padded block), Z_0 = I, W_0 = Y_0
    f64x4 y, z = id;
#pragma unroll
    for (int e = 0; e < 4; ++e) y[e] = in[e] ? w[e] * is : w[e];
    w = y;
    // The iterates are symmetric only up to rounding.  Reading Z and Y
    // transposed as left factors keeps the iteration's accuracy, but T must
    // enter T Z as itself (with T^T the iteration stalls or drifts once cond(A)
    // passes about 1e3), so its transpose is formed too, from W^T = Y^T Z:
    // the same products in the same order as W = Z^T Y.
    f64x4 wt = y;
    double prev = INFINITY;
    bool ok = false;
    for (int it = 0; it < kNsCap; ++it) {
        if (it > 0) {
            w = ns_tmm(z, y);    // W = Z^T Y
            wt = ns_tmm(y, z);   // W^T
        }
        f64x4 t, tt;
        double d2 = 0.0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            t[e] = fma(-0.5, w[e], 1.5 * id[e]);
            tt[e] = fma(-0.5, wt[e], 1.5 * id[e]);
            const double d = w[e] - id[e];
            if (in[e]) d2 = fma(d, d, d2);
        }
        const f64x4 yn = ns_tmm(y, t);    // Y^T T
        const f64x4 zn = ns_tmm(tt, z);   // T Z
        d2 = ns_wave_sum(d2);
        if (!(d2 < prev)) break;   // not finite, or no longer contracting
        prev = d2;
        y = yn;
        z = zn;
        if (prev <= kNsTol * kNsTol) {
            ok = true;
            break;
        }
    }
    if (!ok) return false;
    // C = Sym(Z) / sqrt(s)
    const f64x4 zt = ns_tile_t(z, S);
    const double rs = sqrt(is);
    double z2 = 0.0;
    f64x4 cv;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const double zz = 0.5 * (z[e] + zt[e]);
        if (in[e]) z2 = fma(zz, zz, z2);
        cv[e] = in[e] ? zz * rs : id[e];
    }
    z2 = ns_wave_sum(z2);
    if (!(z2 < kappa_max)) return false;
    cout = cv;
    return true;
}

// ns_lstep for one wavefront with every matrix in registers.  b0: the lane's
// entries of B_0; Gp, Gq: the Grams in LDS (read only); S: LDS scratch.  On
// success bn = B, tu = B_0 C1 B (row factor transform), tubar = B_0 C1 (U
// transform), tv = K C2 (V transform), as the lane's entries.  Uniform.
__device__ inline bool ns1_lstep(const f64x4& b0, const double* Gp, const double* Gq, double* S, int r,
                                 double kappa_max, f64x4& bn, f64x4& tu, f64x4& tubar, f64x4& tv)
{
    const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4;
    f64x4 gp, gq;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        gp[e] = Gp[(g + 4 * e) * LDP + c];
        gq[e] = Gq[(g + 4 * e) * LDP + c];
    }
    // A1 = B_0 G_P B_0, symmetrised: B_0 (G_P B_0) and (G_P B_0)^T B_0
    const f64x4 x1 = ns_tmm(gp, b0);
    const f64x4 a1 = 0.5 * (ns_tmm(b0, x1) + ns_tmm(x1, b0));
    f64x4 c1;
    if (!ns1_invsqrt(a1, c1, S, r, kappa_max)) return false;
    const f64x4 t1 = ns_tmm(b0, c1);   // B_0 C1
    const f64x4 r1 = ns_tmm(c1, b0);   // C1 B_0 = T1^T
    // K = Sym(T1 B_0): T1 B_0 = R1^T B_0 and its transpose B_0 R1
    const f64x4 kk = 0.5 * (ns_tmm(r1, b0) + ns_tmm(b0, r1));
    // A2 = K G_Q K, symmetrised
    const f64x4 x2 = ns_tmm(gq, kk);
    const f64x4 a2 = 0.5 * (ns_tmm(kk, x2) + ns_tmm(x2, kk));
    f64x4 c2;
    if (!ns1_invsqrt(a2, c2, S, r, kappa_max)) return false;
    tv = ns_tmm(kk, c2);                // K C2
    // B = Sym(C1 B_0 G_Q TV) = Sym(T1^T X3), X3 = G_Q TV
    const f64x4 x3 = ns_tmm(gq, tv);
    bn = 0.5 * (ns_tmm(t1, x3) + ns_tmm(x3, t1));
    tubar = t1;
    tu = ns_tmm(r1, bn);                // R1^T B = T1 B
    return true;
}

}  // namespace sfr
