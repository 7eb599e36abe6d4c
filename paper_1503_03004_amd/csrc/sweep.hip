// One fused pass over the data per FR-ADM iteration (Alg. 1 with the
// L-step of Alg. 2), gfx950.
//
// Work decomposition
//   * Rows are cut into bands of H rows (one or more per wavefront).  Each
//     band is owned by a cluster of c workgroups; member q of a cluster
//     covers the column slice [q W, (q+1) W).  Clusters are formed from
//     workgroups of one XCD (workgroup g runs on XCD g % 8), so their
//     exchange stays in one L2; clusters wider than one XCD's share of the
//     grid span XCDs instead.  A workgroup is 8 wavefronts (one per CU)
//     while two wavefronts fit a SIMD, else 4.
//   * Row pass (phase 1): a group of `lpr` lanes owns one row of the band;
//     each lane streams `nv` 16-byte vectors of M and Y_{k-1}, rebuilds
//     l_ij = a_i . V_j (r FMAs, V slice staged in LDS), applies the S- and
//     dual steps, writes Y_k, forms x_ij and accumulates p_i = sum_j x_ij V_j.
//     x goes to LDS for phase 2.
//   * If c > 1 the members add their partial p_i through tagged 64-bit
//     words in global memory (value | tag << 32, so no fences are needed),
//     two bands behind the row pass (three band buffers of x and p in LDS),
//     so a member may run up to two bands ahead of the slowest one before
//     it waits.  A member can then publish at most five bands ahead of one
//     still reading, so eight exchange slots are cycled.
//   * Column pass (phase 2): Q_j += x_ij p_i from the LDS copy of x:
//     Q = X^T X V with no second read of the data.  For FP32 wide slices
//     (rank buckets up to 10, slices of 512 or 1024 columns) it runs on the
//     matrix cores: wave w owns 16-column tiles of its member's slice and
//     adds X_tile^T (16 columns x 4 rows) . P (4 rows x 16 ranks) with
//     v_mfma_f32_16x16x4_f32 (exact FP32 products, FP32 accumulation), H/4
//     steps per band.  Otherwise thread-owned columns accumulate it on the
//     vector ALU.
// HBM traffic per element: read M, read Y_{k-1}, write Y_k.
#include "exchange.hpp"
#include "sfr_internal.hpp"

#include <hip/hip_ext.h>

namespace sfr {

template <typename T>
__device__ __forceinline__ T group_sum(T v, int width)
{
    for (int off = width >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// DPP lane exchange within rows of 16 lanes (compile-time control word).
template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum each of the R values over aligned groups of `width` lanes (a power of
// two, 2..64); every lane of a group receives its group's sums.  Steps
// inside a row of 16 lanes use DPP (quad permutations, half-row and row
// mirrors, each of which pairs lanes holding disjoint partial sums); the
// 16- and 32-lane steps use one cross-lane permute per value, all issued
// together.
template <typename T, int R>
__device__ __forceinline__ void group_sum_all(T (&p)[R], int width)
{
    if (width >= 2) {
#pragma unroll
        for (int k = 0; k < R; ++k) p[k] += dpp<0xB1>(p[k]);   // quad_perm [1,0,3,2]
    }
    if (width >= 4) {
#pragma unroll
        for (int k = 0; k < R; ++k) p[k] += dpp<0x4E>(p[k]);   // quad_perm [2,3,0,1]
    }
    if (width >= 8) {
#pragma unroll
        for (int k = 0; k < R; ++k) p[k] += dpp<0x141>(p[k]);  // row_half_mirror
    }
    if (width >= 16) {
#pragma unroll
        for (int k = 0; k < R; ++k) p[k] += dpp<0x140>(p[k]);  // row_mirror
    }
    if (width >= 32) {
        T t[R];
#pragma unroll
        for (int k = 0; k < R; ++k) t[k] = __shfl_xor(p[k], 16, 64);
#pragma unroll
        for (int k = 0; k < R; ++k) p[k] += t[k];
    }
    if (width >= 64) {
        T t[R];
#pragma unroll
        for (int k = 0; k < R; ++k) t[k] = __shfl_xor(p[k], 32, 64);
#pragma unroll
        for (int k = 0; k < R; ++k) p[k] += t[k];
    }
}

template <typename T>
__device__ __forceinline__ T readlane(T v, int lane)
{
    if constexpr (sizeof(T) == 4) {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
    } else {
        const long long b = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
        const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
        return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    }
}

// Exchange words of one band are read ahead of use: a lane holds up to
// kGatherAhead words, loaded before its row pass and checked after it.
constexpr int kGatherAhead = 2;
// Exchange words a lane reads together when it gathers a band's words after
// its row pass (clusters too wide for the words read ahead): 8 for FP32
// values, 4 for FP64 (two words each).
template <typename T>
constexpr int gather_batch() { return sizeof(T) == 4 ? 8 : 4; }

// Byte offsets of the dynamic LDS regions of one sweep workgroup.
struct SweepLds {
    size_t tu, tv, vs, xs, ps, gx, qred, red, total;
};

__host__ __device__ inline size_t al16(size_t x) { return (x + 15) & ~size_t(15); }

// Gather lag (bands between a row pass and the column pass that uses it)
// and the number of band buffers of x and p.
__host__ __device__ inline int sweep_lag(int c) { return c > 1 ? 2 : 1; }

// Whether the column pass runs on the matrix cores: FP32, rank buckets up to
// 10 (512-thread workgroups), slices of whole 16-column tiles per wave.
template <typename T>
__host__ __device__ inline bool sweep_mcol(int R, int lpr, int W, int tpb)
{
    return sizeof(T) == 4 && R <= 10 && tpb == 512 && W >= tpb && W % (16 * (tpb / 64)) == 0 &&
           W / (16 * (tpb / 64)) <= 8 && lpr >= 32;
}

// Row pitch (elements) of the LDS copy of x: the matrix-core column pass
// reads four rows of 16 consecutive columns per instruction, so its rows
// are offset by 16 banks.
template <typename T>
__host__ __device__ inline int sweep_xpitch(int R, int lpr, int W, int tpb)
{
    return sweep_mcol<T>(R, lpr, W, tpb) ? W + 16 : W;
}

template <typename T>
__host__ __device__ inline SweepLds sweep_lds(int R, int lpr, int W, int c, int tpb)
{
    const int H = (tpb / 64) * (64 / lpr);
    const int HG = (W >= tpb) ? 1 : tpb / W;
    const int nbuf = sweep_lag(c) + 1;
    const int XP = sweep_xpitch<T>(R, lpr, W, tpb);
    SweepLds L;
    size_t o = 0;
    L.tu = o; o = al16(o + sizeof(T) * R * R);
    L.tv = o; o = al16(o + sizeof(T) * R * R);
    L.vs = o; o = al16(o + sizeof(T) * (size_t)R * W);
    L.xs = o; o = al16(o + sizeof(T) * nbuf * (size_t)H * XP);
    L.ps = o; o = al16(o + sizeof(T) * nbuf * (size_t)H * R);
    L.gx = o; o = al16(o + (c > 1 ? sizeof(T) * (tpb / 64) * (size_t)c * R : 0));
    L.qred = o; o = al16(o + (W < tpb ? sizeof(T) * (size_t)HG * W * R : 0));
    L.red = o; o = al16(o + sizeof(double) * (tpb / 64));
    L.total = o;
    return L;
}

// Two waves per SIMD while the per-lane register state fits in 256 VGPRs
// (workgroups of 8 waves); larger ranks take one wave per SIMD and the full
// register file (workgroups of 4 waves).
template <typename T, int R>
constexpr int sweep_waves_per_simd() { return (sizeof(T) * R <= 40) ? 2 : 1; }
template <typename T, int R>
constexpr int sweep_tpb() { return sweep_waves_per_simd<T, R>() == 2 ? 512 : 256; }
// Columns a thread accumulates in the column pass (bounds the slice width
// W <= cpt2 * threads); two for the widest ranks to keep Q in registers.
template <typename T, int R>
constexpr int sweep_cpt2()
{
    return (R > 16) ? 2 : (64 * 4 * Vec<T>::N + sweep_tpb<T, R>() - 1) / sweep_tpb<T, R>();
}

typedef float sw_f32x4 __attribute__((ext_vector_type(4)));

// MC: the matrix-core column pass (the host launches it exactly where
// sweep_mcol holds).
template <typename T, int R, bool MC>
__global__ void __launch_bounds__((sweep_tpb<T, R>()), 1) sweep_kernel(SweepArgs<T> a)
{
    DevState* st = const_cast<DevState*>(a.st);
    if (st->done) return;
    constexpr int TPB = sweep_tpb<T, R>();
    constexpr int NW = TPB / 64;
    constexpr int VEC = Vec<T>::N;
    constexpr int WD = Words<T>::N;
    constexpr int NVMAX = 4;
    constexpr int CPT2MAX = sweep_cpt2<T, R>();   // columns per thread, column pass

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lpr = a.lpr, nv = a.nv, W = a.W, c = a.c;
    const int rpw = 64 / lpr, H = NW * rpw;
    const int XP = MC ? W + 16 : W;   // sweep_xpitch
    const int lag = sweep_lag(c), nbuf = lag + 1;
    const int li = lane % lpr, rg = lane / lpr, gbase = lane - li;
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
    const int c0 = q * W;
    const int m = a.m, n = a.n;
    const int64_t ldm = st->ldm, ldy = a.ldy;
    const T* __restrict__ M = static_cast<const T*>(st->M);
    const int mode = a.mode;
    const T lam = (T)st->lambda;
    const T mu_prev = (T)st->mu_prev;
    const T imu_prev = (mode != 0) ? (T)(1.0 / st->mu_prev) : T(0);
    const T imu_cur = (T)(1.0 / st->mu);
    const uint32_t kiter = (uint32_t)st->k;
    int32_t* tflag = &st->exch_timeout;

    extern __shared__ __align__(16) unsigned char smem[];
    const SweepLds L = sweep_lds<T>(R, lpr, W, c, TPB);
    T* TUs = reinterpret_cast<T*>(smem + L.tu);
    T* TVs = reinterpret_cast<T*>(smem + L.tv);
    T* Vs = reinterpret_cast<T*>(smem + L.vs);
    T* Xs = reinterpret_cast<T*>(smem + L.xs);
    T* Ps = reinterpret_cast<T*>(smem + L.ps);
    T* Gx = reinterpret_cast<T*>(smem + L.gx);
    T* Qred = reinterpret_cast<T*>(smem + L.qred);
    double* red = reinterpret_cast<double*>(smem + L.red);

    {
        const T* tu = st_TU<T>(st);
        const T* tv = st_TV<T>(st);
        for (int e = tid; e < R * R; e += TPB) {
            const int r0 = e / R, r1 = e % R;
            TUs[e] = tu[r0 * kMaxR + r1];
            TVs[e] = tv[r0 * kMaxR + r1];
        }
    }
    __syncthreads();
    // V slice of this member: V_j = Q_j TV, stored k-major (Vs[k][jj]).
    for (int jj = tid; jj < W; jj += TPB) {
        const int j = c0 + jj;
        T qrow[R];
#pragma unroll
        for (int t = 0; t < R; ++t) qrow[t] = (j < n) ? a.Qprev[(int64_t)j * R + t] : T(0);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            T s = 0;
#pragma unroll
            for (int t = 0; t < R; ++t) s = fma(qrow[t], TVs[t * R + k], s);
            Vs[k * W + jj] = s;
        }
    }
    __syncthreads();

    const int nbands = a.nbands, ncl = a.ncl;
    const int nbl = (cl < nbands) ? (nbands - 1 - cl) / ncl + 1 : 0;
    const int cpt2 = (W >= TPB) ? (W + TPB - 1) / TPB : 1;
    const int HG = (W >= TPB) ? 1 : TPB / W;
    double acc2 = 0.0;
    // column-pass accumulators: thread-owned columns (vector ALU), or this
    // lane's part of the wave's 16 x 16 Q tiles (matrix cores)
    constexpr int QE = MC ? 1 : CPT2MAX;
    constexpr int MT = MC ? 8 : 1;
    T Qacc[QE][R];
#pragma unroll
    for (int e = 0; e < QE; ++e)
#pragma unroll
        for (int k = 0; k < R; ++k) Qacc[e][k] = T(0);
    sw_f32x4 qm[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) qm[t] = sw_f32x4{0.f, 0.f, 0.f, 0.f};

    // Row-pass operands of the band being processed: all 2 * nv vectors of
    // a lane are issued together, one band ahead of their use.  Vectors out
    // of range read a valid dummy address and are zeroed at use.
    T mvv[NVMAX][VEC], ypv[NVMAX][VEC];
    auto issue_load = [&](int jb, int v) {
        const int bb = cl + jb * ncl;
        const int ii = bb * H + wave * rpw + rg;
        const int col = c0 + (li + lpr * v) * VEC;
        const bool ok = (v < nv) && (ii < m) && (col < n);
        load_vec_stream<T>(M + (ok ? (int64_t)ii * ldm + col : 0), mvv[v]);
        if (mode == 2) load_vec_stream<T>(a.Yprev + (ok ? (int64_t)ii * ldy + col : 0), ypv[v]);
    };
    if (nbl > 0) {
#pragma unroll
        for (int v = 0; v < NVMAX; ++v) issue_load(0, v);
    }

    for (int j = 0; j < nbl + lag; ++j) {
        // exchange words of band j - lag (c > 1): issued now, consumed after
        // this band's row pass
        const int nwords = c * R * WD;
        const bool ahead = (c > 1) && (j >= lag) && (nwords <= 64 * kGatherAhead);
        unsigned long long gw[kGatherAhead];
        if (ahead) {
            const int slot = (j - lag) & (kExchSlots - 1);
            const unsigned long long* base = a.exch + (((size_t)cl * kExchSlots + slot) * c) * H * R * WD;
#pragma unroll
            for (int g = 0; g < kGatherAhead; ++g) {
                const int e = lane + 64 * g;      // word index over (member, k, half)
                const int qq = e / (R * WD), rem = e % (R * WD);
                gw[g] = (e < nwords) ? peek_word(base + ((size_t)qq * H + wave) * R * WD + rem) : 0ull;
            }
        }
        if (j < nbl) {
            // ---------------- phase 1: row pass over band b ----------------
            const int b = cl + j * ncl;
            const int buf = j % nbuf;
            const int h = wave * rpw + rg;
            const int i = b * H + h;
            const bool row_ok = i < m;
            T av[R];
            if (mode != 0) {
                T prow[R];
#pragma unroll
                for (int t = 0; t < R; ++t) prow[t] = row_ok ? a.Pprev[(int64_t)i * R + t] : T(0);
                if (lpr == 64) {
                    // one row per wavefront: a_i is uniform, broadcast by readlane
                    T s = 0;
                    if (li < R) {
#pragma unroll
                        for (int t = 0; t < R; ++t) s = fma(prow[t], TUs[t * R + li], s);
                    }
#pragma unroll
                    for (int kk = 0; kk < R; ++kk) av[kk] = readlane(s, kk);
                } else if (lpr >= R) {
                    T s = 0;
                    if (li < R) {
#pragma unroll
                        for (int t = 0; t < R; ++t) s = fma(prow[t], TUs[t * R + li], s);
                    }
#pragma unroll
                    for (int kk = 0; kk < R; ++kk) av[kk] = __shfl(s, gbase + kk, 64);
                } else {
#pragma unroll
                    for (int kk = 0; kk < R; ++kk) {
                        T s = 0;
#pragma unroll
                        for (int t = 0; t < R; ++t) s = fma(prow[t], TUs[t * R + kk], s);
                        av[kk] = s;
                    }
                }
            } else {
#pragma unroll
                for (int kk = 0; kk < R; ++kk) av[kk] = T(0);
            }
            T p[R];
#pragma unroll
            for (int k = 0; k < R; ++k) p[k] = T(0);
            T rowacc = 0;
#pragma unroll
            for (int v = 0; v < NVMAX; ++v) {
                if (v >= nv) break;
                const int jj = (li + lpr * v) * VEC;
                const int col = c0 + jj;
                const bool ok = row_ok && (col < n);
                T mv[VEC], yp[VEC], x[VEC];
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    mv[e] = ok ? mvv[v][e] : T(0);
                    yp[e] = (ok && mode == 2) ? ypv[v][e] : T(0);
                }
                T vk[R][VEC];
#pragma unroll
                for (int k = 0; k < R; ++k) load_vec<T>(Vs + k * W + jj, vk[k]);
                if (mode == 0) {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) { x[e] = mv[e]; rowacc = fma(mv[e], mv[e], rowacc); }
                } else {
                    T yn[VEC];
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        T l = 0;
#pragma unroll
                        for (int k = 0; k < R; ++k) l = fma(av[k], vk[k][e], l);
                        const T Rr = mv[e] - l + yp[e] * imu_prev;
                        const T y = fmin(fmax(mu_prev * Rr, -lam), lam);
                        const T dy = y - yp[e];
                        rowacc = fma(dy, dy, rowacc);
                        x[e] = l + dy * imu_prev + y * imu_cur;
                        yn[e] = y;
                    }
                    if (ok) store_vec_stream<T>(a.Ynext + (int64_t)i * ldy + col, yn);
                }
                if (!ok) {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) x[e] = T(0);
                }
                store_vec<T>(Xs + ((size_t)buf * H + h) * XP + jj, x);
#pragma unroll
                for (int k = 0; k < R; ++k)
#pragma unroll
                    for (int e = 0; e < VEC; ++e) p[k] = fma(x[e], vk[k][e], p[k]);
                // this vector's registers are free: the next band's load
                // goes out now and lands during the rest of this row pass,
                // the reduction, the exchange and the column pass
                if (j + 1 < nbl) issue_load(j + 1, v);
            }
            acc2 += (double)rowacc;
            group_sum_all<T, R>(p, lpr);
            if (c == 1) {
                if (li == 0) {
#pragma unroll
                    for (int k = 0; k < R; ++k) Ps[((size_t)buf * H + h) * R + k] = p[k];
                }
            } else if (li < R) {
                // c > 1 only with lpr == 64 (one row per wave)
                T mine = 0;
#pragma unroll
                for (int kk = 0; kk < R; ++kk) mine = (kk == li) ? p[kk] : mine;
                const uint32_t tag = kiter * (uint32_t)a.nbl_max + (uint32_t)j + 1u;
                const int slot = j & (kExchSlots - 1);
                unsigned long long* dst =
                    a.exch + (((((size_t)cl * kExchSlots + slot) * c + q) * H + h) * R + li) * WD;
                publish<T>(dst, mine, tag);
            }
        }
        if (j >= lag) {
            const int jb = j - lag;
            const int b = cl + jb * ncl;
            const int buf = jb % nbuf;
            if (c > 1) {
                // gather the c partials of this wave's row of band jb
                const int h = wave;
                const uint32_t tag = kiter * (uint32_t)a.nbl_max + (uint32_t)jb + 1u;
                const int slot = jb & (kExchSlots - 1);
                T* gx = Gx + (size_t)wave * c * R;
                if (ahead) {
                    // words read before the row pass; re-poll only those whose
                    // tag has not arrived yet
                    uint32_t* gxw = reinterpret_cast<uint32_t*>(gx);
                    const unsigned long long* base = a.exch + (((size_t)cl * kExchSlots + slot) * c) * H * R * WD;
#pragma unroll
                    for (int g = 0; g < kGatherAhead; ++g) {
                        const int e = lane + 64 * g;
                        if (e < nwords) {
                            unsigned long long w = gw[g];
                            if ((uint32_t)(w >> 32) != tag) {
                                const int qq = e / (R * WD), rem = e % (R * WD);
                                w = spin_word(base + ((size_t)qq * H + h) * R * WD + rem, tag, tflag);
                            }
                            gxw[e] = (uint32_t)(w & 0xffffffffull);
                        }
                    }
                } else {
                    // a lane reads gather_batch<T>() of its words together (word
                    // indices clamped into range), then polls those whose tag
                    // has not arrived: one round trip per batch
                    const int nw = c * R;
                    const unsigned long long* base = a.exch + (((size_t)cl * kExchSlots + slot) * c) * H * R * WD;
                    constexpr int GB = gather_batch<T>();
                    for (int e0 = lane; e0 < nw; e0 += 64 * GB) {
                        unsigned long long w[GB][WD];
#pragma unroll
                        for (int u = 0; u < GB; ++u) {
                            const int e = min(e0 + 64 * u, nw - 1);
                            const int qq = e / R, k = e % R;
                            const unsigned long long* src = base + (((size_t)qq * H + h) * R + k) * WD;
#pragma unroll
                            for (int hw = 0; hw < WD; ++hw) w[u][hw] = peek_word(src + hw);
                        }
#pragma unroll
                        for (int u = 0; u < GB; ++u) {
                            const int e = e0 + 64 * u;
                            if (e < nw) {
                                const int qq = e / R, k = e % R;
                                const unsigned long long* src = base + (((size_t)qq * H + h) * R + k) * WD;
#pragma unroll
                                for (int hw = 0; hw < WD; ++hw)
                                    if ((uint32_t)(w[u][hw] >> 32) != tag) w[u][hw] = spin_word(src + hw, tag, tflag);
                                if constexpr (WD == 1) {
                                    gx[e] = __uint_as_float((uint32_t)(w[u][0] & 0xffffffffull));
                                } else {
                                    gx[e] = __longlong_as_double(
                                        (long long)((w[u][WD - 1] << 32) | (w[u][0] & 0xffffffffull)));
                                }
                            }
                        }
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (lane < R) {
                    T s = 0;
                    for (int qq = 0; qq < c; ++qq) s += gx[qq * R + lane];
                    Ps[((size_t)buf * H + h) * R + lane] = s;
                }
            }
            __syncthreads();
            if (q == 0) {
                for (int e = tid; e < H * R; e += TPB) {
                    const int hh = e / R, k = e % R;
                    const int i = b * H + hh;
                    if (i < m) a.Pnext[(int64_t)i * R + k] = Ps[((size_t)buf * H + hh) * R + k];
                }
            }
            // ---------------- phase 2: column pass, Q += X^T p --------------
            if constexpr (MC) {
                // lane (lr, lq) supplies A[lr][lq] = x[row 4 s + lq][column 16 t + lr]
                // and B[lq][lr] = p[row 4 s + lq][rank lr]; it receives
                // Q[column 16 t + 4 lq + e][rank lr]
                const int lr = lane & 15, lq = lane >> 4;
                const int tpw = W / (16 * NW);
                const float* xb = reinterpret_cast<const float*>(Xs) + (size_t)buf * H * XP + wave * tpw * 16 + lr;
                const float* pb = reinterpret_cast<const float*>(Ps) + (size_t)buf * H * R;
                for (int s4 = 0; s4 < H; s4 += 4) {
                    const float bv = (lr < R) ? pb[(s4 + lq) * R + lr] : 0.f;
                    const float* xr = xb + (size_t)(s4 + lq) * XP;
#pragma unroll
                    for (int t = 0; t < MT; ++t)
                        if (t < tpw) qm[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xr[16 * t], bv, qm[t], 0, 0, 0);
                }
            } else if (W >= TPB) {
                for (int hh = 0; hh < H; ++hh) {
                    const T* xr = Xs + ((size_t)buf * H + hh) * W;
                    T pk[R];
#pragma unroll
                    for (int k = 0; k < R; ++k) pk[k] = Ps[((size_t)buf * H + hh) * R + k];
#pragma unroll
                    for (int e = 0; e < CPT2MAX; ++e) {
                        const int col = tid + e * TPB;
                        if (e < cpt2 && col < W) {
                            const T xv = xr[col];
#pragma unroll
                            for (int k = 0; k < R; ++k) Qacc[e][k] = fma(xv, pk[k], Qacc[e][k]);
                        }
                    }
                }
            } else {
                const int col = tid % W, grp = tid / W;
                if (grp < HG) {
                    for (int hh = grp; hh < H; hh += HG) {
                        const T xv = Xs[((size_t)buf * H + hh) * W + col];
#pragma unroll
                        for (int k = 0; k < R; ++k)
                            Qacc[0][k] = fma(xv, Ps[((size_t)buf * H + hh) * R + k], Qacc[0][k]);
                    }
                }
            }
            __syncthreads();
        }
    }

    // ---------------- write the column partials of this cluster -----------
    if constexpr (MC) {
        const int lr = lane & 15, lq = lane >> 4;
        const int tpw = W / (16 * NW);
        if (lr < R) {
#pragma unroll
            for (int t = 0; t < MT; ++t) {
                if (t < tpw) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int jcol = c0 + (wave * tpw + t) * 16 + 4 * lq + e;
                        if (jcol < n) a.Qpart[((size_t)cl * n + jcol) * R + lr] = qm[t][e];
                    }
                }
            }
        }
    } else if (W >= TPB) {
#pragma unroll
        for (int e = 0; e < CPT2MAX; ++e) {
            const int col = tid + e * TPB;
            const int jcol = c0 + col;
            if (e < cpt2 && col < W && jcol < n) {
#pragma unroll
                for (int k = 0; k < R; ++k) a.Qpart[((size_t)cl * n + jcol) * R + k] = Qacc[e][k];
            }
        }
    } else {
        const int col = tid % W, grp = tid / W;
        if (grp < HG) {
#pragma unroll
            for (int k = 0; k < R; ++k) Qred[((size_t)grp * W + col) * R + k] = Qacc[0][k];
        }
        __syncthreads();
        for (int e = tid; e < W * R; e += TPB) {
            const int colx = e / R, k = e % R;
            T s = 0;
            for (int gg = 0; gg < HG; ++gg) s += Qred[((size_t)gg * W + colx) * R + k];
            const int jcol = c0 + colx;
            if (jcol < n) a.Qpart[((size_t)cl * n + jcol) * R + k] = s;
        }
    }
    // ---------------- ||Y_k - Y_{k-1}||^2 (or ||M||^2) partial ------------
    acc2 = group_sum(acc2, 64);
    if (lane == 0) red[wave] = acc2;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) t += red[w];
        a.dy2part[g] = t;
    }
}

#define SFR_R_LIST(X) X(1) X(2) X(3) X(4) X(5) X(6) X(8) X(10) X(12) X(16) X(20) X(24) X(32)

// Kernel of rank bucket R; MC: the matrix-core column pass (FP32, R <= 10).
template <typename T, int R>
static void* sweep_fn_r(bool mc)
{
    if constexpr (sizeof(T) == 4 && R <= 10) {
        if (mc) return reinterpret_cast<void*>(&sweep_kernel<T, R, true>);
    }
    return reinterpret_cast<void*>(&sweep_kernel<T, R, false>);
}

template <typename T>
size_t sweep_lds_bytes_c(int R, int lpr, int W, int c)
{
    return sweep_lds<T>(R, lpr, W, c, sweep_threads<T>(R)).total;
}

template <typename T>
int sweep_threads(int R)
{
    switch (R) {
#define CASE(r) case r: return sweep_tpb<T, r>();
        SFR_R_LIST(CASE)
#undef CASE
    default: return 0;
    }
}

template <typename T>
int sweep_max_width(int R)
{
    switch (R) {
#define CASE(r) case r: return sweep_cpt2<T, r>() * sweep_tpb<T, r>();
        SFR_R_LIST(CASE)
#undef CASE
    default: return 0;
    }
}

template <typename T>
static void* sweep_fn(int R, bool mc)
{
    switch (R) {
#define CASE(r) case r: return sweep_fn_r<T, r>(mc);
        SFR_R_LIST(CASE)
#undef CASE
    default: return nullptr;
    }
}

template <typename T, int R, bool MC>
static hipError_t launch_sweep_r(const SweepArgs<T>& a, int grid, size_t lds, hipStream_t s, hipEvent_t ev0,
                                 hipEvent_t ev1)
{
    if (ev0)
        hipExtLaunchKernelGGL((sweep_kernel<T, R, MC>), dim3(grid), dim3(sweep_tpb<T, R>()), (uint32_t)lds, s, ev0,
                              ev1, 0u, a);
    else
        hipLaunchKernelGGL((sweep_kernel<T, R, MC>), dim3(grid), dim3(sweep_tpb<T, R>()), lds, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sweep(const SweepArgs<T>& a, int R, int grid, size_t lds, hipStream_t s, hipEvent_t ev0,
                        hipEvent_t ev1)
{
    switch (R) {
#define CASE(r)                                                                                   \
    case r:                                                                                       \
        if constexpr (sizeof(T) == 4 && r <= 10) {                                                \
            if (sweep_mcol<T>(r, a.lpr, a.W, sweep_tpb<T, r>()))                                  \
                return launch_sweep_r<T, r, true>(a, grid, lds, s, ev0, ev1);                     \
        }                                                                                         \
        return launch_sweep_r<T, r, false>(a, grid, lds, s, ev0, ev1);
        SFR_R_LIST(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t sweep_prepare(int R, int lpr, int W, size_t lds, int* blocks_per_cu)
{
    void* fn = sweep_fn<T>(R, sweep_mcol<T>(R, lpr, W, sweep_threads<T>(R)));
    if (!fn) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, sweep_threads<T>(R), lds);
}

template hipError_t launch_sweep<float>(const SweepArgs<float>&, int, int, size_t, hipStream_t, hipEvent_t,
                                        hipEvent_t);
template hipError_t launch_sweep<double>(const SweepArgs<double>&, int, int, size_t, hipStream_t, hipEvent_t,
                                         hipEvent_t);
template size_t sweep_lds_bytes_c<float>(int, int, int, int);
template size_t sweep_lds_bytes_c<double>(int, int, int, int);
template int sweep_threads<float>(int);
template int sweep_threads<double>(int);
template int sweep_max_width<float>(int);
template int sweep_max_width<double>(int);
template hipError_t sweep_prepare<float>(int, int, int, size_t, int*);
template hipError_t sweep_prepare<double>(int, int, int, size_t, int*);

}  // namespace sfr
