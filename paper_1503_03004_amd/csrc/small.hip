// FP64 r x r algebra of one FR-ADM iteration, on the device.
//
// Given the Grams G_P = P^T P, G_Q = Q^T Q of the sweep and the previous
// SPD factor B0, the closed-form projectors of Sec. 4.1 become
//   C1 = (B0 G_P B0)^{-1/2}            U  = P B0 C1          (eq. (7))
//   K  = B0 C1 B0,  C2 = (K G_Q K)^{-1/2}, V = Q K C2         (eq. (7))
//   B  = Sym(C1 B0 G_Q K C2)                                  (eq. (8))
// and the next sweep rebuilds L rows as a_i = P_i (B0 C1 B).
//
// The products run on the matrix cores and the inverse square roots by
// Newton-Schulz (small_ns.hpp); Gram products too ill-conditioned for its
// accuracy take the warm-started Jacobi eigendecompositions of small_la.hpp
// (the eigenbases of the last such step are kept in the state).  The
// smallest rank buckets take the Jacobi route directly, with the matrices in
// registers up to R = 3 (small_reg.hpp).
#include "small_ns.hpp"
#include "small_reg.hpp"

namespace sfr {

// Rank buckets up to this take the Jacobi route directly (the step's
// Newton-Schulz products cost the same 16 x 16 tiles at every rank).
constexpr int kStepJacobiMaxR = 4;
// Rank buckets up to this run that route in registers (small_reg.hpp); at
// R = 4 the copies of the matrices no longer fit a lane's registers.
constexpr int kStepRegMaxR = 3;

// LDS of the step kernel: 14 RT x LDP matrices, the two Gram triangles and
// their segment sums, the residual wave sums, the reduction slots and the
// Jacobi scratch.
struct StepLds {
    size_t mats, tri, seg, red, cs, wbuf, total;
};
__host__ __device__ inline StepLds step_lds(int R)
{
    const int RT = R <= 16 ? 16 : 32;
    const int E = R * (R + 1) / 2;
    StepLds L;
    size_t o = 0;
    L.mats = o; o += sizeof(double) * 14 * (size_t)RT * LDP;
    L.tri = o;  o += sizeof(double) * 2 * (size_t)E;
    L.seg = o;  o += sizeof(double) * (size_t)(2 * E > kStepTPB ? 2 * E : kStepTPB);
    L.red = o;  o += sizeof(double) * (kStepTPB / 64 + 12);
    L.cs = o;   o += sizeof(double) * 2 * 16;
    L.wbuf = o; o += sizeof(double) * kMaxR;
    L.total = o;
    return L;
}

// The r x r matrices are held RT x RT (RT = 16 or 32 >= R, the rank
// bucket) with an identity block on the padded indices: every product and
// inverse square root is then block diagonal and exact on the leading r x r
// block, and the padded block is dropped when the transforms are stored.
template <int R>
__global__ void __launch_bounds__(kStepTPB) step_kernel(StepArgs a)
{
    constexpr int NB = ns_nb<R>();
    constexpr int RT = 16 * NB;
    constexpr int TPB = kStepTPB;
    // threads of the r x r algebra: one wavefront, or the whole workgroup
    // (four wavefronts compute, the rest take part in the barriers)
    constexpr int NT = (NB == 1) ? 64 : TPB;
    constexpr int E = R * (R + 1) / 2;
    constexpr int MS = RT * LDP;
    extern __shared__ __align__(16) unsigned char smem[];
    const StepLds SL = step_lds(R);
    double* mats = reinterpret_cast<double*>(smem + SL.mats);
    double* Bm = mats;
    double* Gp = mats + 1 * MS;
    double* Gq = mats + 2 * MS;
    double* X = mats + 3 * MS;
    double* Am = mats + 4 * MS;
    double* C = mats + 5 * MS;
    double* Y0 = mats + 6 * MS;
    double* Y1 = mats + 7 * MS;
    double* Z0 = mats + 8 * MS;
    double* Z1 = mats + 9 * MS;
    double* Tm = mats + 10 * MS;
    double* T1 = mats + 11 * MS;
    double* R1 = mats + 12 * MS;
    double* Km = mats + 13 * MS;
    double* tri = reinterpret_cast<double*>(smem + SL.tri);
    double* seg = reinterpret_cast<double*>(smem + SL.seg);
    double* red = reinterpret_cast<double*>(smem + SL.red);
    double* nsred = red + TPB / 64;
    double* cs = reinterpret_cast<double*>(smem + SL.cs);
    double* wbuf = reinterpret_cast<double*>(smem + SL.wbuf);

    DevState* st = a.st;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const NsLane<NB> L;

    // ---- one round of loads: the previous B (the algebra's lanes, their
    // output block), the residual partials and the Gram partials.  Every
    // load is unconditional (indices clamped into range, the surplus masked
    // afterwards), so each thread has its loads in flight together.
    double rb[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) rb[e] = st->B[L.row(e) * kMaxR + L.col()];
    constexpr int DYU = (kMaxDyPartials + TPB - 1) / TPB;
    double dyv[DYU];
#pragma unroll
    for (int u = 0; u < DYU; ++u) dyv[u] = a.dy2part[min(tid + u * TPB, a.ndy - 1)];
    const int32_t done0 = st->done, tmo = st->exch_timeout;
    const int r = st->r, k = st->k, tsvd = st->tsvd;
    const int fixed_iters = st->fixed_iters, max_iter = st->max_iter, stop_after = st->stop_after;
    const double mu = st->mu, mu_prev = st->mu_prev, nrmM = st->nrmM, tol = st->tol;
    const double rho = st->rho, mu_bar = st->mu_bar;
    if (done0) return;
    if (tmo) {   // a sweep hit its wait bound: stop the solve
        if (tid == 0) st->done = 1;
        return;
    }
    // Gram partials of the 2E upper-triangle entries of (G_P, G_Q).  Summed
    // already (one partial each): thread w takes entries w, w + TPB, ...
    // Otherwise thread w owns entry e of one Gram over the partials
    // b = s, s + nseg, ... (segment s), and the segment sums are added in
    // segment order after the barrier.
    const bool summed = a.npb == 1 && a.nqb == 1;
    constexpr int EPT = (2 * E + TPB - 1) / TPB;
    constexpr int nseg = (2 * E >= TPB) ? 1 : TPB / (2 * E);
    constexpr int PER = (kMaxGramPartials + nseg - 1) / nseg;
    constexpr int CH = PER < kStepPartialLoads ? PER : kStepPartialLoads;
    if (summed) {
        double gv[EPT];
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            const int w = min(tid + u * TPB, 2 * E - 1);
            gv[u] = (w < E) ? a.GPpart[w] : a.GQpart[w - E];
        }
#pragma unroll
        for (int u = 0; u < EPT; ++u)
            if (tid + u * TPB < 2 * E) tri[tid + u * TPB] = gv[u];
    } else {
        for (int w = tid; w < 2 * E * nseg; w += TPB) {
            const int g = w / (E * nseg), rem = w % (E * nseg);
            const int sg = rem / E, e = rem % E;
            const double* part = g ? a.GQpart : a.GPpart;
            const int count = g ? a.nqb : a.npb;
            double sum = 0.0;
            for (int u0 = 0; u0 * nseg < count; u0 += CH) {
                double v[CH];
#pragma unroll
                for (int u = 0; u < CH; ++u) v[u] = part[(size_t)min(sg + (u0 + u) * nseg, count - 1) * E + e];
#pragma unroll
                for (int u = 0; u < CH; ++u) sum += (sg + (u0 + u) * nseg < count) ? v[u] : 0.0;
            }
            seg[w] = sum;
        }
    }

    // ---- convergence test of iteration k-1 (or ||M||_F on the first pass)
    double part = 0.0;
#pragma unroll
    for (int u = 0; u < DYU; ++u) part += (tid + u * TPB < a.ndy) ? dyv[u] : 0.0;
    for (int e = tid + DYU * TPB; e < a.ndy; e += TPB) part += a.dy2part[e];
    part = wave_sum(part);
    if (lane == 0) red[wave] = part;
    __syncthreads();
    double total = 0.0;
#pragma unroll
    for (int w = 0; w < TPB / 64; ++w) total += red[w];
    if (k == 1) {
        const double nrm = sqrt(total);
        if (!(nrm > 0.0) || !isfinite(nrm)) {
            if (tid == 0) { st->nrmM = nrm; st->status = kErrNonFinite; st->iters = 0; st->done = 1; }
            return;
        }
        if (tid == 0) st->nrmM = nrm;
    } else if (!tsvd) {
        const double res = sqrt(total) / (mu_prev * nrmM);
        const int kdone = k - 1;
        bool stop = false;
        int32_t status = kOK;
        if (!isfinite(res)) { stop = true; status = kErrNonFinite; }
        else if (fixed_iters > 0) { stop = kdone >= fixed_iters; }
        else if (res <= tol) { stop = true; }
        else if (kdone >= max_iter) { stop = true; status = kWarnMaxIter; }
        if (tid == 0) {
            a.res_hist[kdone - 1] = res;
            st->res = res;
        }
        if (stop) {
            if (tid == 0) { st->status = status; st->iters = kdone; st->done = 1; }
            return;
        }
    }

    // ---- B_0, G_P and G_Q into LDS, identity on the padded indices
    if (!summed) {
        for (int w = tid; w < 2 * E; w += TPB) {
            const int g = w / E, e = w % E;
            double sum = 0.0;
#pragma unroll
            for (int sg = 0; sg < nseg; ++sg) sum += seg[(g * nseg + sg) * E + e];
            tri[w] = sum;
        }
        __syncthreads();
    }
    if (L.act) {
#pragma unroll
        for (int e = 0; e < 4; ++e) Bm[L.row(e) * LDP + L.col()] = rb[e];
    }
    for (int e = tid; e < 2 * RT * RT; e += TPB) {
        const int g = e / (RT * RT), ij = e % (RT * RT);
        const int i = ij / RT, j = ij % RT;
        const int x = i < j ? i : j, y = i < j ? j : i;
        double v = (i == j) ? 1.0 : 0.0;
        if (i < r && j < r) v = tri[g * E + x * R - x * (x - 1) / 2 + (y - x)];
        (g ? Gq : Gp)[i * LDP + j] = v;
    }
    __syncthreads();
    if constexpr (NB == 1) {
        if (wave != 0) return;
    }

    // ---- the r x r algebra: Newton-Schulz, else the warm-started Jacobi
    // path (which also decides rank loss); outputs left in LDS
    const double *oB, *oTU, *oTUbar, *oTV;
    // Newton-Schulz works on 16 x 16 tiles whatever the rank; up to
    // kStepJacobiMaxR the warm-started eigendecompositions of the R x R
    // Grams are the cheaper route (262144 x 48, r = 3: 13 against 28 us)
    bool use_ns = false;
    if constexpr (R > kStepJacobiMaxR && NB == 1) {
        // one wavefront, every matrix in registers; the outputs go to LDS at
        // the lane's own entries, which the stores below read back
        f64x4 bn, tu, tub, tv;
        f64x4 b0 = {rb[0], rb[1], rb[2], rb[3]};
        use_ns = ns1_lstep(b0, Gp, Gq, X, r, a.ns_kappa, bn, tu, tub, tv);
        if (use_ns) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int li = L.row(e) * LDP + L.col();
                Y0[li] = bn[e];
                Am[li] = tu[e];
                T1[li] = tub[e];
                C[li] = tv[e];
            }
        }
    } else if constexpr (R > kStepJacobiMaxR) {
        use_ns = ns_lstep<R>(Bm, Gp, Gq, X, Am, C, Y0, Y1, Z0, Z1, Tm, T1, R1, Km, nsred, r, a.ns_kappa);
    }
    if (use_ns) {
        oB = Y0; oTU = Am; oTUbar = T1; oTV = (NB == 1) ? C : Gp;
    } else if constexpr (R <= kStepRegMaxR) {
        // the warm-started Jacobi route with every lane holding the whole
        // step in registers (small_reg.hpp); the eigenbases of the last step
        // (identity at the start of a solve) come from the state
        RMat<R> rGp, rGq, rB0, rE1, rE2;
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
            for (int j = 0; j < R; ++j) {
                rGp.v[i][j] = Gp[i * LDP + j];
                rGq.v[i][j] = Gq[i * LDP + j];
                rB0.v[i][j] = Bm[i * LDP + j];
                rE1.v[i][j] = st->E1[i * kMaxR + j];
                rE2.v[i][j] = st->E2[i * kMaxR + j];
            }
        RMat<R> rB, rTU, rTUbar, rTV;
        if (!rm_lstep<R>(rGp, rGq, rB0, rE1, rE2, r, a.dk_tau, rB, rTU, rTUbar, rTV)) {
            if (tid == 0) { st->status = kErrRank; st->iters = k - 1; st->done = 1; }
            return;
        }
        // lane i R + j publishes entry (i, j) of the outputs (every lane holds them all)
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
            for (int j = 0; j < R; ++j)
                if (lane == i * R + j) {
                    Z0[i * LDP + j] = rB.v[i][j];
                    Km[i * LDP + j] = rTU.v[i][j];
                    T1[i * LDP + j] = rTUbar.v[i][j];
                    Gp[i * LDP + j] = rTV.v[i][j];
                    st->E1[i * kMaxR + j] = rE1.v[i][j];
                    st->E2[i * kMaxR + j] = rE2.v[i][j];
                }
        wsync();
        oB = Z0; oTU = Km; oTUbar = T1; oTV = Gp;
    } else {
        // eigenbases of the last Jacobi step (identity at the start of a
        // solve) into Z1 and Tm
        const int t = lid<NT>();
        for (int e = t; e < R * R; e += NT) {
            const int i = e / R, j = e % R;
            Z1[i * LDP + j] = st->E1[i * kMaxR + j];
            Tm[i * LDP + j] = st->E2[i * kMaxR + j];
        }
        lsync<NT>();
        // C1 -> C, C2 -> Y1, T2 (the new B) -> Z0
        if (!lstep_algebra<R, NT>(Gp, Gq, Bm, C, Y1, Km, T1, Z0, Z1, Tm, cs, wbuf, r, a.dk_tau)) {
            if (tid == 0) { st->status = kErrRank; st->iters = k - 1; st->done = 1; }
            return;
        }
        for (int e = t; e < R * R; e += NT) {
            const int i = e / R, j = e % R;
            st->E1[i * kMaxR + j] = Z1[i * LDP + j];
            st->E2[i * kMaxR + j] = Tm[i * LDP + j];
        }
        oB = Z0; oTU = Km; oTUbar = T1; oTV = Gp;
    }
    // ---- the transforms: only the R x R block changes; the rest keeps the
    // values set at the start of the solve (zero, identity on the diagonal of B)
    double d2 = 0.0, n2 = 0.0;
    if (L.act) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int i = L.row(e), j = L.col();
            if (i >= R || j >= R) continue;
            const int gi = i * kMaxR + j, li = i * LDP + j;
            const bool in = (i < r) && (j < r);
            const double bn = oB[li];
            const double tv = in ? oTV[li] : 0.0;
            const double tub = in ? oTUbar[li] : 0.0;
            const double tuv = in ? oTU[li] : 0.0;
            st->B[gi] = in ? bn : (i == j ? 1.0 : 0.0);
            st->TU[gi] = tuv;
            st->TUbar[gi] = tub;
            st->TV[gi] = tv;
            st->TUf[gi] = (float)tuv;
            st->TVf[gi] = (float)tv;
            if (in) {
                const double bo = Bm[li];
                d2 = fma(bn - bo, bn - bo, d2);
                n2 = fma(bn, bn, n2);
            }
        }
    }
    if (tsvd) {
        // Alg. 4 stops after this step once B has settled:
        // ||B_k - B_{k-1}||_F <= tol ||B_k||_F (or after fixed_iters steps)
        d2 = ns_sum<NB>(d2, nsred);
        n2 = ns_sum<NB>(n2, nsred + 4);
        const double res = sqrt(d2 / n2);
        bool stop = false;
        int32_t status = kOK;
        if (!isfinite(res)) { stop = true; status = kErrNonFinite; }
        else if (fixed_iters > 0) { stop = k >= fixed_iters; }
        else if (res <= tol) { stop = true; }
        else if (k >= max_iter) { stop = true; status = kWarnMaxIter; }
        if (tid == 0) {
            a.res_hist[k - 1] = res;
            st->res = res;
            st->k = k + 1;
            if (stop) { st->status = status; st->iters = k; st->done = 1; }
        }
        return;
    }
    if (tid == 0) {
        st->mu_prev = mu;
        const double nm = rho * mu;
        st->mu = nm < mu_bar ? nm : mu_bar;
        st->k = k + 1;
        // a fixed-count solve ends with this step: its returned iterate is
        // iteration k, whose residual the S pass takes
        if (stop_after > 0 && k >= stop_after) {
            st->iters = k;
            st->done = 1;
        }
    }
}

// Smallest eigenvalue of the returned B (is it in SPD_r?  Appendix, Lemma 2).
template <int R>
__global__ void __launch_bounds__(64) final_small_kernel(DevState* st)
{
    __shared__ double A[R * LDP], Ev[R * LDP];
    __shared__ __align__(16) double cs[2 * 16];
    const double w = wmin_eig<R>(st->B, kMaxR, st->r, A, Ev, cs);
    if (threadIdx.x == 0) st->min_eig_B = w;
}

// Largest eigenvalue of the returned B.  After Alg. 4 on M, B has the r
// leading singular values of M as its eigenvalues (Theorem 2), so this is
// ||M||_2 (full Jacobi convergence from the identity basis).
template <int R>
__global__ void __launch_bounds__(64) max_eig_kernel(DevState* st)
{
    __shared__ double A[R * LDP], Ev[R * LDP];
    __shared__ __align__(16) double cs[2 * 16];
    const int lane = threadIdx.x;
    const int r = st->r;
    for (int e = lane; e < R * R; e += 64) {
        const int i = e / R, j = e % R;
        const bool pad = (i >= r) || (j >= r);
        A[i * LDP + j] = pad ? (i == j ? 1.0 : 0.0) : st->B[i * kMaxR + j];
        Ev[i * LDP + j] = (i == j) ? 1.0 : 0.0;
    }
    lsync<64>();
    wjacobi<R, 64>(A, Ev, cs);
    if (lane == 0) {
        double w = -INFINITY;
        for (int i = 0; i < r; ++i) w = fmax(w, A[i * LDP + i]);
        st->max_eig_B = w;
    }
}

#define SFR_R_LIST(X) X(1) X(2) X(3) X(4) X(5) X(6) X(8) X(10) X(12) X(16) X(20) X(24) X(32)

hipError_t launch_step(const StepArgs& a, int R, hipStream_t s)
{
    const size_t lds = step_lds(R).total;
    switch (R) {
#define CASE(rr) case rr: hipLaunchKernelGGL(step_kernel<rr>, dim3(1), dim3(kStepTPB), lds, s, a); break;
        SFR_R_LIST(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t step_prepare(int R)
{
    const int lds = (int)step_lds(R).total;
    switch (R) {
#define CASE(rr) \
    case rr: return hipFuncSetAttribute(reinterpret_cast<const void*>(&step_kernel<rr>), hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        SFR_R_LIST(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
    }
}

// Continue a stopped solve from its returned iterate K (the second phase of
// a BF16 solve): every buffer of iterate K (Y_K, P_K, Q_K) and the state of
// its step (transforms, B, mu) are intact, so this only
// installs the new stopping rule, clears the stop and sets the next sweep to
// K + 1.  A solve that stopped with an error, or with no iterations left in
// the new rule, stays stopped.
__global__ void refine_start_kernel(DevState* st, int fixed_iters, double tol, int max_iter)
{
    if (threadIdx.x != 0) return;
    if (!st->done || st->status < 0 || st->exch_timeout) return;
    const int K = st->iters;
    if (K >= (fixed_iters > 0 ? fixed_iters : max_iter)) return;
    st->status = kOK;
    st->fixed_iters = fixed_iters;
    st->tol = tol;
    st->max_iter = max_iter;
    st->k = K + 1;
    st->done = 0;
}

hipError_t launch_refine_start(DevState* st, int fixed_iters, double tol, int max_iter, hipStream_t s)
{
    hipLaunchKernelGGL(refine_start_kernel, dim3(1), dim3(64), 0, s, st, fixed_iters, tol, max_iter);
    return hipGetLastError();
}

hipError_t launch_max_eig(DevState* st, int R, hipStream_t s)
{
    switch (R) {
#define CASE(rr) case rr: hipLaunchKernelGGL(max_eig_kernel<rr>, dim3(1), dim3(64), 0, s, st); break;
        SFR_R_LIST(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_final_small(DevState* st, int R, hipStream_t s)
{
    switch (R) {
#define CASE(rr) case rr: hipLaunchKernelGGL(final_small_kernel<rr>, dim3(1), dim3(64), 0, s, st); break;
        SFR_R_LIST(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace sfr
