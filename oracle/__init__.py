"""FP64 CPU oracle of the S-FR decomposition -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper over `sfr_oracle.c` (plain C, one thread, FP64).  Only
tests/, ``__graft_entry__.smoke()`` and bench.py's ``cpu_baseline`` leg may
import this package; the HIP library never does, and this package never
imports the HIP library.

Every routine follows the paper's definitions (Alg. 1-4, eq. (7), eq. (8),
the notation section); the readings taken where the paper is silent are
listed in the C source header.  Parity status of each function:

  soft_threshold, sym, svd_jacobi, polar, pinv_rank, fr_step, fr_full,
  fradm_iter, fradm, frnys, frnys_blocks, nys_entries -- all pinned by
  tests/test_oracle_pins.py (closed forms, LAPACK special cases, invariants
  of Lemma 1/2 and Theorems 1/2, brute force on tiny inputs).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sfr_oracle.c")
_LIB = os.path.join(_HERE, "libsfr_oracle.so")

ORC_OK, ORC_RANK, ORC_MAXITER = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2 -ffp-contract=off, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def load(path: str):
    """Open a compiled oracle library and declare its C signatures."""
    L = ctypes.CDLL(path)
    d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int32
    pd = ctypes.POINTER(ctypes.c_double)
    pi32 = ctypes.POINTER(ctypes.c_int32)
    pi64 = ctypes.POINTER(ctypes.c_int64)
    L.orc_soft_threshold.argtypes = [pd, i64, d, pd]
    L.orc_sym.argtypes = [pd, i64, pd]
    L.orc_svd_jacobi.argtypes = [pd, i64, i64, pd, pd, pd]
    L.orc_polar.argtypes = [pd, i64, i64, pd]
    L.orc_pinv_rank.argtypes = [pd, i64, i64, pd]
    L.orc_fr_step.argtypes = [pd, i64, i64, i64, pd, pd, pd, pd, pd]
    L.orc_fr_full.argtypes = [pd, i64, i64, i64, i32, pd, pd, pd]
    L.orc_fradm_init.argtypes = [i64, i64, i64, pd, pd, pd, pd, pd]
    L.orc_fradm_init.restype = None
    L.orc_fradm_iter.argtypes = [pd, i64, i64, i64, d, pd, d, d, d, pd, pd, pd, pd, pd, pd, pd]
    L.orc_fradm.argtypes = [pd, i64, i64, i64, d, d, d, d, d, i32, i32,
                            pd, pd, pd, pd, pd, pi32, pd, pd]
    L.orc_frnys.argtypes = [pd, i64, i64, i64, i64, pi64, d, d, d, d, d, d, i32, i32,
                            pd, pd, pd, pd, pd, pi32, pi32]
    L.orc_frnys_blocks.argtypes = [pd, pd, i64, i64, i64, i64, d, d, d, d, d, d, i32, i32,
                                   pd, pd, pd, pi32, pi32]
    L.orc_nys_entries.argtypes = [pd, pd, pd, i64, i64, pi64, pi64, i64, pd]
    L.orc_nys_entries.restype = None
    L.orc_soft_threshold.restype = None
    L.orc_sym.restype = None
    for f in ("orc_svd_jacobi", "orc_polar", "orc_pinv_rank", "orc_fr_step", "orc_fr_full",
              "orc_fradm_iter", "orc_fradm", "orc_frnys", "orc_frnys_blocks"):
        getattr(L, f).restype = ctypes.c_int
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = load(_LIB)
    return _lib


def _d(a):
    """C-contiguous float64 view/copy and its pointer."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def soft_threshold(x, t):
    x, px = _d(x)
    y = np.empty_like(x)
    lib().orc_soft_threshold(px, x.size, float(t), _p(y))
    return y


def sym(A):
    A, pa = _d(A)
    out = np.empty_like(A)
    lib().orc_sym(pa, A.shape[0], _p(out))
    return out


def svd_jacobi(A):
    """Thin SVD A = W diag(sig) Z^T (unsorted); returns (W, sig, Z, sweeps)."""
    A, pa = _d(A)
    m, k = A.shape
    W = np.empty((m, k)); sig = np.empty(k); Z = np.empty((k, k))
    sw = lib().orc_svd_jacobi(pa, m, k, _p(W), _p(sig), _p(Z))
    return W, sig, Z, sw


def polar(A):
    """P_O[A] of eq. (7); returns (out, rc)."""
    A, pa = _d(A)
    m, k = A.shape
    out = np.empty((m, k))
    rc = lib().orc_polar(pa, m, k, _p(out))
    return out, rc


def pinv_rank(W, r):
    W, pw = _d(W)
    out = np.empty_like(W)
    rc = lib().orc_pinv_rank(pw, W.shape[0], r, _p(out))
    return out, rc


def fr_step(X, B0, V0):
    """FixedRankOptStep (Alg. 2); returns (U, B, V, rc)."""
    X, px = _d(X)
    B0, pb = _d(B0)
    V0, pv = _d(V0)
    m, n = X.shape
    r = B0.shape[0]
    U = np.empty((m, r)); B = np.empty((r, r)); V = np.empty((n, r))
    rc = lib().orc_fr_step(px, m, n, r, pb, pv, _p(U), _p(B), _p(V))
    return U, B, V, rc


def fr_full(X, U, B, V, iters):
    """FixedRankOptFull (Alg. 4): `iters` steps; returns (U, B, V, rc)."""
    X, px = _d(X)
    U = np.array(U, dtype=np.float64, order="C")
    B = np.array(B, dtype=np.float64, order="C")
    V = np.array(V, dtype=np.float64, order="C")
    m, n = X.shape
    rc = lib().orc_fr_full(px, m, n, B.shape[0], int(iters), _p(U), _p(B), _p(V))
    return U, B, V, rc


class FradmState:
    """Explicit Alg. 1 state for stepping one iteration at a time."""

    def __init__(self, M, r, lam, mu0, rho=1.5, mu_bar=1e9):
        self.M, _ = _d(M)
        m, n = self.M.shape
        self.m, self.n, self.r = m, n, r
        self.lam, self.rho, self.mu_bar = float(lam), float(rho), float(mu_bar)
        self.mu = ctypes.c_double(float(mu0))
        self.S = np.zeros((m, n)); self.Y = np.zeros((m, n))
        self.U = np.zeros((m, r)); self.B = np.zeros((r, r)); self.V = np.zeros((n, r))
        lib().orc_fradm_init(m, n, r, _p(self.S), _p(self.Y), _p(self.U), _p(self.B), _p(self.V))
        self.nrmM = float(np.sqrt(np.sum(self.M * self.M)))
        self.L = np.zeros((m, n))
        self.k = 0

    def step(self):
        """One iteration of Alg. 1; returns (res, rc).  self.mu afterwards
        holds mu_{k+1}; mu_k used by the step is returned in `mu_used`."""
        res = ctypes.c_double(0.0)
        self.mu_used = self.mu.value
        rc = lib().orc_fradm_iter(_p(self.M), self.m, self.n, self.r, self.lam,
                                  ctypes.byref(self.mu), self.rho, self.mu_bar, self.nrmM,
                                  _p(self.S), _p(self.Y), _p(self.U), _p(self.B), _p(self.V),
                                  _p(self.L), ctypes.byref(res))
        self.k += 1
        return res.value, rc


def fradm(M, r, lam, mu0, rho=1.5, mu_bar=1e9, tol=1e-7, max_iter=300, fixed_iters=0,
          want_Y=False):
    """Full FR-ADM solve (Alg. 1).  Returns dict(U, B, V, S, Y, iters, res,
    res_hist, rc)."""
    M, pm = _d(M)
    m, n = M.shape
    U = np.empty((m, r)); B = np.empty((r, r)); V = np.empty((n, r)); S = np.empty((m, n))
    Y = np.empty((m, n)) if want_Y else None
    it = ctypes.c_int32(0)
    res = ctypes.c_double(0.0)
    hist = np.full(max(max_iter, fixed_iters, 1), np.nan)
    rc = lib().orc_fradm(pm, m, n, r, float(lam), float(mu0), float(rho), float(mu_bar),
                         float(tol), int(max_iter), int(fixed_iters), _p(U), _p(B), _p(V), _p(S),
                         _p(Y) if want_Y else None, ctypes.byref(it), ctypes.byref(res), _p(hist))
    return dict(U=U, B=B, V=V, S=S, Y=Y, iters=it.value, res=res.value,
                res_hist=hist[: it.value].copy(), rc=rc)


def frnys(M, r, l, perm, lam, mu0_left, mu0_top, rho=1.5, mu_bar=1e9, tol=1e-7, max_iter=300,
          fixed_iters=0, want_dense=True):
    """FR-Nys (Alg. 3) with the given row shuffle.  Returns dict(LL, Wp, LT,
    L, S, iters_left, iters_top, rc); L, S in M's own row order."""
    M, pm = _d(M)
    m, n = M.shape
    perm = np.ascontiguousarray(perm, dtype=np.int64)
    LL = np.empty((m, l)); Wp = np.empty((l, l)); LT = np.empty((l, n))
    L = np.empty((m, n)) if want_dense else None
    S = np.empty((m, n)) if want_dense else None
    il = ctypes.c_int32(0); itp = ctypes.c_int32(0)
    rc = lib().orc_frnys(pm, m, n, r, l, perm.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                         float(lam), float(mu0_left), float(mu0_top), float(rho), float(mu_bar),
                         float(tol), int(max_iter), int(fixed_iters), _p(LL), _p(Wp), _p(LT),
                         _p(L) if want_dense else None, _p(S) if want_dense else None,
                         ctypes.byref(il), ctypes.byref(itp))
    return dict(LL=LL, Wp=Wp, LT=LT, L=L, S=S, iters_left=il.value, iters_top=itp.value, rc=rc)


def frnys_blocks(C, Rb, r, lam, mu0_left, mu0_top, rho=1.5, mu_bar=1e9, tol=1e-7, max_iter=300,
                 fixed_iters=0):
    """Alg. 3 from the two gathered blocks C = Mt[:, :l], Rb = Mt[:l, :]."""
    C, pc = _d(C)
    Rb, pr = _d(Rb)
    m, l = C.shape
    n = Rb.shape[1]
    LL = np.empty((m, l)); Wp = np.empty((l, l)); LT = np.empty((l, n))
    il = ctypes.c_int32(0); itp = ctypes.c_int32(0)
    rc = lib().orc_frnys_blocks(pc, pr, m, n, r, l, float(lam), float(mu0_left), float(mu0_top),
                                float(rho), float(mu_bar), float(tol), int(max_iter),
                                int(fixed_iters), _p(LL), _p(Wp), _p(LT),
                                ctypes.byref(il), ctypes.byref(itp))
    return dict(LL=LL, Wp=Wp, LT=LT, iters_left=il.value, iters_top=itp.value, rc=rc)


def nys_entries(LL, Wp, LT, si, sj):
    """Entries (si, sj) of the shuffled-order Nystrom L = L_L Wp L_T."""
    LL, pa = _d(LL)
    Wp, pb = _d(Wp)
    LT, pc = _d(LT)
    si = np.ascontiguousarray(si, dtype=np.int64)
    sj = np.ascontiguousarray(sj, dtype=np.int64)
    out = np.empty(si.size)
    P64 = ctypes.POINTER(ctypes.c_int64)
    lib().orc_nys_entries(pa, pb, pc, LT.shape[1], LL.shape[1], si.ctypes.data_as(P64),
                          sj.ctypes.data_as(P64), si.size, _p(out))
    return out
