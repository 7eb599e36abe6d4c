"""ctypes binding of libsfr.so (argument marshalling only).

Every step of the decomposition runs in the HIP library; PyTorch only
provides device memory and the stream.  The binding refuses to run if the
library has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsfr.so")

SFR_OK = 0
SFR_ERR_ARG = -1
SFR_ERR_NOMEM = -2
SFR_ERR_DEVICE = -3
SFR_ERR_RANK = -4
SFR_ERR_NONFINITE = -5
SFR_ERR_HANDLE = -6
SFR_ERR_SCRATCH = -7
SFR_ERR_BUSY = -8
SFR_WARN_MAXITER = 1
SFR_WARN_NOT_SPD = 2

SFR_F64 = 0
SFR_F32 = 1


class sfr_options(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("precision", ctypes.c_int32),
        ("rho", ctypes.c_double),
        ("mu_bar", ctypes.c_double),
        ("max_iter", ctypes.c_int32),
        ("fixed_iters", ctypes.c_int32),
        ("nystrom_l", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("mu_left", ctypes.c_double),
        ("mu_top", ctypes.c_double),
        ("bf16", ctypes.c_int32),
        ("bf16_iters", ctypes.c_int32),
        ("bf16_tol", ctypes.c_double),
    ]


class sfr_info(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("iters_top", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("reserved0", ctypes.c_int32),
        ("rel_residual", ctypes.c_double),
        ("min_eig_B", ctypes.c_double),
        ("mu_final", ctypes.c_double),
        ("sweep_ms", ctypes.c_double),
        ("sweeps_timed", ctypes.c_int32),
        ("reserved1", ctypes.c_int32),
        ("mu0", ctypes.c_double),
        ("orth_err", ctypes.c_double),
    ]


class sfr_batch_item(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64),
        ("n", ctypes.c_int64),
        ("r", ctypes.c_int32),
        ("reserved0", ctypes.c_int32),
        ("lam", ctypes.c_double),
        ("mu", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("M", ctypes.c_void_p),
        ("ldm", ctypes.c_int64),
        ("U", ctypes.c_void_p),
        ("B", ctypes.c_void_p),
        ("V", ctypes.c_void_p),
        ("S", ctypes.c_void_p),
        ("lds", ctypes.c_int64),
    ]


class SFRError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {status_string(code)} (status {code})")


_lib = None


def lib():
    """Load libsfr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                              "(python -c 'import __graft_entry__ as g; g.build()')")
        # torch first: the library then binds to the HIP runtime torch loaded
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.sfr_create.argtypes = [ctypes.POINTER(vp), i64, i64, i32, d, d, d, ctypes.POINTER(sfr_options)]
        L.sfr_create.restype = ctypes.c_int
        L.sfr_solve.argtypes = [vp, vp, i64, vp, vp, vp, vp, i64, ctypes.POINTER(sfr_info), vp]
        L.sfr_solve.restype = ctypes.c_int
        L.sfr_solve_nys.argtypes = [vp, vp, i64, ctypes.POINTER(ctypes.c_int64), vp, vp, vp, vp, i64,
                                    ctypes.POINTER(sfr_info), vp]
        L.sfr_solve_nys.restype = ctypes.c_int
        L.sfr_tsvd.argtypes = [vp, vp, i64, vp, vp, vp, ctypes.POINTER(sfr_info), vp]
        L.sfr_tsvd.restype = ctypes.c_int
        L.sfr_create_batch.argtypes = [ctypes.POINTER(vp), i32, i64, i64, i32, ctypes.POINTER(sfr_options)]
        L.sfr_create_batch.restype = ctypes.c_int
        L.sfr_solve_batch.argtypes = [vp, ctypes.POINTER(sfr_batch_item), i32, ctypes.POINTER(sfr_info),
                                      ctypes.POINTER(ctypes.c_int32), vp]
        L.sfr_solve_batch.restype = ctypes.c_int
        L.sfr_tune_batch.argtypes = [vp, ctypes.POINTER(sfr_batch_item), i32, ctypes.POINTER(ctypes.c_int32), vp]
        L.sfr_tune_batch.restype = ctypes.c_int
        L.sfr_queue_start.argtypes = [vp, i32, i32]
        L.sfr_queue_start.restype = ctypes.c_int
        L.sfr_queue_submit.argtypes = [vp, ctypes.POINTER(sfr_batch_item), ctypes.POINTER(ctypes.c_int32)]
        L.sfr_queue_submit.restype = ctypes.c_int
        L.sfr_queue_poll.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(sfr_info),
                                     ctypes.POINTER(ctypes.c_int32)]
        L.sfr_queue_poll.restype = ctypes.c_int
        L.sfr_queue_stop.argtypes = [vp]
        L.sfr_queue_stop.restype = ctypes.c_int
        L.sfr_solve_noalloc.argtypes = [i64, i64, i32, d, d, d, ctypes.POINTER(sfr_options), vp, i64, vp, vp,
                                         vp, vp, i64, ctypes.POINTER(sfr_info), vp]
        L.sfr_solve_noalloc.restype = ctypes.c_int
        L.sfr_destroy.argtypes = [vp]
        L.sfr_destroy.restype = ctypes.c_int
        L.sfr_workspace_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64)]
        L.sfr_workspace_bytes.restype = ctypes.c_int
        L.sfr_status_string.argtypes = [ctypes.c_int]
        L.sfr_status_string.restype = ctypes.c_char_p
        L.sfr_version.argtypes = []
        L.sfr_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def status_string(code: int) -> str:
    try:
        return lib().sfr_status_string(int(code)).decode()
    except ImportError:
        return f"status {code}"


@dataclass
class Info:
    status: int
    iters: int
    iters_top: int
    converged: bool
    rel_residual: float
    min_eig_B: float
    mu_final: float
    sweep_ms: float
    sweeps_timed: int
    mu0: float = 0.0
    orth_err: float = 0.0


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Solver:
    """A handle of the C ABI (sfr_create ... sfr_destroy).

    precision: "f64" (SFR_F64) or "f32" (SFR_F32).  mu is mu_0 of Alg. 1.
    nystrom_l > 0 makes an FR-Nys handle (Alg. 3) that needs mu_left/mu_top.
    bf16 (FP32 FR-ADM handles): BF16-operand contractions on the matrix cores
    for the leading iterations (until bf16_iters iterations or a residual <=
    bf16_tol), then FP32 iterations from that iterate.
    """

    def __init__(self, m, n, r, lam, mu, tol=1e-7, *, precision="f64", rho=1.5, mu_bar=1e9,
                 max_iter=300, fixed_iters=0, nystrom_l=0, mu_left=0.0, mu_top=0.0, profile=False,
                 bf16=False, bf16_iters=0, bf16_tol=0.0):
        self.m, self.n, self.r = int(m), int(n), int(r)
        self.precision = precision
        o = sfr_options()
        o.struct_size = ctypes.sizeof(sfr_options)
        o.precision = SFR_F64 if precision == "f64" else SFR_F32
        if precision not in ("f64", "f32"):
            raise ValueError(precision)
        o.rho, o.mu_bar = float(rho), float(mu_bar)
        o.max_iter, o.fixed_iters = int(max_iter), int(fixed_iters)
        o.nystrom_l = int(nystrom_l)
        o.profile = 1 if profile else 0
        o.mu_left, o.mu_top = float(mu_left), float(mu_top)
        o.bf16, o.bf16_iters, o.bf16_tol = (1 if bf16 else 0), int(bf16_iters), float(bf16_tol)
        self.nystrom_l = int(nystrom_l)
        self._h = ctypes.c_void_p(None)
        rc = lib().sfr_create(ctypes.byref(self._h), self.m, self.n, self.r, float(lam), float(mu), float(tol),
                              ctypes.byref(o))
        if rc != SFR_OK:
            self._h = ctypes.c_void_p(None)
            raise SFRError(rc, "sfr_create")

    @property
    def dtype(self):
        import torch
        return torch.float64 if self.precision == "f64" else torch.float32

    def workspace_bytes(self) -> int:
        b = ctypes.c_uint64(0)
        rc = lib().sfr_workspace_bytes(self._h, ctypes.byref(b))
        if rc != SFR_OK:
            raise SFRError(rc, "sfr_workspace_bytes")
        return int(b.value)

    def _check_M(self, M):
        import torch
        if not (isinstance(M, torch.Tensor) and M.is_cuda):
            raise TypeError("M must be a CUDA (HIP) torch tensor")
        if M.dtype != self.dtype or M.dim() != 2 or tuple(M.shape) != (self.m, self.n):
            raise ValueError(f"M must be {self.m}x{self.n} {self.dtype}")
        if M.stride(1) != 1:
            raise ValueError("M must be row-major (unit column stride)")

    def _outputs(self, M, want_S, out):
        import torch
        dev = M.device
        if out is None:
            U = torch.empty((self.m, self.r), dtype=self.dtype, device=dev)
            B = torch.empty((self.r, self.r), dtype=torch.float64, device=dev)
            V = torch.empty((self.n, self.r), dtype=self.dtype, device=dev)
            S = torch.empty((self.m, self.n), dtype=self.dtype, device=dev) if want_S else None
        else:
            U, B, V, S = out
            check_outputs(U, B, V, S, self.m, self.n, self.r, self.dtype, dev)
        return U, B, V, S

    def solve(self, M, *, want_S=True, out=None, stream=None, raise_on_error=True):
        """FR-ADM.  Returns (U, B, V, S, Info); S is None if want_S is False."""
        self._check_M(M)
        U, B, V, S = self._outputs(M, want_S, out)
        info = sfr_info()
        rc = lib().sfr_solve(self._h, ctypes.c_void_p(M.data_ptr()), M.stride(0), ctypes.c_void_p(U.data_ptr()),
                             ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(V.data_ptr()),
                             ctypes.c_void_p(S.data_ptr()) if S is not None else None,
                             S.stride(0) if S is not None else 0, ctypes.byref(info), _stream_handle(stream))
        if rc < 0 and raise_on_error:
            raise SFRError(rc, "sfr_solve")
        return U, B, V, S, _info(rc, info)

    def solve_nys(self, M, perm, *, want_S=True, out=None, stream=None, raise_on_error=True):
        """FR-Nys with row shuffle `perm` (host int64 array of length m)."""
        import numpy as np
        self._check_M(M)
        U, B, V, S = self._outputs(M, want_S, out)
        p = np.ascontiguousarray(perm, dtype=np.int64)
        if p.shape != (self.m,):
            raise ValueError("perm must have m entries")
        info = sfr_info()
        rc = lib().sfr_solve_nys(self._h, ctypes.c_void_p(M.data_ptr()), M.stride(0),
                                 p.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.c_void_p(U.data_ptr()),
                                 ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(V.data_ptr()),
                                 ctypes.c_void_p(S.data_ptr()) if S is not None else None,
                                 S.stride(0) if S is not None else 0, ctypes.byref(info), _stream_handle(stream))
        if rc < 0 and raise_on_error:
            raise SFRError(rc, "sfr_solve_nys")
        return U, B, V, S, _info(rc, info)

    def tsvd(self, M, *, out=None, stream=None, raise_on_error=True):
        """FixedRankOptFull (Alg. 4) on M: the rank-r truncated SVD as
        (U, B, V, Info); lambda and mu of the handle are not used."""
        self._check_M(M)
        U, B, V, _ = self._outputs(M, False, None if out is None else (*out, None))
        info = sfr_info()
        rc = lib().sfr_tsvd(self._h, ctypes.c_void_p(M.data_ptr()), M.stride(0), ctypes.c_void_p(U.data_ptr()),
                            ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(V.data_ptr()), ctypes.byref(info),
                            _stream_handle(stream))
        if rc < 0 and raise_on_error:
            raise SFRError(rc, "sfr_tsvd")
        return U, B, V, _info(rc, info)

    def close(self):
        if self._h and self._h.value:
            lib().sfr_destroy(self._h)
        self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class BatchSolver:
    """A batched handle (sfr_create_batch ... sfr_destroy): many small FP32
    FR-ADM problems (n <= 512, r <= 16) solved by one kernel launch, one
    workgroup per problem."""

    def __init__(self, capacity, max_m, max_n, max_r, *, rho=1.5, mu_bar=1e9, max_iter=300, fixed_iters=0,
                 bf16=False, bf16_iters=0, bf16_tol=0.0):
        self.capacity, self.max_m, self.max_n, self.max_r = int(capacity), int(max_m), int(max_n), int(max_r)
        o = sfr_options()
        o.struct_size = ctypes.sizeof(sfr_options)
        o.precision = SFR_F32
        o.rho, o.mu_bar = float(rho), float(mu_bar)
        o.max_iter, o.fixed_iters = int(max_iter), int(fixed_iters)
        o.bf16, o.bf16_iters, o.bf16_tol = (1 if bf16 else 0), int(bf16_iters), float(bf16_tol)
        self._h = ctypes.c_void_p(None)
        rc = lib().sfr_create_batch(ctypes.byref(self._h), self.capacity, self.max_m, self.max_n, self.max_r,
                                    ctypes.byref(o))
        if rc != SFR_OK:
            self._h = ctypes.c_void_p(None)
            raise SFRError(rc, "sfr_create_batch")

    def workspace_bytes(self) -> int:
        b = ctypes.c_uint64(0)
        rc = lib().sfr_workspace_bytes(self._h, ctypes.byref(b))
        if rc != SFR_OK:
            raise SFRError(rc, "sfr_workspace_bytes")
        return int(b.value)

    def solve(self, problems, *, want_S=True, outs=None, stream=None, raise_on_error=True):
        """problems: a list of (M, r, lam, mu, tol) with M a float32 CUDA
        tensor (row-major).  Returns a list of (U, B, V, S, Info), one per
        problem (S None if want_S is False)."""
        import torch
        count = len(problems)
        items = (sfr_batch_item * max(count, 1))()
        keep = []
        for i, (M, r, lam, mu, tol) in enumerate(problems):
            if not (isinstance(M, torch.Tensor) and M.is_cuda and M.dtype == torch.float32 and M.dim() == 2):
                raise TypeError("each M must be a 2-D float32 CUDA (HIP) tensor")
            if M.stride(1) != 1:
                raise ValueError("M must be row-major (unit column stride)")
            m, n = M.shape
            if outs is None:
                U = torch.empty((m, r), dtype=torch.float32, device=M.device)
                B = torch.empty((r, r), dtype=torch.float64, device=M.device)
                V = torch.empty((n, r), dtype=torch.float32, device=M.device)
                S = torch.empty((m, n), dtype=torch.float32, device=M.device) if want_S else None
            else:
                U, B, V, S = outs[i]
                check_outputs(U, B, V, S, m, n, int(r), torch.float32, M.device)
            keep.append((U, B, V, S))
            it = items[i]
            it.m, it.n, it.r = m, n, int(r)
            it.lam, it.mu, it.tol = float(lam), float(mu), float(tol)
            it.M, it.ldm = M.data_ptr(), M.stride(0)
            it.U, it.B, it.V = U.data_ptr(), B.data_ptr(), V.data_ptr()
            it.S, it.lds = (S.data_ptr(), S.stride(0)) if S is not None else (None, 0)
        infos = (sfr_info * max(count, 1))()
        st = (ctypes.c_int32 * max(count, 1))()
        rc = lib().sfr_solve_batch(self._h, items, count, infos, st, _stream_handle(stream))
        if rc < 0 and (raise_on_error or rc in (SFR_ERR_ARG, SFR_ERR_HANDLE, SFR_ERR_DEVICE)):
            raise SFRError(rc, "sfr_solve_batch")
        return [(*keep[i], _info(int(st[i]), infos[i])) for i in range(count)]

    # ---- queue form (continuous batching): persistent kernels fed while they run
    def queue_start(self, grid_large=0, grid_small=0):
        """Launch the persistent kernels (sfr_queue_start)."""
        self._tickets = {}
        rc = lib().sfr_queue_start(self._h, int(grid_large), int(grid_small))
        if rc != SFR_OK:
            raise SFRError(rc, "sfr_queue_start")

    def queue_submit(self, M, r, lam, mu, tol, *, want_S=True, out=None):
        """Append one problem (M a row-major float32 CUDA tensor).  Returns
        its ticket, or None if every slot is in flight (SFR_ERR_BUSY).  The
        output tensors are kept until the result is collected."""
        import torch
        if not (isinstance(M, torch.Tensor) and M.is_cuda and M.dtype == torch.float32 and M.dim() == 2):
            raise TypeError("M must be a 2-D float32 CUDA (HIP) tensor")
        if M.stride(1) != 1:
            raise ValueError("M must be row-major (unit column stride)")
        m, n = M.shape
        if out is None:
            U = torch.empty((m, r), dtype=torch.float32, device=M.device)
            B = torch.empty((r, r), dtype=torch.float64, device=M.device)
            V = torch.empty((n, r), dtype=torch.float32, device=M.device)
            S = torch.empty((m, n), dtype=torch.float32, device=M.device) if want_S else None
        else:
            U, B, V, S = out
            check_outputs(U, B, V, S, m, n, int(r), torch.float32, M.device)
        it = sfr_batch_item()
        it.m, it.n, it.r = m, n, int(r)
        it.lam, it.mu, it.tol = float(lam), float(mu), float(tol)
        it.M, it.ldm = M.data_ptr(), M.stride(0)
        it.U, it.B, it.V = U.data_ptr(), B.data_ptr(), V.data_ptr()
        it.S, it.lds = (S.data_ptr(), S.stride(0)) if S is not None else (None, 0)
        t = ctypes.c_int32(-1)
        rc = lib().sfr_queue_submit(self._h, ctypes.byref(it), ctypes.byref(t))
        if rc == SFR_ERR_BUSY:
            return None
        if rc != SFR_OK:
            raise SFRError(rc, "sfr_queue_submit")
        self._tickets[t.value] = (M, U, B, V, S)
        return t.value

    def queue_poll(self, ticket):
        """None while the problem is in flight, else (U, B, V, S, Info)."""
        done = ctypes.c_int32(0)
        info = sfr_info()
        st = ctypes.c_int32(0)
        rc = lib().sfr_queue_poll(self._h, int(ticket), ctypes.byref(done), ctypes.byref(info), ctypes.byref(st))
        if rc != SFR_OK:
            raise SFRError(rc, "sfr_queue_poll")
        if not done.value:
            return None
        _, U, B, V, S = self._tickets.pop(ticket)
        return U, B, V, S, _info(st.value, info)

    def queue_stop(self):
        rc = lib().sfr_queue_stop(self._h)
        if rc != SFR_OK:
            raise SFRError(rc, "sfr_queue_stop")

    VARIANTS = {0: "default", 1: "lane groups", 2: "one row per wavefront", 3: "two rows per wavefront",
                4: "matrix cores"}
    BUCKETS = (1, 2, 3, 4, 5, 6, 8, 10, 12, 16)

    def autotune(self, problems, *, stream=None):
        """Time the batched kernel's band-loop forms on `problems` (a list of
        (M, r, lam, mu, tol), as for solve) and keep the fastest per problem
        class and rank bucket.  Returns {(narrow, bucket): form name} for the
        tuned pairs."""
        import torch
        items = (sfr_batch_item * max(len(problems), 1))()
        keep = []
        for i, (M, r, lam, mu, tol) in enumerate(problems):
            m, n = M.shape
            U = torch.empty((m, r), dtype=torch.float32, device=M.device)
            B = torch.empty((r, r), dtype=torch.float64, device=M.device)
            V = torch.empty((n, r), dtype=torch.float32, device=M.device)
            keep.append((U, B, V))
            it = items[i]
            it.m, it.n, it.r = m, n, int(r)
            it.lam, it.mu, it.tol = float(lam), float(mu), float(tol)
            it.M, it.ldm = M.data_ptr(), M.stride(0)
            it.U, it.B, it.V = U.data_ptr(), B.data_ptr(), V.data_ptr()
            it.S, it.lds = None, 0
        table = (ctypes.c_int32 * 20)()
        rc = lib().sfr_tune_batch(self._h, items, len(problems), table, _stream_handle(stream))
        if rc != SFR_OK:
            raise SFRError(rc, "sfr_tune_batch")
        return {(bool(c), self.BUCKETS[b]): self.VARIANTS[table[c * 10 + b]]
                for c in range(2) for b in range(10) if table[c * 10 + b]}

    def close(self):
        if self._h and self._h.value:
            lib().sfr_destroy(self._h)
        self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def check_outputs(U, B, V, S, m, n, r, dtype, device):
    """Caller-supplied output buffers must be what the C ABI writes: U dense
    m x r, V dense n x r (dtype of the data), B dense r x r float64, S (or
    None) m x n with unit column stride, all on M's device.  Raises
    ValueError before any library call otherwise."""
    import torch
    for name, t, shape, dt in (("U", U, (m, r), dtype), ("B", B, (r, r), torch.float64), ("V", V, (n, r), dtype)):
        if not isinstance(t, torch.Tensor):
            raise ValueError(f"{name} must be a torch tensor")
        if tuple(t.shape) != shape or t.dtype != dt:
            raise ValueError(f"{name} must be {shape[0]}x{shape[1]} {dt}, got {tuple(t.shape)} {t.dtype}")
        if t.device != device:
            raise ValueError(f"{name} must be on {device}, got {t.device}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous (dense row-major)")
    if S is not None:
        if not isinstance(S, torch.Tensor):
            raise ValueError("S must be a torch tensor or None")
        if tuple(S.shape) != (m, n) or S.dtype != dtype:
            raise ValueError(f"S must be {m}x{n} {dtype}, got {tuple(S.shape)} {S.dtype}")
        if S.device != device:
            raise ValueError(f"S must be on {device}, got {S.device}")
        if S.stride(1) != 1 or S.stride(0) < n:
            raise ValueError("S must be row-major with unit column stride and row stride >= n")


def _info(rc, info):
    return Info(status=int(rc), iters=info.iters, iters_top=info.iters_top, converged=bool(info.converged),
                rel_residual=info.rel_residual, min_eig_B=info.min_eig_B, mu_final=info.mu_final,
                sweep_ms=info.sweep_ms, sweeps_timed=info.sweeps_timed, mu0=info.mu0,
                orth_err=info.orth_err)


def _options(precision, rho=1.5, mu_bar=1e9, max_iter=300, fixed_iters=0, nystrom_l=0, mu_left=0.0, mu_top=0.0,
             profile=False, bf16=False, bf16_iters=0, bf16_tol=0.0):
    o = sfr_options()
    o.struct_size = ctypes.sizeof(sfr_options)
    o.precision = SFR_F64 if precision == "f64" else SFR_F32
    o.rho, o.mu_bar = float(rho), float(mu_bar)
    o.max_iter, o.fixed_iters = int(max_iter), int(fixed_iters)
    o.nystrom_l = int(nystrom_l)
    o.profile = 1 if profile else 0
    o.mu_left, o.mu_top = float(mu_left), float(mu_top)
    o.bf16, o.bf16_iters, o.bf16_tol = (1 if bf16 else 0), int(bf16_iters), float(bf16_tol)
    return o


def solve_noalloc(M, r, lam, mu, tol, out, *, stream=None, raise_on_error=True, **opts):
    """sfr_solve_noalloc: FR-ADM with the library's static device scratch
    (no device allocation by the library).  out = (U, B, V, S or None): the
    caller's output tensors, checked as for Solver.solve.  Returns Info."""
    import torch
    if not (isinstance(M, torch.Tensor) and M.is_cuda and M.dim() == 2 and M.stride(1) == 1):
        raise TypeError("M must be a row-major 2-D CUDA (HIP) tensor")
    precision = "f64" if M.dtype == torch.float64 else "f32"
    if M.dtype not in (torch.float64, torch.float32):
        raise ValueError("M must be float64 or float32")
    m, n = M.shape
    U, B, V, S = out
    check_outputs(U, B, V, S, m, n, int(r), M.dtype, M.device)
    o = _options(precision, **opts)
    info = sfr_info()
    rc = lib().sfr_solve_noalloc(m, n, int(r), float(lam), float(mu), float(tol), ctypes.byref(o),
                                 ctypes.c_void_p(M.data_ptr()), M.stride(0), ctypes.c_void_p(U.data_ptr()),
                                 ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(V.data_ptr()),
                                 ctypes.c_void_p(S.data_ptr()) if S is not None else None,
                                 S.stride(0) if S is not None else 0, ctypes.byref(info), _stream_handle(stream))
    if rc < 0 and raise_on_error:
        raise SFRError(rc, "sfr_solve_noalloc")
    return _info(rc, info)


def solve(M, r, lam, mu, tol=1e-7, **opts):
    """One-shot FR-ADM on a CUDA tensor M: returns (U, B, V, S, Info)."""
    import torch
    precision = "f64" if M.dtype == torch.float64 else "f32"
    with Solver(M.shape[0], M.shape[1], r, lam, mu, tol, precision=precision, **opts) as s:
        return s.solve(M)


def solve_nys(M, perm, r, lam, l, mu_left, mu_top, tol=1e-7, **opts):
    """One-shot FR-Nys on a CUDA tensor M: returns (U, B, V, S, Info)."""
    import torch
    precision = "f64" if M.dtype == torch.float64 else "f32"
    with Solver(M.shape[0], M.shape[1], r, lam, 1.0, tol, precision=precision, nystrom_l=l,
                mu_left=mu_left, mu_top=mu_top, **opts) as s:
        return s.solve_nys(M, perm)


def tsvd(M, r, tol=1e-12, **opts):
    """One-shot FixedRankOptFull (Alg. 4) on a CUDA tensor M: the rank-r
    truncated SVD as (U, B, V, Info)."""
    import torch
    precision = "f64" if M.dtype == torch.float64 else "f32"
    with Solver(M.shape[0], M.shape[1], r, 1.0, 1.0, tol, precision=precision, **opts) as s:
        return s.tsvd(M)
