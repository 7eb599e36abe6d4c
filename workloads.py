"""Seeded synthetic inputs for the S-FR decomposition M = L0 + S0.

This module only draws inputs.  It holds none of the decomposition's
arithmetic, and both the HIP library's tests/benchmark and the FP64 oracle
take their inputs from here, so the two sides always see the same matrix.

Workloads (shapes and value distributions follow the synthetic setup of
Sec. 5.1 -- L0 = A B^T with Gaussian factors, a sparse S0 at a given outlier
fraction -- and the photometric-stereo shape of Sec. 5.2):

  plain_fp64      m = n = 400, r = 5, 5 % outliers U[-50, 50] at exactly
                  round(0.05 m n) distinct positions, FP64
  large_fp32      m = n = 8000, r = 10, Bernoulli(0.10) outliers U[-100, 100]
  photometric     m = 262144 pixels x n = 48 images, r = 3 (Lambertian
                  albedo * normals * lights; specular and shadow outliers)
  nystrom_large   m = n = 40000, r = 20, Bernoulli(0.07) outliers Laplace(0, 20)
  stream          Poisson stream of small uneven instances

Every draw uses numpy's PCG64 generator with an explicit seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Instance:
    """One decomposition problem: M = L0 + S0 with rank(L0) = r."""
    M: np.ndarray
    r: int
    lam: float
    L0: np.ndarray | None = None
    S0: np.ndarray | None = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.M.shape


def bernoulli_positions(rng: np.random.Generator, total: int, p: float) -> np.ndarray:
    """Flat indices of a Bernoulli(p) mask over `total` cells, drawn by
    geometric gaps (exactly the Bernoulli process, without a `total`-sized
    temporary)."""
    if p <= 0.0 or total == 0:
        return np.zeros(0, dtype=np.int64)
    out = []
    pos = -1
    while True:
        want = int(p * (total - pos - 1) * 1.05) + 64
        gaps = rng.geometric(p, size=want).astype(np.int64)
        idx = pos + np.cumsum(gaps)
        keep = idx[idx < total]
        out.append(keep)
        if keep.size < idx.size:
            break
        pos = int(idx[-1])
    return np.concatenate(out)


def lowrank(rng: np.random.Generator, m: int, n: int, r: int, dtype=np.float64) -> np.ndarray:
    """L0 = A B^T, A (m x r), B (n x r) i.i.d. N(0, 1) (Sec. 5.1)."""
    A = rng.standard_normal((m, r))
    B = rng.standard_normal((n, r))
    if dtype == np.float64:
        return A @ B.T
    return (A.astype(np.float32) @ B.T.astype(np.float32)).astype(dtype)


def planted(m: int, n: int, r: int, *, seed: int, frac: float, kind: str = "uniform",
            scale: float = 1.0, exact_count: bool = False, dtype=np.float64,
            lam: float | None = None, name: str = "") -> Instance:
    """Planted instance M = L0 + S0.

    kind = "uniform": outlier values U[-scale, scale];
    kind = "laplace": outlier values Laplace(0, scale).
    exact_count: exactly round(frac m n) distinct positions; otherwise a
    Bernoulli(frac) mask.
    """
    rng = np.random.default_rng(seed)
    L0 = lowrank(rng, m, n, r, dtype)
    total = m * n
    if exact_count:
        k = int(round(frac * total))
        pos = rng.choice(total, size=k, replace=False)
    else:
        pos = bernoulli_positions(rng, total, frac)
    if kind == "uniform":
        vals = rng.uniform(-scale, scale, size=pos.size)
    elif kind == "laplace":
        vals = rng.laplace(0.0, scale, size=pos.size)
    else:
        raise ValueError(kind)
    S0 = np.zeros(total, dtype=dtype)
    S0[pos] = vals.astype(dtype)
    S0 = S0.reshape(m, n)
    M = (L0 + S0).astype(dtype)
    if lam is None:
        lam = 1.0 / math.sqrt(max(m, n))
    return Instance(M=M, r=r, lam=lam, L0=L0, S0=S0, name=name,
                    meta=dict(seed=seed, frac=frac, kind=kind, scale=scale))


def plain_fp64(seed: int = 0, m: int = 400, n: int = 400, r: int = 5) -> Instance:
    """400 x 400, r = 5, FP64, 5 % outliers U[-50, 50] at exact positions."""
    return planted(m, n, r, seed=seed, frac=0.05, kind="uniform", scale=50.0,
                   exact_count=True, dtype=np.float64, name=f"plain_fp64_{m}x{n}_r{r}")


def large_fp32(seed: int = 0, m: int = 8000, n: int = 8000, r: int = 10) -> Instance:
    """8000 x 8000, r = 10, FP32, Bernoulli(0.10) outliers U[-100, 100]."""
    return planted(m, n, r, seed=seed, frac=0.10, kind="uniform", scale=100.0,
                   dtype=np.float32, name=f"large_fp32_{m}x{n}_r{r}")


def nystrom_large(seed: int = 0, m: int = 40000, n: int = 40000, r: int = 20) -> Instance:
    """40000 x 40000, r = 20, FP32, Bernoulli(0.07) outliers Laplace(0, 20)."""
    return planted(m, n, r, seed=seed, frac=0.07, kind="laplace", scale=20.0,
                   dtype=np.float32, name=f"nystrom_large_{m}x{n}_r{r}")


def photometric(seed: int = 0, m: int = 262144, n: int = 48, dtype=np.float32) -> Instance:
    """Robust photometric stereo shape (Sec. 5.2): m pixels x n images, r = 3.

    Unit normals uniform on the upper hemisphere, light directions uniform on
    the spherical cap of 60 degree apex (polar angle <= 30 deg) around the
    viewing axis, albedo U[0.2, 1].  L0 = diag(albedo) N L^T has rank 3.
    M = max(0, L0), then 12 % of entries get an additive specular U[0.5, 3]
    and 8 % are set to 0 (cast shadows).  S0 = M - L0 collects the clamp
    residue, the speculars and the shadows.
    """
    rng = np.random.default_rng(seed)
    N = rng.standard_normal((m, 3))
    N[:, 2] = np.abs(N[:, 2])
    N /= np.linalg.norm(N, axis=1, keepdims=True)
    cos_t = rng.uniform(math.cos(math.radians(30.0)), 1.0, size=n)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=n)
    sin_t = np.sqrt(1.0 - cos_t ** 2)
    Ld = np.stack([sin_t * np.cos(phi), sin_t * np.sin(phi), cos_t], axis=1)
    alb = rng.uniform(0.2, 1.0, size=m)
    L0 = (alb[:, None] * N) @ Ld.T
    M = np.maximum(L0, 0.0)
    flat = M.reshape(-1)
    spec = bernoulli_positions(rng, m * n, 0.12)
    flat[spec] += rng.uniform(0.5, 3.0, size=spec.size)
    shadow = bernoulli_positions(rng, m * n, 0.08)
    flat[shadow] = 0.0
    M = M.astype(dtype)
    L0 = L0.astype(dtype)
    return Instance(M=M, r=3, lam=1.0 / math.sqrt(max(m, n)), L0=L0, S0=(M - L0),
                    name=f"photometric_{m}x{n}_r3", meta=dict(seed=seed))


def stream(seed: int = 0, count: int = 20000, rate: float = 2000.0):
    """Poisson stream of independent decompositions: arrival times (s) and
    per-request shapes; `stream_instance` draws each request's matrix."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=count))
    reqs = []
    for i in range(count):
        m = int(rng.integers(64, 2049))
        n = int(rng.integers(32, 513))
        r = int(rng.integers(2, 17))
        r = min(r, m, n)
        frac = float(rng.uniform(0.05, 0.15))
        reqs.append(dict(id=i, t=float(t[i]), m=m, n=n, r=r, frac=frac,
                         seed=int(seed * 1_000_003 + i)))
    return reqs


def stream_instance(req: dict, dtype=np.float32) -> Instance:
    return planted(req["m"], req["n"], req["r"], seed=req["seed"], frac=req["frac"],
                   kind="uniform", scale=50.0, dtype=dtype, name=f"req{req['id']}")


def row_permutation(m: int, seed: int) -> np.ndarray:
    """The random row shuffle that the Nystrom variant draws (Alg. 3),
    drawn here and handed to both sides as an input."""
    return np.random.default_rng(seed).permutation(m).astype(np.int64)


def spectral_norm(M: np.ndarray, iters: int = 60, seed: int = 1234) -> float:
    """||M||_2: exact SVD for small matrices, power iteration on M^T M
    (fixed start, fixed count) for large ones."""
    m, n = M.shape
    if m * n <= 4_000_000:
        return float(np.linalg.norm(M.astype(np.float64), 2))
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n)
    x /= np.linalg.norm(x)
    s = 0.0
    for _ in range(iters):
        y = M @ x.astype(M.dtype)
        x = (M.T @ y).astype(np.float64)
        s = math.sqrt(np.linalg.norm(x))
        x /= np.linalg.norm(x)
    return s


def default_mu0(M: np.ndarray) -> float:
    """Initial penalty mu_0 = 1.25 / ||M||_2 (the iALM scale the continuation
    scheme of Alg. 1 is taken from); passed explicitly to both sides."""
    return 1.25 / spectral_norm(M)


def nystrom_large_device(seed: int = 0, m: int = 40000, n: int = 40000, r: int = 20, frac: float = 0.07,
                         scale: float = 20.0, device="cuda"):
    """The 40000 x 40000, r = 20 workload drawn directly in device memory
    with torch's seeded generator (the host copy would be 6.4 GB): L0 =
    A B^T with N(0,1) factors, a Bernoulli(frac) outlier mask and
    Laplace(0, scale) outlier values (inverse-CDF draw, finite: the uniform
    draw is kept away from 0).  Returns
    (M, A, B, lam) with M float32 on `device`."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    A = torch.randn(m, r, generator=g, device=device, dtype=torch.float32)
    B = torch.randn(n, r, generator=g, device=device, dtype=torch.float32)
    M = A @ B.T
    rows_per = max(1, (1 << 28) // n)
    for i0 in range(0, m, rows_per):
        i1 = min(m, i0 + rows_per)
        u = torch.rand(i1 - i0, n, generator=g, device=device)
        mask = u < frac
        # FP32 uniforms are multiples of 2^-24 and include 0, where the
        # inverse CDF is infinite: the draw is clamped to the smallest
        # representable quantile (|Laplace| <= 24 ln 2 * scale, about 333)
        v = torch.rand(i1 - i0, n, generator=g, device=device).clamp_(min=2.0 ** -25) - 0.5
        lap = -scale * torch.sign(v) * torch.log1p(-2.0 * v.abs())
        M[i0:i1] += torch.where(mask, lap, torch.zeros_like(lap))
        del u, mask, v, lap
    return M, A, B, 1.0 / math.sqrt(max(m, n))


def stream_device(seed: int = 0, count: int = 4000, rate: float = 2000.0, device="cuda"):
    """The Poisson request stream (`stream`: arrival times, m U[64, 2048],
    n U[32, 512], r U{2..16}, outlier fraction U[0.05, 0.15]) with every
    request's matrix drawn in device memory by torch's seeded generator:
    L0 = A B^T with N(0,1) factors, Bernoulli(frac) outliers U[-50, 50].
    mu_0 = 1.25 / ||M||_2 with the norm from a fixed-count power iteration
    on the device (an input of the solve, shared by every side that solves
    the request).  Returns a list of dicts (id, t, m, n, r, frac, M, lam, mu).
    """
    import torch
    reqs = stream(seed=seed, count=count, rate=rate)
    g = torch.Generator(device=device)
    g.manual_seed(seed + 77)
    out = []
    for q in reqs:
        m, n, r = q["m"], q["n"], q["r"]
        A = torch.randn(m, r, generator=g, device=device, dtype=torch.float32)
        B = torch.randn(n, r, generator=g, device=device, dtype=torch.float32)
        M = A @ B.T
        mask = torch.rand(m, n, generator=g, device=device) < q["frac"]
        vals = (torch.rand(m, n, generator=g, device=device) * 2.0 - 1.0) * 50.0
        M = torch.where(mask, M + vals, M).contiguous()
        x = torch.ones(n, 1, device=device, dtype=torch.float32) / math.sqrt(n)
        for _ in range(12):
            x = M.T @ (M @ x)
            x = x / torch.linalg.vector_norm(x)
        s = torch.linalg.vector_norm(M @ x)
        out.append(dict(q, M=M, lam=1.0 / math.sqrt(max(m, n)), mu_t=s))
    for d in out:       # one host sync for all the norms
        d["mu"] = 1.25 / float(d.pop("mu_t"))
    return out
