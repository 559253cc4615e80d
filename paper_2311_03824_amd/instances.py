"""Seeded synthetic instances of low-rank + sparse column-wise compressive sensing.

Problem statement of Sec. 1.1: recover X* = L* + S* (n x q) from y_k = A_k x*_k,
k in [q], with A_k an m x n dense i.i.d. standard Gaussian matrix, L* = U* B* of
rank r and each column of S* holding exactly rho nonzeros.  Data-generation
protocol of Sec. 3: U* is the orthonormalised n x r Gaussian matrix, B* is
i.i.d. Gaussian r x q, the support of each S* column is drawn uniformly without
replacement, and y_k is noise free.

This module holds no arithmetic of the recovery method.  It only draws the
inputs and lays them out for the device and for the oracle.  It is the single
source of inputs shared by the tests, the benchmark and the oracle checks.

Canonical A.  Each A_k entry a is drawn as an FP32 normal and then replaced by
hi + lo with hi = bf16_rne(a) and lo = bf16_rne(a - hi).  hi + lo is exactly
representable in FP32 (and FP64), so the FP32 plane, the BF16 hi/lo planes and
the FP64 oracle all see the same matrix.

Device layout of A.  A_k is stored column-major with the row index i fastest:
element (i, j) of A_k sits at ``At[k, j, i]`` of an array of shape (q, n, lda)
with lda = m rounded up to a multiple of 8; rows m..lda-1 are zero.  Y is (q, m)
with y_k contiguous.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

# Stream tags of the seed sequence: each drawn object has its own stream so that
# changing one size does not change another object's draws.
_TAG_A, _TAG_U, _TAG_B, _TAG_SUPP, _TAG_SVAL, _TAG_START = range(6)

#: Named workloads.  Sizes follow the synthetic set-ups of Sec. 3 and the
#: scaled-up throughput shapes used by the benchmark.
WORKLOADS = {
    # exact-recovery check size: n = q = 100, m = 40, r = 2, rho = 2
    "gauss_n100_q100_m40_r2_rho2": dict(n=100, q=100, m=40, r=2, rho=2, seed=231103824),
    # FP32 throughput shape: n = q = 600, m = 250, r = 4, rho = 30 (5 %)
    "gauss_n600_q600_m250_r4_rho30": dict(n=600, q=600, m=250, r=4, rho=30, seed=231103825),
    # headline shape: n = q = 1000, m = 400, r = 10, rho = 50
    "gauss_n1000_q1000_m400_r10_rho50": dict(n=1000, q=1000, m=400, r=10, rho=50, seed=231103826),
}


def bf16_rne(x: np.ndarray) -> np.ndarray:
    """Round FP32 values to the nearest bfloat16 (ties to even); return FP32."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def split_bf16(a: np.ndarray):
    """Split FP32 ``a`` into (hi_bits, lo_bits, canonical).

    hi = bf16_rne(a), lo = bf16_rne(a - hi) (a - hi is exact in FP32),
    canonical = hi + lo (exact in FP32).  The bit arrays are uint16.
    """
    a = np.ascontiguousarray(a, dtype=np.float32)
    hi = bf16_rne(a)
    lo = bf16_rne(a - hi)
    canon = hi + lo
    hi_bits = (hi.view(np.uint32) >> 16).astype(np.uint16)
    lo_bits = (lo.view(np.uint32) >> 16).astype(np.uint16)
    return hi_bits, lo_bits, canon


def round_up(x: int, mult: int) -> int:
    return (x + mult - 1) // mult * mult


@dataclasses.dataclass
class Instance:
    n: int
    q: int
    m: int
    r: int
    rho: int
    seed: int
    At: np.ndarray        # (q, n, lda) float32, At[k, j, i] = A_k[i, j]; rows >= m are zero
    Y32: np.ndarray       # (q, m) float32, y_k rounded to FP32
    Y64: np.ndarray       # (q, m) float64, exact y_k = A_k x*_k
    U_star: np.ndarray    # (n, r) float64, orthonormal
    B_star: np.ndarray    # (r, q) float64
    S_star: np.ndarray    # (n, q) float64, exactly rho nonzeros per column
    supp: np.ndarray      # (q, rho) int64, ascending support of each S* column
    U_start: np.ndarray   # (n, r) float32, Gaussian start block for subspace iteration
    A_hi: Optional[np.ndarray] = None  # (q, n, lda) uint16 bf16 hi plane
    A_lo: Optional[np.ndarray] = None  # (q, n, lda) uint16 bf16 lo plane

    @property
    def lda(self) -> int:
        return self.At.shape[2]

    @property
    def X_star(self) -> np.ndarray:
        return self.U_star @ self.B_star + self.S_star

    def A64_hi(self) -> np.ndarray:
        """The bf16 hi plane alone as FP64 (q, m, n) arrays: the matrix a hi-only pass reads."""
        hi = (self.A_hi[:, :, : self.m].astype(np.uint32) << 16).view(np.float32)
        return np.ascontiguousarray(hi.transpose(0, 2, 1), dtype=np.float64)

    def A64(self, ks=None) -> np.ndarray:
        """A_k as FP64 (len(ks), m, n) arrays (exact widening of the canonical FP32 values)."""
        At = self.At if ks is None else self.At[ks]
        return np.ascontiguousarray(At[:, :, : self.m].transpose(0, 2, 1), dtype=np.float64)


def _rng(seed: int, tag: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(tag)]))


def make_instance(n: int, q: int, m: int, r: int, rho: int, seed: int,
                  s_dist: str = "normal", s_scale: float = 10.0,
                  s_zero: bool = False, lda_mult: int = 8,
                  bf16_planes: bool = False, chunk: int = 64) -> Instance:
    """Draw one seeded instance.

    s_dist: "normal" draws S* values N(0, s_scale^2); "uniform" draws
    U[-s_scale, s_scale] (the S1 law of Sec. 3); "pm_powers" draws from
    {+-1, +-10, +-100} (the S2 law of Sec. 3).  s_zero=True gives S* = 0.
    """
    if not (1 <= r <= min(m, n)) or not (0 <= rho <= n) or min(n, q, m) < 1:
        raise ValueError("invalid sizes")
    lda = round_up(m, lda_mult)
    # U*: Q factor of an n x r Gaussian matrix, signs fixed so that R has a positive diagonal.
    G = _rng(seed, _TAG_U).standard_normal((n, r))
    Q, R = np.linalg.qr(G)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    U_star = Q * d
    B_star = _rng(seed, _TAG_B).standard_normal((r, q))
    # support: rho rows per column, uniform without replacement
    keys = _rng(seed, _TAG_SUPP).random((q, n))
    supp = np.sort(np.argsort(keys, axis=1, kind="stable")[:, :rho], axis=1)
    rv = _rng(seed, _TAG_SVAL)
    if s_dist == "normal":
        vals = rv.standard_normal((q, rho)) * s_scale
    elif s_dist == "uniform":
        vals = rv.uniform(-s_scale, s_scale, (q, rho))
    elif s_dist == "pm_powers":
        vals = rv.choice(np.array([-1.0, -10.0, -100.0, 1.0, 10.0, 100.0]), size=(q, rho))
    else:
        raise ValueError(s_dist)
    S_star = np.zeros((n, q))
    if not s_zero and rho > 0:
        S_star[supp, np.arange(q)[:, None]] = vals
    X_star = U_star @ B_star + S_star

    # A: canonical hi + lo of an FP32 Gaussian draw, drawn column by column (k)
    ra = _rng(seed, _TAG_A)
    At = np.zeros((q, n, lda), np.float32)
    A_hi = np.zeros((q, n, lda), np.uint16) if bf16_planes else None
    A_lo = np.zeros((q, n, lda), np.uint16) if bf16_planes else None
    Y64 = np.empty((q, m))
    for k0 in range(0, q, chunk):
        k1 = min(q, k0 + chunk)
        a = ra.standard_normal((k1 - k0, n, m), dtype=np.float32)
        hb, lb, canon = split_bf16(a)
        At[k0:k1, :, :m] = canon
        if bf16_planes:
            A_hi[k0:k1, :, :m] = hb
            A_lo[k0:k1, :, :m] = lb
        # y_k = A_k x*_k in FP64 (A_k^T stored row-major, so y_k = x*_k^T At_k)
        Y64[k0:k1] = np.matmul(X_star[:, k0:k1].T[:, None, :], canon.astype(np.float64))[:, 0, :]
    U_start = _rng(seed, _TAG_START).standard_normal((n, r)).astype(np.float32)
    return Instance(n=n, q=q, m=m, r=r, rho=rho, seed=seed, At=At,
                    Y32=Y64.astype(np.float32), Y64=Y64, U_star=U_star, B_star=B_star,
                    S_star=S_star, supp=supp, U_start=U_start, A_hi=A_hi, A_lo=A_lo)


def make_workload(name: str, **kw) -> Instance:
    cfg = dict(WORKLOADS[name])
    cfg.update(kw)
    return make_instance(**cfg)
