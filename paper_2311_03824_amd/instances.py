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


# ---------------------------------------------------------------- Philox form of A
# A_k entries regenerated from a counter: Philox4x32-10 (Salmon, Moraes, Dror,
# Shaw, SC'11) with key = (seed low word, seed high word) and counter
# (chunk, j, k, 0), where chunk = i // 4 indexes 4 consecutive rows of column j;
# output word i % 4 gives element (i, j) of A_k.  A 32-bit word x becomes a normal
# deviate by an inverse-CDF table, log-spaced in v = (2 (x & 0x7fffffff) + 1) 2^-33
# (v in (0, 1/2], the smaller of u and 1 - u for u uniform on (0, 1)):
# |z| = T[idx] + (T[idx+1] - T[idx]) t with idx from the exponent and the top 6
# mantissa bits of v and t from the remaining 17 bits, and sign(z) = top bit of x.
# Only correctly rounded FP32 conversions, subtractions, multiplications and
# additions are used, so every implementation of this definition gives the same bits.

PHILOX_M0, PHILOX_M1 = 0xD2511F53, 0xCD9E8D57
PHILOX_W0, PHILOX_W1 = 0x9E3779B9, 0xBB67AE85
NORMAL_TABLE_EXPONENTS = 32          # v in [2^-33, 2^-1); v = 1/2 maps to the last two entries
NORMAL_TABLE_SUB = 64                # 6 mantissa bits per exponent


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Philox4x32 with 10 rounds on arrays of counter words; returns four uint32 arrays."""
    m = np.uint64(0xFFFFFFFF)
    c = [np.asarray(x).astype(np.uint64) for x in (c0, c1, c2, c3)]
    M0, M1 = np.uint64(PHILOX_M0), np.uint64(PHILOX_M1)
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + PHILOX_W0) & 0xFFFFFFFF
            k1 = (k1 + PHILOX_W1) & 0xFFFFFFFF
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        c = [(p1 >> np.uint64(32)) ^ c[1] ^ np.uint64(k0), p1 & m, (p0 >> np.uint64(32)) ^ c[3] ^ np.uint64(k1), p0 & m]
    return [x.astype(np.uint32) for x in c]


def normal_table() -> np.ndarray:
    """|z| = -ndtri(v) at v = 2^(e-33) (1 + s/64), e = 0..31, s = 0..63, then two entries for
    v = 1/2 (z = 0); FP32 values of the FP64 ndtri, 32 * 64 + 2 entries."""
    from scipy.special import ndtri
    e = np.arange(NORMAL_TABLE_EXPONENTS)[:, None]
    s_ = np.arange(NORMAL_TABLE_SUB)[None, :]
    v = np.ldexp(1.0 + s_ / NORMAL_TABLE_SUB, e - 33).ravel()
    t = -ndtri(np.concatenate([v, [0.5, 0.5]]))
    return np.abs(t).astype(np.float32)


def words_to_normal(x: np.ndarray, table: np.ndarray) -> np.ndarray:
    """The table transform of uint32 words x into FP32 normal deviates."""
    x = np.asarray(x, dtype=np.uint32)
    w = (x & np.uint32(0x7FFFFFFF)).astype(np.uint64)
    v = (np.uint64(2) * w + np.uint64(1)).astype(np.float32) * np.float32(2.0 ** -33)
    bits = v.view(np.uint32)
    e_idx = (bits >> np.uint32(23)).astype(np.int64) - (127 - 33)
    mant = bits & np.uint32(0x7FFFFF)
    idx = e_idx * NORMAL_TABLE_SUB + (mant >> np.uint32(17)).astype(np.int64)
    t = (mant & np.uint32(0x1FFFF)).astype(np.float32) * np.float32(2.0 ** -17)
    lo = table[idx]
    hi = table[idx + 1]
    z = lo + (hi - lo) * t
    return np.where(x >> np.uint32(31) != 0, -z, z).astype(np.float32)


def philox_A(seed: int, k_range, n: int, m: int, lda: int, table: np.ndarray) -> np.ndarray:
    """A_k^T (len(k_range), n, lda) FP32 for the Philox form; rows m..lda-1 are zero."""
    ks = np.asarray(list(k_range), dtype=np.uint64)
    nch = (m + 3) // 4
    K, J, C = np.meshgrid(ks, np.arange(n, dtype=np.uint64), np.arange(nch, dtype=np.uint64), indexing="ij")
    w = philox4x32_10(C, J, K, np.zeros_like(C), seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    z = np.stack([words_to_normal(wi, table) for wi in w], axis=-1).reshape(len(ks), n, nch * 4)
    out = np.zeros((len(ks), n, lda), np.float32)
    out[:, :, :m] = z[:, :, :m]
    return out


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
    a_seed: Optional[int] = None       # Philox form: the 64-bit key of A
    table: Optional[np.ndarray] = None # Philox form: the normal table

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
                  bf16_planes: bool = False, chunk: int = 64, a_form: str = "gauss") -> Instance:
    """Draw one seeded instance.

    s_dist: "normal" draws S* values N(0, s_scale^2); "uniform" draws
    U[-s_scale, s_scale] (the S1 law of Sec. 3); "pm_powers" draws from
    {+-1, +-10, +-100} (the S2 law of Sec. 3).  s_zero=True gives S* = 0.
    a_form="philox" draws A from the Philox definition above (key derived from the
    seed) instead of the canonical bf16 hi + lo of a NumPy Gaussian draw.
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

    a_seed = table = None
    if a_form == "philox":
        a_seed = int(_rng(seed, _TAG_A).integers(0, 2**63))
        table = normal_table()
    elif a_form != "gauss":
        raise ValueError(a_form)
    # A: canonical hi + lo of an FP32 Gaussian draw, drawn column by column (k)
    ra = _rng(seed, _TAG_A)
    At = np.zeros((q, n, lda), np.float32)
    A_hi = np.zeros((q, n, lda), np.uint16) if bf16_planes else None
    A_lo = np.zeros((q, n, lda), np.uint16) if bf16_planes else None
    Y64 = np.empty((q, m))
    starts = list(range(0, q, chunk))
    philox_chunks = None
    if a_form == "philox":
        # independent column ranges, generated in parallel (NumPy releases the GIL in its loops)
        import concurrent.futures as cf
        import os as _os
        workers = max(1, min(16, len(_os.sched_getaffinity(0))))
        with cf.ThreadPoolExecutor(max_workers=workers) as ex:
            philox_chunks = list(ex.map(
                lambda k0: philox_A(a_seed, range(k0, min(q, k0 + chunk)), n, m, m, table), starts))
    for ci, k0 in enumerate(starts):
        k1 = min(q, k0 + chunk)
        if a_form == "philox":
            canon = philox_chunks[ci]
            philox_chunks[ci] = None
            hb = lb = None
        else:
            a = ra.standard_normal((k1 - k0, n, m), dtype=np.float32)
            hb, lb, canon = split_bf16(a)
        At[k0:k1, :, :m] = canon
        if bf16_planes and hb is not None:
            A_hi[k0:k1, :, :m] = hb
            A_lo[k0:k1, :, :m] = lb
        # y_k = A_k x*_k in FP64 (A_k^T stored row-major, so y_k = x*_k^T At_k)
        Y64[k0:k1] = np.matmul(X_star[:, k0:k1].T[:, None, :], canon.astype(np.float64))[:, 0, :]
    U_start = _rng(seed, _TAG_START).standard_normal((n, r)).astype(np.float32)
    return Instance(n=n, q=q, m=m, r=r, rho=rho, seed=seed, At=At,
                    Y32=Y64.astype(np.float32), Y64=Y64, U_star=U_star, B_star=B_star,
                    S_star=S_star, supp=supp, U_start=U_start, A_hi=A_hi, A_lo=A_lo,
                    a_seed=a_seed, table=table)


def make_workload(name: str, **kw) -> Instance:
    cfg = dict(WORKLOADS[name])
    cfg.update(kw)
    return make_instance(**cfg)


# ---------------------------------------------------------------- serving workload
# A stream of independent problems of mixed sizes (the serving set-up): per
# request n ~ logU[256, 2048], q ~ logU[128, 1024], r ~ logU[2, 16] rounded,
# m = round(n U[0.3, 0.5]), rho = round(n U[0.01, 0.05]); the stored form of A
# alternates between the FP32 plane and the BF16 hi/lo pair.  U*, B*, S* follow
# the laws of make_instance; A is the canonical hi + lo of the Philox draw with a
# per-request key, so the device can write it without a host copy.

_TAG_SERVE = 7


@dataclasses.dataclass
class ServeRequest:
    idx: int
    n: int
    q: int
    m: int
    r: int
    rho: int
    a_format: str          # "f32" or "bf16x2"
    seed: int              # seed of this request's U*, B*, S* and A key
    arrival: float = 0.0   # seconds after the start of the run
    eta_scale: float = 1.0  # multiplies the step constant eta_c (a serving retry sets it below 1)

    @property
    def lda(self) -> int:
        return round_up(self.m, 8)

    @property
    def a_seed(self) -> int:
        return int(_rng(self.seed, _TAG_A).integers(0, 2**63))

    def a_bytes(self) -> int:
        """Device bytes of the stored A (4 per element in both forms)."""
        return 4 * self.q * self.n * self.lda


def _log_uniform(rng: np.random.Generator, lo: float, hi: float) -> float:
    return float(np.exp(rng.uniform(np.log(lo), np.log(hi))))


def serving_requests(count: int, seed: int, n_range=(256, 2048), q_range=(128, 1024),
                     r_range=(2, 16)) -> list:
    """Sizes and seeds of `count` requests (arrival times zero)."""
    rng = _rng(seed, _TAG_SERVE)
    out = []
    for i in range(count):
        n = int(round(_log_uniform(rng, *n_range)))
        q = int(round(_log_uniform(rng, *q_range)))
        r = int(round(_log_uniform(rng, *r_range)))
        m = int(round(n * rng.uniform(0.3, 0.5)))
        rho = int(round(n * rng.uniform(0.01, 0.05)))
        r = max(1, min(r, m, n))
        out.append(ServeRequest(idx=i, n=n, q=q, m=m, r=r, rho=rho,
                                a_format="f32" if i % 2 == 0 else "bf16x2",
                                seed=int(seed) * 1000003 + i))
    return out


def poisson_arrivals(count: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process of the given rate (requests/s)."""
    gaps = _rng(seed, _TAG_SERVE + 1).exponential(1.0 / rate, count)
    return np.cumsum(gaps) - gaps[0]


def _s_values(rng: np.random.Generator, shape, s_dist: str, s_scale: float) -> np.ndarray:
    """Nonzero values of S*: N(0, s_scale^2) ("normal"), U[-s_scale, s_scale] ("uniform", the
    S1 law of Sec. 3) or uniform over {+-1, +-10, +-100} ("pm_powers", the S2 law)."""
    if s_dist == "normal":
        return rng.standard_normal(shape) * s_scale
    if s_dist == "uniform":
        return rng.uniform(-s_scale, s_scale, shape)
    if s_dist == "pm_powers":
        return rng.choice(np.array([-1.0, -10.0, -100.0, 1.0, 10.0, 100.0]), size=shape)
    raise ValueError(s_dist)


def request_truth(req: ServeRequest, s_scale: float = 10.0, s_dist: str = "normal") -> dict:
    """U* (n, r), B* (r, q), the support (q, rho) and values, and Xt = X*^T (q, n) FP64."""
    n, q, r, rho = req.n, req.q, req.r, req.rho
    G = _rng(req.seed, _TAG_U).standard_normal((n, r))
    Q, R = np.linalg.qr(G)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    U_star = Q * d
    B_star = _rng(req.seed, _TAG_B).standard_normal((r, q))
    keys = _rng(req.seed, _TAG_SUPP).random((q, n))
    supp = np.sort(np.argpartition(keys, rho - 1, axis=1)[:, :rho], axis=1) if rho > 0 else np.zeros((q, 0), np.int64)
    vals = _s_values(_rng(req.seed, _TAG_SVAL), (q, rho), s_dist, s_scale)
    Xt = (U_star @ B_star).T.copy()
    if rho > 0:
        Xt[np.arange(q)[:, None], supp] += vals
    return dict(U_star=U_star, B_star=B_star, supp=supp, vals=vals, Xt=Xt)


def canonical_philox_A(a_seed: int, k_range, n: int, m: int, lda: int, table: np.ndarray):
    """(hi_bits, lo_bits, canonical FP32) of the Philox draw, each (len(k_range), n, lda)."""
    return split_bf16(philox_A(a_seed, k_range, n, m, lda, table))


# ---------------------------------------------------------------- partial Fourier form
# Frames of N1 x N2 complex pixels (x_k flattened row-major, n = N1 N2); A_k keeps
# m distinct rows of the unitary 2D DFT, the frequency indices of frame k drawn
# uniformly without replacement and stored ascending (index u = u1 N2 + u2).
# U* is the Q factor (real positive diagonal R) of an n x r complex Gaussian; B*
# is i.i.d. CN(0, 1); S* holds rho entries per column at uniformly drawn rows with
# CN(0, s_var) values.  y_k = rows mask_k of the unitary 2D DFT of x*_k.

_TAG_MASK = 9


@dataclasses.dataclass
class FourierInstance:
    N1: int
    N2: int
    q: int
    m: int
    r: int
    rho: int
    seed: int
    mask: np.ndarray      # (q, m) int64, ascending frequency indices of each frame
    Y: np.ndarray         # (q, m) complex128
    U_star: np.ndarray    # (n, r) complex128, orthonormal columns
    B_star: np.ndarray    # (r, q) complex128
    S_star: np.ndarray    # (n, q) complex128
    supp: np.ndarray      # (q, rho) int64

    @property
    def n(self) -> int:
        return self.N1 * self.N2

    @property
    def X_star(self) -> np.ndarray:
        return self.U_star @ self.B_star + self.S_star


def _complex_normal(rng: np.random.Generator, shape, var: float) -> np.ndarray:
    s = np.sqrt(var / 2.0)
    return rng.standard_normal(shape) * s + 1j * (rng.standard_normal(shape) * s)


def make_fourier_instance(N1: int, N2: int, q: int, m: int, r: int, rho: int, seed: int,
                          s_var: float = 25.0, s_zero: bool = False, real_signal: bool = False,
                          s_dist: str = "normal", s_scale: float = 6.0) -> FourierInstance:
    """Complex instance (defaults above), or with real_signal=True a real X*: U* the Q factor
    of a real Gaussian, B* i.i.d. N(0, 1) and S* values by `s_dist` / `s_scale` as in
    make_instance (the real protocol of Sec. 3 measured through partial Fourier rows)."""
    n = N1 * N2
    if not (1 <= r <= min(m, n)) or not (0 <= rho <= n) or not (1 <= m <= n) or q < 1:
        raise ValueError("invalid sizes")
    if real_signal:
        G = _rng(seed, _TAG_U).standard_normal((n, r)).astype(np.complex128)
    else:
        G = _complex_normal(_rng(seed, _TAG_U), (n, r), 1.0)
    Q, R = np.linalg.qr(G)
    d = np.diag(R)
    ph = np.where(np.abs(d) > 0, d / np.where(np.abs(d) > 0, np.abs(d), 1.0), 1.0)
    U_star = Q * ph
    if real_signal:
        U_star = U_star.real.astype(np.complex128)
        B_star = _rng(seed, _TAG_B).standard_normal((r, q)).astype(np.complex128)
    else:
        B_star = _complex_normal(_rng(seed, _TAG_B), (r, q), 1.0)
    keys = _rng(seed, _TAG_SUPP).random((q, n))
    supp = np.sort(np.argsort(keys, axis=1, kind="stable")[:, :rho], axis=1)
    if real_signal:
        vals = _s_values(_rng(seed, _TAG_SVAL), (q, rho), s_dist, s_scale).astype(np.complex128)
    else:
        vals = _complex_normal(_rng(seed, _TAG_SVAL), (q, rho), s_var)
    S_star = np.zeros((n, q), np.complex128)
    if not s_zero and rho > 0:
        S_star[supp, np.arange(q)[:, None]] = vals
    mkeys = _rng(seed, _TAG_MASK).random((q, n))
    mask = np.sort(np.argsort(mkeys, axis=1, kind="stable")[:, :m], axis=1)
    X = (U_star @ B_star + S_star).T.reshape(q, N1, N2)
    F = np.fft.fft2(X, norm="ortho").reshape(q, n)
    Y = F[np.arange(q)[:, None], mask]
    return FourierInstance(N1=N1, N2=N2, q=q, m=m, r=r, rho=rho, seed=seed, mask=mask, Y=Y,
                           U_star=U_star, B_star=B_star, S_star=S_star, supp=supp)
