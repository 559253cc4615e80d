// Shared device helpers and argument blocks of the AltGDmin-LR+S kernels (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace altg {

constexpr int kWaves = 4;            // waves per column workgroup
constexpr int kThreads = kWaves * 64;
constexpr int kRMax = 16;            // largest rank r with an instantiation
constexpr int kNCMax = 4;            // largest number of 256-row chunks per lane (m <= 1024)
constexpr int kQRThreads = 1024;

// A-operand formats (loader template argument)
enum { FMT_F32 = 0, FMT_BF16X2 = 1, FMT_BF16HI = 2, FMT_PHILOX = 3, FMT_BF16MIX = 4, FMT_PFOURIER = 5 };

// The column kernel reads A_k in two roles: the gathers that form A_k s_k (and
// so every residual) and the streaming passes (A_k^T u, and the step-length
// product A_k g_T on the support).  The mixed BF16 form takes the exact
// hi + lo planes for the first and the hi plane alone for the second; every
// other format reads the same view in both roles.
constexpr int gather_fmt(int f) { return f == FMT_BF16MIX ? FMT_BF16X2 : f; }
constexpr int stream_fmt(int f) { return f == FMT_BF16MIX ? FMT_BF16HI : f; }
constexpr int kNormalTable = 32 * 64 + 2;   // entries of the normal table of the Philox form

// Device-side control block of one solve.
struct Ctl {
  double eta;        // step size of the U update (0 until set at t = 1)
  double resid;      // ||Y - A(UB+S)||_F / ||Y||_F of the last iteration
  double power_sd;   // last subspace-iteration change
  double ynorm2;     // ||Y||_F^2
  int eta_set;       // 1 once eta is fixed
  int conv;          // subspace iteration converged
  int t;             // GDmin iterations done
  int power_it;      // subspace iterations done
  int err;           // OR of column error flags
  int phase;         // BF16X2 solves: 0 while the hi plane alone is read, 1 once hi + lo are read
  int refine_t;      // first iteration with phase 1 (-1 before)
  int done;          // batched stepping: the residual reached tol_resid; the problem is not advanced further
  int pad[4];
  double prev_resid; // residual of the previous iteration (stall test of the hi-only phase)
};

// Column kernel modes
enum { TAIL_NONE = 0, TAIL_LSGRAD = 1, TAIL_BACKPROJ = 2 };

struct ColArgs {
  int n, q, m, r, rho;
  const void* A;        // F32 plane, or BF16 hi plane
  const void* Alo;      // BF16 lo plane
  long long lda, sA;    // column stride and column-k stride, in elements
  const float* Y;
  long long ldy;
  const float* P;       // q x m x r (project mode)
  const double* Ginv;   // q x r x r (project mode)
  int* Tidx;            // q x rho, in/out
  float* Tval;          // q x rho, in/out
  float* G_out;         // optional q x n: gradient of the last IHT iteration
  double* mu_out;       // optional q: step of the last IHT iteration
  float* H;             // q x n: h_k (LSGRAD) or l_k (BACKPROJ)
  float* Bt;            // q x r (LSGRAD)
  double* rr;           // q: ||r_k||^2 (LSGRAD) or ||y_k||^2 (BACKPROJ)
  int* flags;           // q, OR-ed
  int tau, project, has_support, tail;
  const int* gate;      // if non-null, the kernel runs only when *gate == gate_want
  int gate_want;
  unsigned long long seed;  // Philox form: key of A
  const float* table;       // Philox form: normal table (kNormalTable FP32)
  int waves;                // waves of the column workgroup: 4 (also for 0), 8 or 16
};

struct AUArgs {
  int n, q, m, r;
  const void* A;
  const void* Alo;
  long long lda, sA;
  const float* U;       // n x r row-major
  float* P;             // q x m x r
  double* Ginv;         // q x r x r
  int* flags;
  const int* gate;      // if non-null, the kernel runs only when *gate == gate_want
  int gate_want;
  unsigned long long seed;  // Philox form: key of A
  const float* table;       // Philox form: normal table (kNormalTable FP32)
  int waves;                // waves per workgroup: 8 (at most 512 columns) or 4 (0 reads as 4)
};

// ---------------------------------------------------------------- wave reductions
// Butterfly sums: every lane ends with the same, bitwise identical total.
__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) x += __shfl_xor(x, o);
  return x;
}
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) x += __shfl_xor(x, o);
  return x;
}
__device__ __forceinline__ int wave_sum(int x) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) x += __shfl_xor(x, o);
  return x;
}

// DPP sums: quad swaps, half-row and row mirrors give every lane its 16-lane
// row sum; the four row sums are read with readlane and added in a fixed
// order, so every lane gets the same, bitwise identical total.
__device__ __forceinline__ float row_sum_dpp(float x) {
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));   // quad [1,0,3,2]
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xF, 0xF, false));   // quad [2,3,0,1]
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x141, 0xF, 0xF, false));  // row half mirror
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x140, 0xF, 0xF, false));  // row mirror
  return x;
}
__device__ __forceinline__ float wave_sum_dpp(float x) {
  x = row_sum_dpp(x);
  const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 0));
  const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 16));
  const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 32));
  const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 48));
  return (a + b) + (c + d);
}
__device__ __forceinline__ double dpp_f64(double x, int ctrl_sel) {
  const long long v = __double_as_longlong(x);
  int lo = (int)(v & 0xffffffffll), hi = (int)(v >> 32);
  switch (ctrl_sel) {
    case 0: lo = __builtin_amdgcn_update_dpp(0, lo, 0xB1, 0xF, 0xF, false); hi = __builtin_amdgcn_update_dpp(0, hi, 0xB1, 0xF, 0xF, false); break;
    case 1: lo = __builtin_amdgcn_update_dpp(0, lo, 0x4E, 0xF, 0xF, false); hi = __builtin_amdgcn_update_dpp(0, hi, 0x4E, 0xF, 0xF, false); break;
    case 2: lo = __builtin_amdgcn_update_dpp(0, lo, 0x141, 0xF, 0xF, false); hi = __builtin_amdgcn_update_dpp(0, hi, 0x141, 0xF, 0xF, false); break;
    default: lo = __builtin_amdgcn_update_dpp(0, lo, 0x140, 0xF, 0xF, false); hi = __builtin_amdgcn_update_dpp(0, hi, 0x140, 0xF, 0xF, false); break;
  }
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double readlane_f64(double x, int l) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double wave_sum_dpp(double x) {
  x += dpp_f64(x, 0);
  x += dpp_f64(x, 1);
  x += dpp_f64(x, 2);
  x += dpp_f64(x, 3);
  return (readlane_f64(x, 0) + readlane_f64(x, 16)) + (readlane_f64(x, 32) + readlane_f64(x, 48));
}

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

__device__ __forceinline__ float bf16_to_f32(uint32_t bits16) { return __uint_as_float(bits16 << 16); }

// ---------------------------------------------------------------- A_k loaders
// load(j, ch) returns rows 4*ch .. 4*ch+3 of column j of A_k.  Two load
// policies, the same values (so the same bits) either way:
//   POL_STREAM: non-temporal loads.  Each element is read once per pass, and
//     keeping A out of the caches lets a large A stream at 7.0 TB/s instead of
//     6.15 TB/s (one 256-thread workgroup per 1.6 MB column block, measured).
//   POL_CACHED: ordinary loads.  When the plane a pass streams fits in the
//     256 MB Infinity Cache, the passes after the first (and the next
//     iteration's) hit it: at n = 1000, m = 400, q = 125 (200 MB) the column
//     kernel takes 0.175 instead of 0.216 ms.
enum { POL_STREAM = 0, POL_CACHED = 1 };
typedef float f32x4_nt __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2_nt __attribute__((ext_vector_type(2)));
template <int POL>
__device__ __forceinline__ float4 ld_a(const float* p) {
  f32x4_nt v;
  if constexpr (POL == POL_CACHED) v = *reinterpret_cast<const f32x4_nt*>(p);
  else v = __builtin_nontemporal_load(reinterpret_cast<const f32x4_nt*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
template <int POL>
__device__ __forceinline__ uint2 ld_a(const uint16_t* p) {
  u32x2_nt v;
  if constexpr (POL == POL_CACHED) v = *reinterpret_cast<const u32x2_nt*>(p);
  else v = __builtin_nontemporal_load(reinterpret_cast<const u32x2_nt*>(p));
  return make_uint2(v.x, v.y);
}

template <int FMT, int POL = POL_STREAM> struct ALoader;

template <int POL> struct ALoader<FMT_F32, POL> {
  const float* base;
  long long lda;
  __device__ ALoader(const ColArgs& a, int k)
      : base(static_cast<const float*>(a.A) + (long long)k * a.sA), lda(a.lda) {}
  __device__ ALoader(const AUArgs& a, int k)
      : base(static_cast<const float*>(a.A) + (long long)k * a.sA), lda(a.lda) {}
  // fetch() issues the loads of 4 rows of column j; expand() turns them into
  // FP32.  Pipelined loops keep raw_t in flight and expand at the point of use,
  // so that a conversion never waits for loads issued after it.
  typedef float4 raw_t;
  __device__ __forceinline__ raw_t fetch(int j, int ch) const { return ld_a<POL>(base + (long long)j * lda + 4 * ch); }
  __device__ static __forceinline__ float4 expand(raw_t v) { return v; }
  __device__ __forceinline__ float4 load(int j, int ch) const { return fetch(j, ch); }
};

template <int POL> struct ALoader<FMT_BF16X2, POL> {
  const uint16_t* hi;
  const uint16_t* lo;
  long long lda;
  __device__ ALoader(const ColArgs& a, int k)
      : hi(static_cast<const uint16_t*>(a.A) + (long long)k * a.sA),
        lo(static_cast<const uint16_t*>(a.Alo) + (long long)k * a.sA), lda(a.lda) {}
  __device__ ALoader(const AUArgs& a, int k)
      : hi(static_cast<const uint16_t*>(a.A) + (long long)k * a.sA),
        lo(static_cast<const uint16_t*>(a.Alo) + (long long)k * a.sA), lda(a.lda) {}
  typedef uint4 raw_t;   // (hi pair, lo pair)
  __device__ __forceinline__ raw_t fetch(int j, int ch) const {
    const uint2 h = ld_a<POL>(hi + (long long)j * lda + 4 * ch);
    const uint2 l = ld_a<POL>(lo + (long long)j * lda + 4 * ch);
    return make_uint4(h.x, h.y, l.x, l.y);
  }
  __device__ static __forceinline__ float4 expand(raw_t v) {
    // hi + lo is exact in FP32 (lo is the bf16 rounding of the FP32 remainder)
    float4 o;
    o.x = bf16_to_f32(v.x & 0xffffu) + bf16_to_f32(v.z & 0xffffu);
    o.y = bf16_to_f32(v.x >> 16) + bf16_to_f32(v.z >> 16);
    o.z = bf16_to_f32(v.y & 0xffffu) + bf16_to_f32(v.w & 0xffffu);
    o.w = bf16_to_f32(v.y >> 16) + bf16_to_f32(v.w >> 16);
    return o;
  }
  __device__ __forceinline__ float4 load(int j, int ch) const { return expand(fetch(j, ch)); }
};

template <int POL> struct ALoader<FMT_BF16HI, POL> {
  const uint16_t* hi;
  long long lda;
  __device__ ALoader(const ColArgs& a, int k)
      : hi(static_cast<const uint16_t*>(a.A) + (long long)k * a.sA), lda(a.lda) {}
  __device__ ALoader(const AUArgs& a, int k)
      : hi(static_cast<const uint16_t*>(a.A) + (long long)k * a.sA), lda(a.lda) {}
  typedef uint2 raw_t;
  __device__ __forceinline__ raw_t fetch(int j, int ch) const { return ld_a<POL>(hi + (long long)j * lda + 4 * ch); }
  __device__ static __forceinline__ float4 expand(raw_t h) {
    return make_float4(bf16_to_f32(h.x & 0xffffu), bf16_to_f32(h.x >> 16),
                       bf16_to_f32(h.y & 0xffffu), bf16_to_f32(h.y >> 16));
  }
  __device__ __forceinline__ float4 load(int j, int ch) const { return expand(fetch(j, ch)); }
};

// Philox form: element (i, j) of A_k is word i % 4 of Philox4x32-10 (Salmon et
// al., SC'11) at counter (i / 4, j, k, 0) with key (seed low, seed high),
// turned into a normal deviate by the inverse-CDF table in LDS: with
// v = (2 (x & 0x7fffffff) + 1) 2^-33, idx from the exponent and the top six
// mantissa bits of v, t from the other 17, |z| = T[idx] + (T[idx+1] - T[idx]) t
// and the sign from the top bit of x.  Every operation is a correctly rounded
// conversion or a non-contracted add/sub/mul, so the host definition gives the
// same bits.
__device__ __forceinline__ void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    // one 32 x 32 -> 64-bit multiply per product (v_mad_u64_u32) gives both halves
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0, n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = (uint32_t)p1;
    c[2] = n2;
    c[3] = (uint32_t)p0;
  }
}

__device__ __forceinline__ float word_to_normal(uint32_t x, const float* tab) {
#pragma clang fp contract(off)   // the definition rounds after the multiply and after the add
  const uint32_t w = x & 0x7fffffffu;
  const float v = (float)(2u * w + 1u) * 0x1p-33f;
  const uint32_t bits = __float_as_uint(v);
  const int idx = ((int)(bits >> 23) - (127 - 33)) * 64 + (int)((bits & 0x7fffffu) >> 17);
  const float t = (float)(bits & 0x1ffffu) * 0x1p-17f;
  const float lo = tab[idx], hi = tab[idx + 1];
  const float d = hi - lo;
  const float z = lo + d * t;
  return (x >> 31) ? -z : z;
}

template <int POL> struct ALoader<FMT_PHILOX, POL> {   // generated, not loaded: POL has no effect
  uint32_t k0, k1, col;
  const float* tab;   // LDS copy of the normal table, set by the kernel
  __device__ ALoader(const ColArgs& a, int k)
      : k0((uint32_t)a.seed), k1((uint32_t)(a.seed >> 32)), col((uint32_t)k), tab(nullptr) {}
  __device__ ALoader(const AUArgs& a, int k)
      : k0((uint32_t)a.seed), k1((uint32_t)(a.seed >> 32)), col((uint32_t)k), tab(nullptr) {}
  typedef float4 raw_t;   // generated, not loaded: fetch() does the work
  __device__ __forceinline__ raw_t fetch(int j, int ch) const {
    uint32_t c[4] = {(uint32_t)ch, (uint32_t)j, col, 0u};
    philox4x32_10(c, k0, k1);
    return make_float4(word_to_normal(c[0], tab), word_to_normal(c[1], tab), word_to_normal(c[2], tab),
                       word_to_normal(c[3], tab));
  }
  __device__ static __forceinline__ float4 expand(raw_t v) { return v; }
  __device__ __forceinline__ float4 load(int j, int ch) const { return fetch(j, ch); }
};

// Zero the components of a 4-row chunk that lie at or beyond row m (nv = valid rows, 0..4).
__device__ __forceinline__ float4 mask_rows(float4 v, int nv) {
  v.x = nv > 0 ? v.x : 0.f;
  v.y = nv > 1 ? v.y : 0.f;
  v.z = nv > 2 ? v.z : 0.f;
  v.w = nv > 3 ? v.w : 0.f;
  return v;
}

__device__ __forceinline__ float dot4(float4 a, float4 b) {
  return fmaf(a.w, b.w, fmaf(a.z, b.z, fmaf(a.y, b.y, a.x * b.x)));
}
__device__ __forceinline__ float4 axpy4(float s, float4 x, float4 y) {
  return make_float4(fmaf(s, x.x, y.x), fmaf(s, x.y, y.y), fmaf(s, x.z, y.z), fmaf(s, x.w, y.w));
}
__device__ __forceinline__ float4 add4(float4 a, float4 b) {
  return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
}
__device__ __forceinline__ float4 sub4(float4 a, float4 b) {
  return make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w);
}
__device__ __forceinline__ float get4(float4 v, int e) {
  return e == 0 ? v.x : (e == 1 ? v.y : (e == 2 ? v.z : v.w));
}

// G^{-1} of an SPD r x r FP64 matrix G (row-major, r <= 16) by Gauss-Jordan
// elimination without pivoting (an SPD matrix has positive pivots and needs
// none), by one wave with no barriers: the wave's LDS accesses complete in
// order, and each step reads every entry it needs before it writes.  W (LDS,
// 2 r^2 doubles) holds [G | I]; step k scales row k by 1 / W[k][k] and takes
// W[i][k] times it from every other row; the right half ends as G^{-1}, copied
// to Ginv.  Returns false, with the identity in Ginv, when a pivot is not
// positive (or not a number); the result is the same on every lane.  One
// reciprocal per step and a chain of r steps, with the other waves idle: the
// A_k U launch at n = q = 1000, m = 400, r = 10 went from 0.269 to 0.262 ms
// against a workgroup-wide Cholesky with two triangular solves (which chain r
// square roots and 3r divisions under barriers).
__device__ inline bool wave_spd_inverse(const double* G, double* W, double* Ginv, int r) {
  const int lane = threadIdx.x & 63, w2 = 2 * r, ne = r * w2;   // ne <= 512: at most 8 entries per lane
  for (int e = lane; e < ne; e += 64) {
    const int i = e / w2, c = e - i * w2;
    W[e] = c < r ? G[i * r + c] : (c - r == i ? 1.0 : 0.0);
  }
  bool ok = true;
  for (int k = 0; k < r && ok; ++k) {
    const double piv = W[k * w2 + k];
    if (!(piv > 0.0)) {
      ok = false;
      break;
    }
    const double inv = 1.0 / piv;
    double nv[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int e = lane + 64 * t;
      nv[t] = 0.0;
      if (e < ne) {
        const int i = e / w2, c = e - i * w2;
        const double rk = W[k * w2 + c] * inv;   // the new row k
        nv[t] = i == k ? rk : fma(-W[i * w2 + k], rk, W[e]);
      }
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int e = lane + 64 * t;
      if (e < ne) W[e] = nv[t];
    }
  }
  for (int e = lane; e < r * r; e += 64) {
    const int i = e / r, c = e - i * r;
    Ginv[e] = ok ? W[i * w2 + r + c] : (i == c ? 1.0 : 0.0);
  }
  return ok;
}

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

// LDS layout of the column kernel in bytes; used by the host to size the
// launch and by the kernel to carve its dynamic shared memory.
constexpr size_t kPInLdsMax = 32 * 1024;   // P_k is staged in LDS up to this size

struct ColLayout {
  size_t ginv, P, wpart, g, sd, inT, Ti, Tv, red, hist, cbuf, tab, total;
  int mq, p_in_lds;
  // waves: waves of the column workgroup (its per-wave partial vectors and sums)
  __host__ __device__ ColLayout(int n, int m, int r, int rho, int project, int philox = 0, int waves = kWaves) {
    mq = ((m + 3) / 4) * 4;
    p_in_lds = 4 * (size_t)m * r <= kPInLdsMax;
    size_t o = 0;
    ginv = o; o = align16(o + (project ? 8 * (size_t)r * r : 0));
    P = o;    o = align16(o + (project && p_in_lds ? 4 * (size_t)m * r : 0));
    wpart = o; o = align16(o + 4 * (size_t)waves * mq);
    g = o;    o = align16(o + 4 * (size_t)n);
    sd = o;   o = align16(o + 4 * (size_t)n);
    inT = o;  o = align16(o + 4 * (size_t)((n + 31) / 32));
    Ti = o;   o = align16(o + 4 * (size_t)rho);
    Tv = o;   o = align16(o + 4 * (size_t)rho);
    red = o;  o = align16(o + 8 * 2 * (size_t)waves);
    hist = o; o = align16(o + 4 * (256 + 8));
    cbuf = o; o = align16(o + 8 * kRMax);
    tab = o;  o = align16(o + (philox ? 4 * (size_t)kNormalTable : 0));
    total = o;
  }
};

// LDS layout of the A_k U kernel.
struct AULayout {
  size_t P, gpart, G, W, Gi, tab, total;
  int p_in_lds, mp;
  __host__ __device__ AULayout(int m, int r, int philox = 0, int waves = kWaves) {
    mp = ((m + 3) / 4) * 4 + 4;                     // LDS row stride of the column-major P
    p_in_lds = 4 * (size_t)mp * r <= kPInLdsMax;
    const size_t ust = 4 * (size_t)waves * 64 * ((((r + 1) / 2 * 2) + 3) / 4 * 4);   // staged rows of U
    const size_t pb = p_in_lds ? 4 * (size_t)mp * r : 0;
    size_t o = 0;
    P = o;     o = align16(o + (pb > ust ? pb : ust));
    gpart = o; o = align16(o + 4 * 8 * (size_t)kThreads);
    G = o;     o = align16(o + 8 * (size_t)r * r);
    W = o;     o = align16(o + 16 * (size_t)r * r);   // [G | I], r x 2r, for the inverse
    Gi = o;    o = align16(o + 8 * (size_t)r * r);
    tab = o;   o = align16(o + (philox ? 4 * (size_t)kNormalTable : 0));
    total = o;
  }
};

}  // namespace altg
