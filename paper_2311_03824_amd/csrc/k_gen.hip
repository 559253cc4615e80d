// Synthetic instances made on the device (input generation; none of Alg. 1).
//
//  k_make_a : the canonical measurement matrices of the synthetic workloads.  The
//             draw a of element (i, j) of A_k is the Philox form's value (counter
//             (i / 4, j, k, 0), table normal transform); the stored matrix is
//             A = hi + lo with hi = bf16_RN(a), lo = bf16_RN(a - hi), which is
//             exact in FP32, so an FP32 plane and a BF16 hi/lo pair hold the same A.
//  k_measure: y_k = A_k x_k for the measurement model of Sec. 1.1, accumulated in
//             FP64 in index order j = 0..n-1 and rounded once to FP32.
#include "common.h"
#include "launch.h"

namespace altg {

// Round-to-nearest-even of an FP32 value to bfloat16 (bit pattern).  NaN is kept
// quiet; the draws here are always finite.
__device__ __forceinline__ uint32_t f32_to_bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

// One thread per 4-row chunk of one column j of one A_k; chunks run over lda / 4
// so the padding rows m..lda-1 are written as zeros.
__global__ __launch_bounds__(256) void k_make_a(unsigned long long seed, const float* table, int q, int n, int m,
                                                long long lda, int fmt, float* A32, uint16_t* hi, uint16_t* lo) {
  __shared__ float tab[kNormalTable];
  for (int t = threadIdx.x; t < kNormalTable; t += blockDim.x) tab[t] = table[t];
  __syncthreads();
  const int nch = (int)(lda / 4);
  const long long total = (long long)q * n * nch;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    const int ch = (int)(e % nch);
    const long long jk = e / nch;               // = k * n + j
    const int j = (int)(jk % n);
    const int k = (int)(jk / n);
    uint32_t c[4] = {(uint32_t)ch, (uint32_t)j, (uint32_t)k, 0u};
    philox4x32_10(c, k0, k1);
    uint32_t h[4], l[4];
    float v[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const float a = (4 * ch + w < m) ? word_to_normal(c[w], tab) : 0.f;
      h[w] = f32_to_bf16_rne(a);
      const float hv = __uint_as_float(h[w] << 16);
      l[w] = f32_to_bf16_rne(a - hv);           // a - hi is exact in FP32
      v[w] = hv + __uint_as_float(l[w] << 16);  // exact as well
    }
    const long long off = jk * lda + 4 * (long long)ch;
    if (fmt == FMT_F32) {
      *reinterpret_cast<float4*>(A32 + off) = make_float4(v[0], v[1], v[2], v[3]);
    } else {
      *reinterpret_cast<uint2*>(hi + off) = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
      *reinterpret_cast<uint2*>(lo + off) = make_uint2(l[0] | (l[1] << 16), l[2] | (l[3] << 16));
    }
  }
}

hipError_t launch_make_a(unsigned long long seed, const float* table, int q, int n, int m, long long lda, int fmt,
                         float* A32, uint16_t* hi, uint16_t* lo, hipStream_t st) {
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  hipLaunchKernelGGL(k_make_a, dim3(4096), dim3(256), 0, st, seed, table, q, n, m, lda, fmt, A32, hi, lo);
  return hipGetLastError();
}

// Element (i..i+3, j) of A_k in the stored formats; rows beyond m are masked by
// the caller.
template <int FMT>
__device__ __forceinline__ float4 gen_load(const MeasureArgs& a, int k, int j, int ch, const float* tab) {
  if constexpr (FMT == FMT_F32) {
    return *reinterpret_cast<const float4*>(static_cast<const float*>(a.A) + k * a.sA + j * a.lda + 4 * ch);
  } else if constexpr (FMT == FMT_BF16X2) {
    const long long off = k * a.sA + j * a.lda + 4 * ch;
    const uint2 h = *reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(a.A) + off);
    const uint2 l = *reinterpret_cast<const uint2*>(static_cast<const uint16_t*>(a.Alo) + off);
    return make_float4(bf16_to_f32(h.x & 0xffffu) + bf16_to_f32(l.x & 0xffffu),
                       bf16_to_f32(h.x >> 16) + bf16_to_f32(l.x >> 16),
                       bf16_to_f32(h.y & 0xffffu) + bf16_to_f32(l.y & 0xffffu),
                       bf16_to_f32(h.y >> 16) + bf16_to_f32(l.y >> 16));
  } else {
    uint32_t c[4] = {(uint32_t)ch, (uint32_t)j, (uint32_t)k, 0u};
    philox4x32_10(c, (uint32_t)a.seed, (uint32_t)(a.seed >> 32));
    return make_float4(word_to_normal(c[0], tab), word_to_normal(c[1], tab), word_to_normal(c[2], tab),
                       word_to_normal(c[3], tab));
  }
}

// Block (x: 256-row slab, y: column k); thread t holds rows 4 (64 x + t) .. + 3.
template <int FMT>
__global__ __launch_bounds__(64) void k_measure(MeasureArgs a) {
  __shared__ float tab[FMT == FMT_PHILOX ? kNormalTable : 1];
  if constexpr (FMT == FMT_PHILOX) {
    for (int t = threadIdx.x; t < kNormalTable; t += blockDim.x) tab[t] = a.table[t];
    __syncthreads();
  }
  const int k = blockIdx.y;
  const int ch = blockIdx.x * 64 + threadIdx.x;
  if (4 * ch >= a.m) return;
  const int nv = a.m - 4 * ch < 4 ? a.m - 4 * ch : 4;
  const double* x = a.Xt + (long long)k * a.n;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
  for (int j = 0; j < a.n; ++j) {
    const float4 v = gen_load<FMT>(a, k, j, ch, tab);
    const double xj = x[j];
    acc[0] = fma((double)v.x, xj, acc[0]);
    acc[1] = fma((double)v.y, xj, acc[1]);
    acc[2] = fma((double)v.z, xj, acc[2]);
    acc[3] = fma((double)v.w, xj, acc[3]);
  }
  float* y = a.Y + (long long)k * a.ldy + 4 * ch;
  for (int e = 0; e < nv; ++e) y[e] = (float)acc[e];
}

hipError_t launch_measure(int fmt, const MeasureArgs& a, hipStream_t st) {
  const dim3 grid((a.m + 255) / 256, a.q);
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  if (fmt == FMT_F32) hipLaunchKernelGGL(k_measure<FMT_F32>, grid, dim3(64), 0, st, a);
  else if (fmt == FMT_BF16X2) hipLaunchKernelGGL(k_measure<FMT_BF16X2>, grid, dim3(64), 0, st, a);
  else hipLaunchKernelGGL(k_measure<FMT_PHILOX>, grid, dim3(64), 0, st, a);
  return hipGetLastError();
}

}  // namespace altg
