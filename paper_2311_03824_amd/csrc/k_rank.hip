// Automatic rank of Sec. 2.6 on the GPU (gfx950).
//
// The rank r is the smallest k whose k leading singular values of L_0 hold a
// fraction `energy` (65 % in the paper) of the energy sum_i sigma_i^2 of the
// first K = max(1, floor(min(n, q, m) / 10)).  The K values come from a block
// subspace iteration on L_0 (n x q, given as L_0^T, q x n row-major) with
// b = K + p columns (p <= 8 extra columns speed up the trailing values), each
// step Z = L_0 (L_0^T U) followed by CholeskyQR2 (FP64 Gram, Cholesky and
// R^{-1}), then a Rayleigh-Ritz step: the eigenvalues of M = T^T T, T = L_0^T U,
// are the squared Ritz values, found by a parallel cyclic Jacobi (round-robin
// pairs, all b/2 rotations of a round at once).
//
// Kernels: k_rank_mm (C = A B or A^T B, FP32 tiles staged in LDS), k_rank_gram
// (W = X^T X in FP64), k_rank_chol (one workgroup: W = R^T R, R^{-1}),
// k_rank_jacobi (one workgroup: eigenvalues, their order, the rank).  Every
// reduction runs in a fixed order, so results do not depend on timing.
#include "common.h"
#include "launch.h"

namespace altg {

namespace {

constexpr int kTile = 32;       // output tile of k_rank_mm (kTile x kTile), 256 threads x 4 outputs
constexpr int kKc = 32;         // contraction chunk staged in LDS
constexpr int kGT = 16;         // tile of k_rank_gram (kGT x kGT entries, one per thread)
constexpr int kGRows = 64;      // rows per LDS stage of k_rank_gram

// C (M x N, row-major, ldc) = A' B with A' = A (M x K, row-major lda) or, with
// TRANS, A' = A^T where A is K x M row-major (lda); B is K x N row-major (ldb).
// Each thread accumulates 4 outputs of its column in FP32 over the chunks in order.
template <bool TRANS>
__global__ __launch_bounds__(256) void k_rank_mm(const float* __restrict__ A, long long lda,
                                                 const float* __restrict__ B, long long ldb, float* __restrict__ C,
                                                 long long ldc, int M, int N, int K) {
  __shared__ float sa[kKc][kTile + 1];   // sa[kk][i] = A'(i0 + i, k0 + kk)
  __shared__ float sb[kKc][kTile + 1];   // sb[kk][c] = B(k0 + kk, c0 + c)
  const int tid = threadIdx.x;
  const int i0 = blockIdx.y * kTile, c0 = blockIdx.x * kTile;
  const int tc = tid & (kTile - 1), ti = (tid >> 5) * 4;   // this thread: column tc, rows ti .. ti + 3
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += kKc) {
    for (int e = tid; e < kKc * kTile; e += 256) {
      const int kk = e / kTile, x = e % kTile;
      // A' tile: consecutive threads read consecutive addresses (along k for A, along i for A^T)
      const int ii = TRANS ? x : e / kKc;
      const int kx = TRANS ? kk : e % kKc;
      const int gi = i0 + ii, gk = k0 + kx;
      float v = 0.f;
      if (gi < M && gk < K) v = TRANS ? A[(long long)gk * lda + gi] : A[(long long)gi * lda + gk];
      sa[kx][ii] = v;
      const int bk = k0 + kk, bc = c0 + x;
      sb[kk][x] = (bk < K && bc < N) ? B[(long long)bk * ldb + bc] : 0.f;
    }
    __syncthreads();
#pragma unroll 8
    for (int kk = 0; kk < kKc; ++kk) {
      const float b = sb[kk][tc];
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[e] = fmaf(sa[kk][ti + e], b, acc[e]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int gi = i0 + ti + e, gc = c0 + tc;
    if (gi < M && gc < N) C[(long long)gi * ldc + gc] = acc[e];
  }
}

// W (b x b, FP64) = X^T X for X (rows x b, row-major): one entry per thread,
// rows summed in order in FP64.
__global__ __launch_bounds__(kGT * kGT) void k_rank_gram(const float* __restrict__ X, int rows, int b,
                                                         double* __restrict__ W) {
  __shared__ float sx[kGRows][2 * kGT + 1];
  const int tid = threadIdx.x, ta = tid / kGT, tb = tid % kGT;
  const int a0 = blockIdx.y * kGT, b0 = blockIdx.x * kGT;
  double s = 0.0;
  for (int j0 = 0; j0 < rows; j0 += kGRows) {
    for (int e = tid; e < kGRows * 2 * kGT; e += kGT * kGT) {
      const int jj = e / (2 * kGT), cc = e % (2 * kGT);
      const int c = cc < kGT ? a0 + cc : b0 + cc - kGT;
      sx[jj][cc] = (j0 + jj < rows && c < b) ? X[(long long)(j0 + jj) * b + c] : 0.f;
    }
    __syncthreads();
    const int lim = min(kGRows, rows - j0);
    for (int jj = 0; jj < lim; ++jj) s = fma((double)sx[jj][ta], (double)sx[jj][kGT + tb], s);
    __syncthreads();
  }
  const int ga = a0 + ta, gb = b0 + tb;
  if (ga < b && gb < b) W[(long long)ga * b + gb] = s;
}

// One workgroup: W = R^T R (R upper triangular, positive diagonal) in LDS, then
// X = R^{-1} (FP64 in Xinv, FP32 copy in Xf for the next product).  A pivot at
// or below 1e-13 times the largest diagonal of W (a numerically rank-deficient
// block) is replaced by 1 with a zero row, so the factor stays finite; flag
// bit 0 records it.
__global__ __launch_bounds__(256) void k_rank_chol(const double* __restrict__ W, int b, double* __restrict__ Xinv,
                                                   float* __restrict__ Xf, int* __restrict__ flag) {
  extern __shared__ double sw[];   // b x b
  const int tid = threadIdx.x;
  for (int e = tid; e < b * b; e += 256) sw[e] = W[e];
  __shared__ double dmax;
  __syncthreads();
  if (tid == 0) {
    double mx = 0.0;
    for (int i = 0; i < b; ++i) mx = fmax(mx, sw[i * b + i]);
    dmax = mx;
  }
  __syncthreads();
  const double floor_d = 1e-13 * dmax;
  bool deficient = false;
  for (int k = 0; k < b; ++k) {
    const double d = sw[k * b + k];
    const bool ok = d > floor_d && isfinite(d);
    deficient |= !ok;
    const double rkk = ok ? sqrt(d) : 1.0;
    __syncthreads();   // every thread has read the pivot
    for (int j = k + 1 + tid; j < b; j += 256) sw[k * b + j] = ok ? sw[k * b + j] / rkk : 0.0;
    if (tid == 0) sw[k * b + k] = rkk;
    __syncthreads();
    // trailing update of the upper triangle: W[i][j] -= R[k][i] R[k][j], k < i <= j
    const int t = b - k - 1;
    for (int e = tid; e < t * t; e += 256) {
      const int i = k + 1 + e / t, j = k + 1 + e % t;
      if (j >= i) sw[i * b + j] -= sw[k * b + i] * sw[k * b + j];
    }
    __syncthreads();
  }
  if (tid == 0 && deficient) atomicOr(flag, 1);
  // R^{-1}: column c by back substitution (thread c), rows c .. 0 in order
  for (int c = tid; c < b; c += 256) {
    for (int i = b - 1; i >= 0; --i) {
      double v = 0.0;
      if (i <= c) {
        v = (i == c) ? 1.0 : 0.0;
        for (int l = i + 1; l <= c; ++l) v -= sw[i * b + l] * Xinv[(long long)l * b + c];
        v /= sw[i * b + i];
      }
      Xinv[(long long)i * b + c] = v;
    }
  }
  __syncthreads();
  for (int e = tid; e < b * b; e += 256) Xf[e] = (float)Xinv[e];
}

// One workgroup: eigenvalues of the symmetric b x b matrix M (FP64) by cyclic
// Jacobi with round-robin pairs (b - 1 rounds of b / 2 disjoint rotations per
// sweep, odd b padded with an idle index), until the off-diagonal mass is at
// most 1e-28 of the diagonal mass or 40 sweeps.  Then the eigenvalues in
// descending order, sv[i] = sqrt(max(lambda_i, 0)) for i < K, and the rank:
// the smallest k with sum_{i<k} lambda_i >= energy * sum_{i<K} lambda_i
// (sums in index order, FP64).
__global__ __launch_bounds__(256) void k_rank_jacobi(const double* __restrict__ Mg, int b, int K, double energy,
                                                     double* __restrict__ sv, int* __restrict__ r_out) {
  extern __shared__ double sm[];              // b x b, then the rotations (c, s) of a round
  double* cs = sm + b * b;                    // 2 * (b / 2 + 1)
  __shared__ double red[2][4];
  __shared__ int stop;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int e = tid; e < b * b; e += 256) sm[e] = Mg[e];
  const int bp = b + (b & 1), np = bp / 2;    // players (with an idle one when b is odd), pairs per round
  __syncthreads();
  for (int sweep = 0; sweep < 40; ++sweep) {
    // convergence test: off-diagonal and diagonal mass
    double off = 0.0, dg = 0.0;
    for (int e = tid; e < b * b; e += 256) {
      const int i = e / b, j = e % b;
      const double v = sm[e] * sm[e];
      if (i == j) dg += v;
      else off += v;
    }
    off = wave_sum(off);
    dg = wave_sum(dg);
    if (lane == 0) {
      red[0][wave] = off;
      red[1][wave] = dg;
    }
    __syncthreads();
    if (tid == 0) {
      const double o = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
      const double d = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
      stop = (o <= 1e-28 * d || o == 0.0) ? 1 : 0;
    }
    __syncthreads();
    if (stop) break;
    for (int rd = 0; rd < bp - 1; ++rd) {
      // pair i of this round: positions i and bp - 1 - i of the circle (position 0 fixed)
      auto player = [&](int pos) { return pos == 0 ? 0 : (pos - 1 + rd) % (bp - 1) + 1; };
      for (int i = tid; i < np; i += 256) {
        int p = player(i), q = player(bp - 1 - i);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        double c = 1.0, s = 0.0;
        if (q < b) {
          const double apq = sm[p * b + q];
          if (apq != 0.0) {
            const double theta = (sm[q * b + q] - sm[p * b + p]) / (2.0 * apq);
            const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        }
        cs[2 * i] = c;
        cs[2 * i + 1] = s;
      }
      __syncthreads();
      // rows p, q of every pair
      for (int e = tid; e < np * b; e += 256) {
        const int i = e / b, k = e % b;
        int p = player(i), q = player(bp - 1 - i);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        if (q >= b) continue;
        const double c = cs[2 * i], s = cs[2 * i + 1];
        const double xp = sm[p * b + k], xq = sm[q * b + k];
        sm[p * b + k] = c * xp - s * xq;
        sm[q * b + k] = s * xp + c * xq;
      }
      __syncthreads();
      // columns p, q of every pair
      for (int e = tid; e < np * b; e += 256) {
        const int i = e / b, k = e % b;
        int p = player(i), q = player(bp - 1 - i);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        if (q >= b) continue;
        const double c = cs[2 * i], s = cs[2 * i + 1];
        const double xp = sm[k * b + p], xq = sm[k * b + q];
        sm[k * b + p] = c * xp - s * xq;
        sm[k * b + q] = s * xp + c * xq;
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    // eigenvalues (the diagonal) in descending order, by selection
    double* lam = cs;   // reuse: b values
    for (int i = 0; i < b; ++i) lam[i] = sm[i * b + i];
    for (int i = 0; i < b; ++i) {
      int best = i;
      for (int j = i + 1; j < b; ++j)
        if (lam[j] > lam[best]) best = j;
      const double t = lam[i];
      lam[i] = lam[best];
      lam[best] = t;
    }
    const int kk = K < b ? K : b;
    double tot = 0.0;
    for (int i = 0; i < kk; ++i) tot += fmax(lam[i], 0.0);
    double cum = 0.0;
    int r = kk;
    for (int i = 0; i < kk; ++i) {
      cum += fmax(lam[i], 0.0);
      if (cum >= energy * tot) {
        r = i + 1;
        break;
      }
    }
    for (int i = 0; i < kk; ++i) sv[i] = sqrt(fmax(lam[i], 0.0));
    *r_out = r;
  }
}

// The real embedding of a complex L_0 = X + iY (n x q), given as L0t (q x n
// complex, L0t[k][j] = L_0[j][k]): E = [[X, -Y], [Y, X]] (2n x 2q), written as its
// transpose Et (2q x 2n, row-major).  The singular values of E are those of L_0,
// each twice.
__global__ void k_rank_embed(const float2* __restrict__ L0t, int q, int n, float* __restrict__ Et) {
  const long long n2 = 2LL * n;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < (long long)q * n;
       e += (long long)gridDim.x * blockDim.x) {
    const long long k = e / n, j = e % n;
    const float2 v = L0t[e];
    Et[k * n2 + j] = v.x;
    Et[k * n2 + n + j] = v.y;
    Et[(q + k) * n2 + j] = -v.y;
    Et[(q + k) * n2 + n + j] = v.x;
  }
}

// U (n x r, row-major) = the first r columns of Ub (n x b, row-major).
__global__ void k_rank_slice(const float* __restrict__ Ub, int n, int b, int r, float* __restrict__ U) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < (long long)n * r;
       e += (long long)gridDim.x * blockDim.x) {
    const long long j = e / r;
    const int c = (int)(e % r);
    U[e] = Ub[j * b + c];
  }
}

}  // namespace

size_t rank_lds_bytes(int b) { return (size_t)b * b * sizeof(double) + 2 * (size_t)(b / 2 + 2) * sizeof(double); }

hipError_t launch_rank_mm(bool trans, const float* A, long long lda, const float* B, long long ldb, float* C,
                          long long ldc, int M, int N, int K, hipStream_t st) {
  (void)hipGetLastError();
  const dim3 grid((N + kTile - 1) / kTile, (M + kTile - 1) / kTile);
  if (trans) hipLaunchKernelGGL(k_rank_mm<true>, grid, dim3(256), 0, st, A, lda, B, ldb, C, ldc, M, N, K);
  else hipLaunchKernelGGL(k_rank_mm<false>, grid, dim3(256), 0, st, A, lda, B, ldb, C, ldc, M, N, K);
  return hipGetLastError();
}

hipError_t launch_rank_gram(const float* X, int rows, int b, double* W, hipStream_t st) {
  (void)hipGetLastError();
  const dim3 grid((b + kGT - 1) / kGT, (b + kGT - 1) / kGT);
  hipLaunchKernelGGL(k_rank_gram, grid, dim3(kGT * kGT), 0, st, X, rows, b, W);
  return hipGetLastError();
}

hipError_t launch_rank_chol(const double* W, int b, double* Xinv, float* Xf, int* flag, hipStream_t st) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_rank_chol, dim3(1), dim3(256), (size_t)b * b * sizeof(double), st, W, b, Xinv, Xf, flag);
  return hipGetLastError();
}

hipError_t launch_rank_jacobi(const double* M, int b, int K, double energy, double* sv, int* r_out,
                              hipStream_t st) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_rank_jacobi, dim3(1), dim3(256), rank_lds_bytes(b), st, M, b, K, energy, sv, r_out);
  return hipGetLastError();
}

hipError_t launch_rank_embed(const float* L0t, int q, int n, float* Et, hipStream_t st) {
  (void)hipGetLastError();
  long long g = ((long long)q * n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_rank_embed, dim3((unsigned)g), dim3(256), 0, st, reinterpret_cast<const float2*>(L0t), q, n, Et);
  return hipGetLastError();
}

hipError_t launch_rank_slice(const float* Ub, int n, int b, int r, float* U, hipStream_t st) {
  (void)hipGetLastError();
  long long g = ((long long)n * r + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_rank_slice, dim3((unsigned)g), dim3(256), 0, st, Ub, n, b, r, U);
  return hipGetLastError();
}

}  // namespace altg
