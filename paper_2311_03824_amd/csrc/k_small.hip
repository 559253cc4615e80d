// Reductions across columns and the U update of AltGDmin-LR+S for gfx950.
//
//  k_grad  : partials of grad_U f = sum_k h_k b_k^T (Sec. 2.1) over KS column
//            splits, each summed in a fixed order (deterministic, no atomics).
//            The same kernel forms Z = L_0 (L_0^T U) in the subspace iteration.
//  k_ltu   : T = L_0^T U for the subspace iteration (one wave per column).
//  k_qr    : one workgroup: sums the partials, sets eta = eta_c / ||grad||_2 at
//            t = 1 (Sec. 2.6), forms U - eta grad and re-orthonormalises it by
//            CholeskyQR2 (FP64 Gram and Cholesky, positive-diagonal R), the QR of
//            the projected GD step in Alg. 1; also the subspace-iteration
//            orthonormalisation and the residual monitor.
#include <mutex>

#include "launch.h"

namespace altg {

// One workgroup of 16 waves per block of 64 rows j; wave w sums the columns
// k = w, w + 16, ... of its split; the 16 wave partials are added in a fixed
// pairwise order.  Row k of B is fetched by lanes 0..r-1 with one vector load
// and broadcast with readlane, so that loads of later columns stay in flight.
__device__ __forceinline__ void grad_body(const float* __restrict__ H, const float* __restrict__ B, int n, int q, int r,
                                          int KS, float* __restrict__ gpart, int jblock, int ks,
                                          float (*red)[64][kRMax + 1]) {
  const int lane = threadIdx.x & 63, ph = wave_id();
  const int j = jblock * 64 + lane;
  const int jc = j < n ? j : n - 1;
  const int k0 = (int)((long long)q * ks / KS), k1 = (int)((long long)q * (ks + 1) / KS);
  float acc[kRMax];
#pragma unroll
  for (int c = 0; c < kRMax; ++c) acc[c] = 0.f;
  constexpr int KU = 16;   // loads in flight per wave; the order of the k terms does not depend on it
  for (int kb = k0 + ph; kb < k1; kb += kGradWaves * KU) {
    float h[KU], bv[KU];
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int k = kb + u * kGradWaves;
      const int kc = k < k1 ? k : k0;
      h[u] = H[(long long)kc * n + jc];
      bv[u] = B[(long long)kc * r + (lane < r ? lane : 0)];
    }
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const bool ok = kb + u * kGradWaves < k1;
      const float hu = ok ? h[u] : 0.f;
#pragma unroll
      for (int c = 0; c < kRMax; ++c)
        if (c < r) acc[c] = fmaf(hu, __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bv[u]), c)), acc[c]);
    }
  }
  // pairwise tree over the waves in a fixed order: (w, w + h) for h = 8, 4, 2, 1
  for (int hh = kGradWaves / 2; hh >= 1; hh >>= 1) {
    if (ph >= hh && ph < 2 * hh)
#pragma unroll
      for (int c = 0; c < kRMax; ++c) red[ph - hh][lane][c] = acc[c];
    __syncthreads();
    if (ph < hh)
#pragma unroll
      for (int c = 0; c < kRMax; ++c) acc[c] += red[ph][lane][c];
    __syncthreads();
  }
  if (ph == 0 && j < n)
    for (int c = 0; c < r; ++c) gpart[((long long)ks * n + j) * r + c] = acc[c];
}

__global__ __launch_bounds__(kGradWaves * 64) void k_grad(const float* __restrict__ H, const float* __restrict__ B,
                                                          int n, int q, int r, int KS, float* __restrict__ gpart,
                                                          const int* skip) {
  if (skip && *skip) return;
  __shared__ float red[kGradWaves / 2][64][kRMax + 1];
  grad_body(H, B, n, q, r, KS, gpart, blockIdx.x, blockIdx.y, red);
}

// Several problems in one launch: block b is (problem, row block, split) = map[b].
__global__ __launch_bounds__(kGradWaves * 64) void k_grad_grp(const GradArgs* tab, const int4* map) {
  __shared__ float red[kGradWaves / 2][64][kRMax + 1];
  const int4 mp = map[blockIdx.x];
  const GradArgs a = tab[mp.x];
  if (a.skip && *a.skip) return;
  grad_body(a.H, a.B, a.n, a.q, a.r, a.KS, a.gpart, mp.y, mp.z, red);
}

__global__ __launch_bounds__(256) void k_ltu(const float* __restrict__ L0t, const float* __restrict__ U, int n,
                                             int q, int r, float* __restrict__ T, const int* skip) {
  if (skip && *skip) return;
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * kWaves + wave_id();
  if (k >= q) return;
  float acc[kRMax];
#pragma unroll
  for (int c = 0; c < kRMax; ++c) acc[c] = 0.f;
  for (int j = lane; j < n; j += 64) {
    const float l = L0t[(long long)k * n + j];
#pragma unroll
    for (int c = 0; c < kRMax; ++c)
      if (c < r) acc[c] = fmaf(l, U[(long long)j * r + c], acc[c]);
  }
#pragma unroll
  for (int c = 0; c < kRMax; ++c) {
    if (c < r) {
      const float s = wave_sum(acc[c]);
      if (lane == 0) T[(long long)k * r + c] = s;
    }
  }
}

// C = X^T Y (r x r, FP64) over n rows of the n x r row-major X and Y; block-wide.
__device__ void block_gram(const float* X, const float* Y, int n, int r, double* C, bool sym) {
  // C = X^T Y (r x r, FP64) over the n rows of X and Y (row-major n x r).  Wave
  // w computes the entries e = w, w + 16, ... (with sym, the entries a <= b only,
  // mirrored); its lanes stride over the rows and the 64 lane sums are added by
  // the fixed DPP tree, so the result does not depend on timing.
  const int lane = threadIdx.x & 63, wave = wave_id();
  const int E = sym ? r * (r + 1) / 2 : r * r;
  for (int e = wave; e < E; e += kQRThreads / 64) {
    int ra = 0, rb = 0;
    if (sym) {
      int base = 0;
      while (e >= base + (r - ra)) {
        base += r - ra;
        ++ra;
      }
      rb = ra + (e - base);
    } else {
      ra = e / r;
      rb = e - ra * r;
    }
    double s = 0.0;
    for (int j = lane; j < n; j += 64) s = fma((double)X[(long long)j * r + ra], (double)Y[(long long)j * r + rb], s);
    s = wave_sum_dpp(s);
    if (lane == 0) {
      C[ra * r + rb] = s;
      if (sym) C[rb * r + ra] = s;
    }
  }
  __syncthreads();
}

// Largest eigenvalue of a symmetric r x r matrix (cyclic Jacobi, single thread, in place).
__device__ double jacobi_max_eig(double* W, int r) {
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int a = 0; a < r; ++a) {
      diag += W[a * r + a] * W[a * r + a];
      for (int b = a + 1; b < r; ++b) off += W[a * r + b] * W[a * r + b];
    }
    if (off <= 1e-30 * diag || off == 0.0) break;
    for (int p = 0; p < r; ++p) {
      for (int q = p + 1; q < r; ++q) {
        const double apq = W[p * r + q];
        if (apq == 0.0) continue;
        const double theta = (W[q * r + q] - W[p * r + p]) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < r; ++k) {   // columns p, q
          const double wkp = W[k * r + p], wkq = W[k * r + q];
          W[k * r + p] = c * wkp - s * wkq;
          W[k * r + q] = s * wkp + c * wkq;
        }
        for (int k = 0; k < r; ++k) {   // rows p, q
          const double wpk = W[p * r + k], wqk = W[q * r + k];
          W[p * r + k] = c * wpk - s * wqk;
          W[q * r + k] = s * wpk + c * wqk;
        }
      }
    }
  }
  double lam = W[0];
  for (int a = 1; a < r; ++a) lam = fmax(lam, W[a * r + a]);
  return lam;
}

// In-place lower Cholesky factor of the SPD r x r matrix W (row-major LDS) by
// one wave, right-looking: column j is scaled by lane-parallel divisions and
// the trailing submatrix is updated by all lanes.  Writes 1/L_jj to rdiag.
// Returns false (wave-uniform) if a pivot is not positive.
__device__ bool wave_cholesky(double* W, double* rdiag, int r) {
  const int lane = threadIdx.x & 63;
  for (int j = 0; j < r; ++j) {
    const double piv = W[j * r + j];
    if (!(piv > 0.0)) return false;
    const double d = sqrt(piv);
    const double inv = 1.0 / d;
    if (lane == 0) {
      W[j * r + j] = d;
      rdiag[j] = inv;
    }
    if (lane > j && lane < r) W[lane * r + j] *= inv;
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    const int t = r - j - 1;                      // trailing size
    for (int e = lane; e < t * t; e += 64) {
      const int i = j + 1 + e / t, k = j + 1 + e % t;
      if (k <= i) W[i * r + k] -= W[i * r + j] * W[k * r + j];
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
  }
  return true;
}

// X (n x r, in place) <- X R^{-1} where X^T X = R^T R (R upper, positive diagonal).
// Returns false if the Gram matrix is not positive definite.
__device__ __forceinline__ bool block_cholqr_pass(float* X, int n, int r, double* sh, double* W, double* rdiag, int* okflag) {
  const int tid = threadIdx.x;
  block_gram(X, X, n, r, W, true);
  if (tid < 64) {
    const bool ok = wave_cholesky(W, rdiag, r);
    if (tid == 0) *okflag = ok ? 1 : 0;
  }
  __syncthreads();
  if (!*okflag) return false;
  // row x of X: solve x_new R = x, R[a][c] = L[c][a]
  for (int j = tid; j < n; j += kQRThreads) {
    double xn[kRMax];
#pragma unroll
    for (int c = 0; c < kRMax; ++c) {
      if (c < r) {
        double t = (double)X[(long long)j * r + c];
#pragma unroll
        for (int a = 0; a < kRMax; ++a)
          if (a < c) t -= xn[a] * W[c * r + a];
        xn[c] = t * rdiag[c];
      } else {
        xn[c] = 0.0;
      }
    }
#pragma unroll
    for (int c = 0; c < kRMax; ++c)
      if (c < r) X[(long long)j * r + c] = (float)xn[c];
  }
  __syncthreads();
  return true;
}

// The n x r block lives in LDS when it fits (a.lds != 0), else in a.Utmp.
struct QRShared {
  double sh[kQRThreads];
  double W[kRMax * kRMax], Lf[kRMax];
  double eta_s;
  int okflag;
};

__device__ __forceinline__ void qr_body(const QRArgs& a, unsigned char* dsm, QRShared& S) {
  double* sh = S.sh;
  double* W = S.W;
  double* Lf = S.Lf;
  double& eta_s = S.eta_s;
  int& okflag = S.okflag;
  const int tid = threadIdx.x;
  const int n = a.n, r = a.r, nr = n * r;
  if (a.mode == QR_POWER && a.ctl && a.ctl->conv) return;
  if (a.mode == QR_GD && a.gate_done && a.ctl && a.ctl->done) return;
  float* X = a.lds ? reinterpret_cast<float*>(dsm) : a.Utmp;

  if (a.mode != QR_ORTH) {
    if ((nr & 3) == 0) {   // float4 loads; the same per-element order as below
      const int nr4 = nr >> 2;
      for (int i4 = tid; i4 < nr4; i4 += kQRThreads) {
        float4 s = reinterpret_cast<const float4*>(a.gpart)[i4];
        for (int ks = 1; ks < a.KS; ++ks) {
          const float4 t = reinterpret_cast<const float4*>(a.gpart + (long long)ks * nr)[i4];
          s.x += t.x; s.y += t.y; s.z += t.z; s.w += t.w;
        }
        reinterpret_cast<float4*>(X)[i4] = s;
        if (a.grad_out) {
          a.grad_out[4 * i4] = s.x; a.grad_out[4 * i4 + 1] = s.y;
          a.grad_out[4 * i4 + 2] = s.z; a.grad_out[4 * i4 + 3] = s.w;
        }
      }
    } else {
      for (int idx = tid; idx < nr; idx += kQRThreads) {
        float s = a.gpart[idx];
        for (int ks = 1; ks < a.KS; ++ks) s += a.gpart[(long long)ks * nr + idx];
        X[idx] = s;
        if (a.grad_out) a.grad_out[idx] = s;
      }
    }
  } else if (a.lds) {
    for (int idx = tid; idx < nr; idx += kQRThreads) X[idx] = a.Utmp[idx];
  }
  __syncthreads();
  if (a.mode == QR_GD) {
    const bool have = a.ctl ? (a.ctl->eta_set != 0) : (*a.eta_io > 0.0);
    if (!have) {
      block_gram(X, X, n, r, W, true);
      if (tid == 0) {
        const double lam = jacobi_max_eig(W, r);
        const double eta = lam > 0.0 ? a.eta_c / sqrt(lam) : 0.0;
        eta_s = eta;
        if (a.ctl) {
          a.ctl->eta = eta;
          a.ctl->eta_set = 1;
        } else {
          *a.eta_io = eta;
        }
      }
    } else if (tid == 0) {
      eta_s = a.ctl ? a.ctl->eta : *a.eta_io;
    }
    __syncthreads();
    const double eta = eta_s;
    for (int idx = tid; idx < nr; idx += kQRThreads) X[idx] = (float)fma(-eta, (double)X[idx], (double)a.U[idx]);
    __syncthreads();
  }
  // CholeskyQR2.  A Gram that is not positive definite (a non-finite step, or a
  // rank-deficient block) raises error bit 1 and leaves U as it was; a GD step
  // still records the iteration below (its residual, the column flags, the count).
  bool ok = block_cholqr_pass(X, n, r, sh, W, Lf, &okflag);
  if (ok) ok = block_cholqr_pass(X, n, r, sh, W, Lf, &okflag);
  if (!ok) {
    if (tid == 0 && a.ctl) atomicOr(&a.ctl->err, 2);
    if (a.mode != QR_GD) return;
  }
  if (ok && a.mode == QR_POWER) {
    // subspace change ||U_new - U_old (U_old^T U_new)||_F, summed directly from the
    // residual entries (r - ||U_old^T U_new||_F^2 cancels below angles of ~3e-4 in FP32)
    block_gram(a.U, X, n, r, W, false);   // U_old^T U_new
    double acc = 0.0;
    for (int i = tid; i < n; i += kQRThreads) {   // one row per thread: U_old row in registers
      float u[kRMax];
#pragma unroll
      for (int e = 0; e < kRMax; ++e) u[e] = e < r ? a.U[(long long)i * r + e] : 0.f;
      for (int c = 0; c < r; ++c) {
        double d = (double)X[(long long)i * r + c];
#pragma unroll
        for (int e = 0; e < kRMax; ++e)
          if (e < r) d = fma(-(double)u[e], W[e * r + c], d);
        acc = fma(d, d, acc);
      }
    }
    acc = wave_sum_dpp(acc);
    if ((tid & 63) == 0) sh[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
      double f = 0.0;
      for (int w = 0; w < kQRThreads / 64; ++w) f += sh[w];
      const double sd = sqrt(f);
      const double prev = a.ctl->power_sd;   // 0 before the first step
      a.ctl->power_sd = sd;
      a.ctl->power_it += 1;
      // converged at power_tol, or once the change has stopped shrinking below 1e-3
      // (by less than 1 % in a step): the FP32 iterate's rounding floor.  A change
      // that still shrinks by a steady factor above 0.9 is a slow iteration (a
      // small gap sigma_{r+1} / sigma_r of L_0), not the floor, and goes on.
      if (sd <= a.power_tol || (sd <= 1e-3 && prev > 0.0 && sd >= 0.99 * prev)) a.ctl->conv = 1;
    }
  }
  for (int idx = tid; idx < nr; idx += kQRThreads) {
    if (a.mode == QR_GD && a.Uprev) a.Uprev[idx] = a.U[idx];
    if (ok) a.U[idx] = X[idx];
  }
  if (a.mode == QR_GD && a.ctl) {
    double s = 0.0;
    int fl = 0;
    for (int k = tid; k < a.q; k += kQRThreads) {
      s += a.colrr[k];
      fl |= a.colflags[k];
    }
    sh[tid] = s;
    __syncthreads();
    for (int st = kQRThreads / 2; st > 0; st >>= 1) {
      if (tid < st) sh[tid] += sh[tid + st];
      __syncthreads();
    }
    if (fl) atomicOr(&a.ctl->err, fl);
    if (tid == 0) {
      const double resid = a.ctl->ynorm2 > 0.0 ? sqrt(sh[0] / a.ctl->ynorm2) : sqrt(sh[0]);
      const int t = a.ctl->t;
      if (a.rlog && t < a.rlog_len) a.rlog[t] = resid;
      a.ctl->resid = resid;
      a.ctl->t = t + 1;
      // BF16X2 hi-only phase: switch to hi + lo when the residual stalls or the budget is spent
      if (a.ctl->phase == 0 && (t + 1 >= a.hi_max || (t > 0 && resid >= a.stall * a.ctl->prev_resid))) {
        a.ctl->phase = 1;
        a.ctl->refine_t = t + 1;
      }
      a.ctl->prev_resid = resid;
      if (a.gate_done && a.tol > 0.0 && resid <= a.tol) a.ctl->done = 1;
    }
  }
}

__global__ __launch_bounds__(kQRThreads) void k_qr(QRArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char dsm[];
  __shared__ QRShared S;
  qr_body(a, dsm, S);
}

// Several problems in one launch: block b updates the U of problem b.
__global__ __launch_bounds__(kQRThreads) void k_qr_grp(const QRArgs* tab) {
  extern __shared__ __attribute__((aligned(16))) unsigned char dsm[];
  __shared__ QRShared S;
  const QRArgs a = tab[blockIdx.x];
  qr_body(a, dsm, S);
}

// ||Y||_F^2 from the per-column values, fixed order.
__global__ __launch_bounds__(kQRThreads) void k_sum_ctl(const double* colrr, int q, Ctl* ctl) {
  __shared__ double sh[kQRThreads];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int k = tid; k < q; k += kQRThreads) s += colrr[k];
  sh[tid] = s;
  __syncthreads();
  for (int st = kQRThreads / 2; st > 0; st >>= 1) {
    if (tid < st) sh[tid] += sh[tid + st];
    __syncthreads();
  }
  if (tid == 0) ctl->ynorm2 = sh[0];
}

__global__ void k_set_phase(Ctl* ctl, int phase) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->phase = phase;
    ctl->refine_t = phase ? 0 : -1;
  }
}

__global__ void k_reset_ctl(Ctl* ctl, int full) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->eta = 0.0;
    ctl->eta_set = 0;
    ctl->t = 0;
    ctl->resid = 0.0;
    ctl->prev_resid = 0.0;
    ctl->done = 0;
    if (full) {
      ctl->power_sd = 0.0;
      ctl->ynorm2 = 0.0;
      ctl->conv = 0;
      ctl->power_it = 0;
      ctl->err = 0;
    }
  }
}

__global__ void k_fill_int(int* p, int v, long long count) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x) p[i] = v;
}

// U[j][c] = 1 if j % r == c else 0: an orthogonal start block with disjoint supports.
__global__ void k_fill_basis(float* U, int n, int r) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < (long long)n * r; i += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(i / r), c = (int)(i % r);
    U[i] = (j % r == c) ? 1.f : 0.f;
  }
}

__global__ void k_copy_f(float* dst, const float* src, long long count) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x) dst[i] = src[i];
}

__global__ void k_copy_i(int* dst, const int* src, long long count) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count; i += (long long)gridDim.x * blockDim.x) dst[i] = src[i];
}

// A support loaded into a solver (altgdmin_set_state) must hold rho distinct
// in-range indices in ascending order in every column; a column that does not
// gets the no-start support 0 .. rho - 1 with zero values and error bit 2.
// One 64-thread workgroup per column; vpe = floats per value (2 for complex).
__global__ void k_check_support(int* idx, float* val, int vpe, int q, int rho, int n, int* flags) {
  const int k = blockIdx.x, lane = threadIdx.x;
  if (k >= q) return;
  int* ik = idx + (long long)k * rho;
  float* vk = val + (long long)k * rho * vpe;
  int bad = 0;
  for (int t = lane; t < rho; t += 64) {
    const int j = ik[t];
    bad |= (j < 0 || j >= n || (t > 0 && j <= ik[t - 1])) ? 1 : 0;
  }
  if (__ballot(bad != 0) == 0ull) return;
  for (int t = lane; t < rho; t += 64) {
    ik[t] = t;
    for (int c = 0; c < vpe; ++c) vk[(long long)t * vpe + c] = 0.f;
  }
  if (lane == 0) flags[k] |= 4;
}

__global__ void k_put_words(long long* dst, StateWords w) {
  if (threadIdx.x < kStateWords && blockIdx.x == 0) dst[threadIdx.x] = w.v[threadIdx.x];
}

__global__ void k_sum_partials(const float* gpart, int KS, long long nr, float* out) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nr; i += (long long)gridDim.x * blockDim.x) {
    float s = gpart[i];
    for (int ks = 1; ks < KS; ++ks) s += gpart[(long long)ks * nr + i];
    out[i] = s;
  }
}

// ---------------------------------------------------------------- launchers

static inline int grid_for(long long count, int block) {
  long long g = (count + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  return (int)g;
}

hipError_t launch_grad(const float* H, const float* B, int n, int q, int r, int KS, float* gpart,
                       const int* skip, hipStream_t st) {
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  hipLaunchKernelGGL(k_grad, dim3((n + 63) / 64, KS), dim3(kGradWaves * 64), 0, st, H, B, n, q, r, KS, gpart, skip);
  return hipGetLastError();
}

hipError_t launch_ltu(const float* L0t, const float* U, int n, int q, int r, float* T, const int* skip,
                      hipStream_t st) {
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  hipLaunchKernelGGL(k_ltu, dim3((q + kWaves - 1) / kWaves), dim3(256), 0, st, L0t, U, n, q, r, T, skip);
  return hipGetLastError();
}

// Raise the dynamic LDS limit of the QR kernels to kQRLdsMax, once, before the
// first launch whose n x r block needs more than the default.  The block in LDS
// or in global memory goes through the same arithmetic in the same order.
static hipError_t qr_allow_lds(size_t bytes) {
  if (bytes <= kQRLdsDefault) return hipSuccess;
  static std::mutex mu;
  static bool done = false;
  std::lock_guard<std::mutex> lk(mu);
  if (done) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_qr), hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)kQRLdsMax);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_qr_grp), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)kQRLdsMax);
  done = e == hipSuccess;
  return e;
}

hipError_t launch_qr(const QRArgs& a_in, hipStream_t st) {
  QRArgs a = a_in;
  const size_t bytes = (size_t)a.n * a.r * sizeof(float);
  a.lds = bytes <= kQRLdsMax ? 1 : 0;
  if (a.lds) {
    const hipError_t e = qr_allow_lds(bytes);
    if (e != hipSuccess) return e;
  }
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  hipLaunchKernelGGL(k_qr, dim3(1), dim3(kQRThreads), a.lds ? bytes : 0, st, a);
  return hipGetLastError();
}

hipError_t launch_grad_grp(const GradArgs* tab, const int4* map, int blocks, hipStream_t st) {
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  hipLaunchKernelGGL(k_grad_grp, dim3(blocks), dim3(kGradWaves * 64), 0, st, tab, map);
  return hipGetLastError();
}

hipError_t launch_qr_grp(const QRArgs* tab, int count, size_t lds, hipStream_t st) {
  const hipError_t ea = qr_allow_lds(lds);
  if (ea != hipSuccess) return ea;
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  hipLaunchKernelGGL(k_qr_grp, dim3(count), dim3(kQRThreads), lds, st, tab);
  return hipGetLastError();
}

hipError_t launch_sum_ctl(const double* colrr, int q, Ctl* ctl, hipStream_t st) {
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  hipLaunchKernelGGL(k_sum_ctl, dim3(1), dim3(kQRThreads), 0, st, colrr, q, ctl);
  return hipGetLastError();
}

hipError_t launch_reset_ctl(Ctl* ctl, int full, hipStream_t st) {
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  hipLaunchKernelGGL(k_reset_ctl, dim3(1), dim3(64), 0, st, ctl, full);
  return hipGetLastError();
}

hipError_t launch_set_phase(Ctl* ctl, int phase, hipStream_t st) {
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  hipLaunchKernelGGL(k_set_phase, dim3(1), dim3(64), 0, st, ctl, phase);
  return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int v, long long count, hipStream_t st) {
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  hipLaunchKernelGGL(k_fill_int, dim3(grid_for(count, 256)), dim3(256), 0, st, p, v, count);
  return hipGetLastError();
}

hipError_t launch_fill_basis(float* U, int n, int r, hipStream_t st) {
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  hipLaunchKernelGGL(k_fill_basis, dim3(grid_for((long long)n * r, 256)), dim3(256), 0, st, U, n, r);
  return hipGetLastError();
}

hipError_t launch_copy_f(float* dst, const float* src, long long count, hipStream_t st) {
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  hipLaunchKernelGGL(k_copy_f, dim3(grid_for(count, 256)), dim3(256), 0, st, dst, src, count);
  return hipGetLastError();
}

hipError_t launch_sum_partials(const float* gpart, int KS, long long nr, float* out, hipStream_t st) {
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  hipLaunchKernelGGL(k_sum_partials, dim3(grid_for(nr, 256)), dim3(256), 0, st, gpart, KS, nr, out);
  return hipGetLastError();
}

hipError_t launch_check_support(int* idx, float* val, int vpe, int q, int rho, int n, int* flags, hipStream_t st) {
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  if (q < 1 || rho < 1) return hipSuccess;
  hipLaunchKernelGGL(k_check_support, dim3(q), dim3(64), 0, st, idx, val, vpe, q, rho, n, flags);
  return hipGetLastError();
}

hipError_t launch_put_words(long long* dst, const StateWords& w, hipStream_t st) {
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  hipLaunchKernelGGL(k_put_words, dim3(1), dim3(64), 0, st, dst, w);
  return hipGetLastError();
}

hipError_t launch_copy_i(int* dst, const int* src, long long count, hipStream_t st) {
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  hipLaunchKernelGGL(k_copy_i, dim3(grid_for(count, 256)), dim3(256), 0, st, dst, src, count);
  return hipGetLastError();
}

}  // namespace altg
