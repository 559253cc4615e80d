// Partial Fourier form of the measurement operators (gfx950).
//
// A_k keeps the rows mask_k of the unitary 2D DFT of 96 x 96 complex frames
// (x_k flattened row-major; frequency index u = u1 * 96 + u2), so
// A_k x = (F x)[mask_k] and A_k^H v = F^H (v scattered to mask_k).  All data are
// complex64 (float2 = re, im); every transpose of the real path is a conjugate
// transpose and HardThreshold ranks by modulus.  Per GDmin iteration of Alg. 1:
//
//   k_fu   : F U (the DFT of each column of U): a row pass and a column pass,
//            one 96-point line per 32 lanes;
//   k_fcol : per column k (one 1024-thread workgroup): P_k = (F U)[mask_k],
//            G_k = P_k^H P_k and its inverse in FP64, the projected IHT of
//            Alg. 2 (tau iterations, three 2D FFTs each), b_k by least squares
//            (eq. (bk_LS)), r_k and h_k = A_k^H r_k;
//   k_fgrad_gd: grad_U f = sum_k h_k b_k^H (four column splits in a fixed order)
//            and per-block partial Grams;
//   k_fqr_a .. k_fqr_d: eta at t = 1, U - eta grad, CholeskyQR2 with a real
//            positive diagonal over many workgroups, the residual.
// The initialisation uses k_fcol with M = A_k (IHT from 0, then the columns of
// L_0 = [A_k^H (y_k - A_k s_k)]), k_fqr for the orthonormal start block, and the
// subspace iteration k_fltu / k_fgrad_gd / k_fqr_a .. k_fqr_f.
//
// 2D FFT.  A frame lives in LDS as 96 rows of 97 complex values (one pad column
// keeps the column pass free of bank conflicts).  Each 96-point transform is
// done by a group of 32 lanes: lane l holds elements l, l + 32, l + 64; a
// radix-3 butterfly with twiddles W96^(l k2) is followed by a 32-point radix-2
// decimation-in-frequency transform across the lanes (ds_swizzle exchanges), so
// lane l ends with outputs 3 bitrev5(l) + k2.  Rows first, then columns; the
// unitary scale 1/96 is applied in the column pass.
//
// Other frame sizes (n1 x n2 with n = n1 n2 <= 4096 and lines of at most 1024
// points; e.g. the 20 x 20 frames or the 1 x 400 rows of a 1D DFT) take the
// generic instantiation (GEN) of the column kernel: frames are stored unpadded
// and each 2D DFT is a row pass and a column pass of direct line DFTs, every
// output a sum over its line in index order with twiddles W_N^((u j) mod N) from
// a table in LDS (n1 + n2 entries); up to four outputs per thread are held in
// registers across a barrier, so the passes run in place.  k_fu_gen is the same
// transform of the columns of U.
#include "common.h"
#include "launch.h"

namespace altg {

namespace {

__device__ __forceinline__ float2 c_add(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 c_sub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 c_mul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 c_scale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// |v|^2 as the ranking key: two products and one sum, each rounded to FP32.
__device__ __forceinline__ float c_abs2_key(float2 v) {
#pragma clang fp contract(off)
  const float a = v.x * v.x;
  const float b = v.y * v.y;
  return a + b;
}

__device__ __forceinline__ int fpos(int j) { return j + j / kFN; }   // element j -> padded grid slot

template <int H>
__device__ __forceinline__ float2 swz_xor(float2 v) {
  // ds_swizzle bit mode inside groups of 32 lanes: partner = lane ^ H
  constexpr int pat = (H << 10) | 0x1f;
  return make_float2(__int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v.x), pat)),
                     __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v.y), pat)));
}

template <bool INV>
__device__ __forceinline__ float2 twid(const float2* tw, int e) {   // W96^e (conjugated for the inverse)
  const float2 w = tw[e];
  return INV ? make_float2(w.x, -w.y) : w;
}

template <bool INV, int H>
__device__ __forceinline__ void dif_stage(float2 (&v)[3], int l, const float2* tw) {
  const bool up = (l & H) != 0;
  const float2 w = twid<INV>(tw, 3 * ((l & (H - 1)) * (16 / H)));   // W32^((l mod H) 16 / H)
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float2 t = swz_xor<H>(v[a]);
    v[a] = up ? c_mul(c_sub(t, v[a]), w) : c_add(v[a], t);
  }
}

// 96-point DFT by the 32 lanes of a group: in v[a] = x[l + 32 a], out v[a] = X[3 bitrev5(l) + a].
template <bool INV>
__device__ __forceinline__ void fft96(float2 (&v)[3], int l, const float2* tw) {
  const float2 w1 = twid<INV>(tw, 32), w2 = twid<INV>(tw, 64);   // W3, W3^2
  const float2 x0 = v[0], x1 = v[1], x2 = v[2];
  v[0] = c_add(c_add(x0, x1), x2);
  v[1] = c_mul(c_add(c_add(x0, c_mul(x1, w1)), c_mul(x2, w2)), twid<INV>(tw, l));
  v[2] = c_mul(c_add(c_add(x0, c_mul(x1, w2)), c_mul(x2, w1)), twid<INV>(tw, 2 * l));
  dif_stage<INV, 16>(v, l, tw);
  dif_stage<INV, 8>(v, l, tw);
  dif_stage<INV, 4>(v, l, tw);
  dif_stage<INV, 2>(v, l, tw);
  dif_stage<INV, 1>(v, l, tw);
}

// Unitary 2D DFT (INV: its inverse) of the frame in `grid`, in place.  All 1024
// threads call it; it ends with a barrier.
template <bool INV>
__device__ __attribute__((noinline)) void fft2_grid(float2* grid, const float2* tw) {
  const int g = threadIdx.x >> 5, l = threadIdx.x & 31;
  const int k1 = (int)(__builtin_bitreverse32((unsigned)l) >> 27);
  for (int rr = 0; rr < 3; ++rr) {
    float2* row = grid + (g + 32 * rr) * kFP;
    float2 v[3] = {row[l], row[l + 32], row[l + 64]};
    fft96<INV>(v, l, tw);
    row[3 * k1] = v[0];
    row[3 * k1 + 1] = v[1];
    row[3 * k1 + 2] = v[2];
  }
  __syncthreads();
  const float s = 1.0f / kFN;
  for (int cc = 0; cc < 3; ++cc) {
    float2* col = grid + g + 32 * cc;
    float2 v[3] = {col[l * kFP], col[(l + 32) * kFP], col[(l + 64) * kFP]};
    fft96<INV>(v, l, tw);
    col[(3 * k1) * kFP] = c_scale(v[0], s);
    col[(3 * k1 + 1) * kFP] = c_scale(v[1], s);
    col[(3 * k1 + 2) * kFP] = c_scale(v[2], s);
  }
  __syncthreads();
}

__device__ __forceinline__ void zero_grid(float2* grid, int count = kFGrid) {
  for (int t = threadIdx.x; t < count; t += kFThreads) grid[t] = make_float2(0.f, 0.f);
}

// Unitary 2D DFT (INV: inverse) of an unpadded n1 x n2 frame in `grid`, in place,
// by direct line sums: first X[j1][u2] = sum_j2 x[j1][j2] W_n2^(u2 j2), then
// X[u1][u2] = scale sum_j1 X[j1][u2] W_n1^(u1 j1), each sum in index order.  tw
// holds W_n1^t (t < n1) then W_n2^t (t < n2).  All threads of the workgroup call
// it (blockDim.x = kFThreads, n1 n2 <= kFGenPer kFThreads); it ends with a barrier.
template <bool INV>
__device__ __attribute__((noinline)) void dft2_gen(float2* grid, const float2* tw, int n1, int n2, float scale) {
  const int n = n1 * n2;
  const float2* tw1 = tw;
  const float2* tw2 = tw + n1;
  float2 acc[kFGenPer];
#pragma unroll
  for (int e = 0; e < kFGenPer; ++e) {
    const int t = threadIdx.x + e * kFThreads;
    float2 sum = make_float2(0.f, 0.f);
    if (t < n) {
      const int j1 = t / n2, u2 = t - j1 * n2;
      const float2* row = grid + j1 * n2;
      int w = 0;   // (u2 j2) mod n2
      for (int j2 = 0; j2 < n2; ++j2) {
        const float2 x = row[j2], tt = twid<INV>(tw2, w);
        sum.x = fmaf(x.x, tt.x, fmaf(-x.y, tt.y, sum.x));
        sum.y = fmaf(x.x, tt.y, fmaf(x.y, tt.x, sum.y));
        w += u2;
        if (w >= n2) w -= n2;
      }
    }
    acc[e] = sum;
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < kFGenPer; ++e) {
    const int t = threadIdx.x + e * kFThreads;
    if (t < n) grid[t] = acc[e];
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < kFGenPer; ++e) {
    const int t = threadIdx.x + e * kFThreads;
    float2 sum = make_float2(0.f, 0.f);
    if (t < n) {
      const int u1 = t / n2, u2 = t - u1 * n2;
      int w = 0;   // (u1 j1) mod n1
      for (int j1 = 0; j1 < n1; ++j1) {
        const float2 x = grid[j1 * n2 + u2], tt = twid<INV>(tw1, w);
        sum.x = fmaf(x.x, tt.x, fmaf(-x.y, tt.y, sum.x));
        sum.y = fmaf(x.x, tt.y, fmaf(x.y, tt.x, sum.y));
        w += u1;
        if (w >= n1) w -= n1;
      }
    }
    acc[e] = c_scale(sum, scale);
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < kFGenPer; ++e) {
    const int t = threadIdx.x + e * kFThreads;
    if (t < n) grid[t] = acc[e];
  }
  __syncthreads();
}

// Sum over the workgroup of NV doubles per thread, in a fixed order (DPP inside
// each wave, then the 16 wave totals in wave order).  out[0..NV) in LDS; ends
// with a barrier.  red holds kFWaves * NV doubles.
template <int NV>
__device__ void fblock_sum(double (&v)[NV], double* red, double* out) {
  const int lane = threadIdx.x & 63, wave = wave_id();
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum_dpp(v[i]);
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) red[wave * NV + i] = v[i];
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
    for (int w = 0; w < kFWaves; ++w) s += red[w * NV + threadIdx.x];
    out[threadIdx.x] = s;
  }
  __syncthreads();
}

// Whether HardThreshold keeps the support marked in the bitmap `mark`: it does
// when every key on it is larger than every key off it (with a tie or a NaN key
// the full select decides).  slot holds 3 kFWaves words of LDS; a barrier on
// entry to the reduction and on exit.
template <class Val>
__device__ bool fsupport_kept(Val val, int n, const unsigned* mark, unsigned* slot) {
  const int lane = threadIdx.x & 63, wave = wave_id();
  unsigned kmin = 0xffffffffu, kmax = 0u;
  bool bad = false;
  for (int j = threadIdx.x; j < n; j += kFThreads) {
    const unsigned key = __float_as_uint(c_abs2_key(val(j)));
    bad |= key > 0x7f800000u;
    if ((mark[j >> 5] >> (j & 31)) & 1u)
      kmin = min(kmin, key);
    else
      kmax = max(kmax, key);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    kmin = min(kmin, __shfl_xor(kmin, o));
    kmax = max(kmax, __shfl_xor(kmax, o));
  }
  const bool wbad = __ballot(bad) != 0ull;
  if (lane == 0) {
    slot[3 * wave] = kmin;
    slot[3 * wave + 1] = kmax;
    slot[3 * wave + 2] = wbad ? 1u : 0u;
  }
  __syncthreads();
  unsigned mn = 0xffffffffu, mx = 0u, b = 0u;
#pragma unroll
  for (int w = 0; w < kFWaves; ++w) {
    mn = min(mn, slot[3 * w]);
    mx = max(mx, slot[3 * w + 1]);
    b |= slot[3 * w + 2];
  }
  __syncthreads();
  return b == 0u && mn > mx;
}

// Whether any thread of the workgroup has f != 0 (every thread calls it; a
// barrier on entry and on exit).  slot holds kFWaves ints of LDS.
__device__ bool fblock_any(int f, int* slot) {
  const int lane = threadIdx.x & 63, wave = wave_id();
  const bool any = __ballot(f != 0) != 0ull;
  if (lane == 0) slot[wave] = any ? 1 : 0;
  __syncthreads();
  int r = 0;
#pragma unroll
  for (int w = 0; w < kFWaves; ++w) r |= slot[w];
  __syncthreads();
  return r != 0;
}

// Exclusive prefix sum of one int per thread over the workgroup in thread order;
// *total gets the sum.  tmp holds kFWaves + 1 ints.
__device__ int fblock_exscan(int v, int* tmp, int* total) {
  const int lane = threadIdx.x & 63, wave = wave_id();
  int incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  if (lane == 63) tmp[wave] = incl;
  __syncthreads();
  int base = 0, all = 0;
  for (int w = 0; w < kFWaves; ++w) {
    const int t = tmp[w];
    base += w < wave ? t : 0;
    all += t;
  }
  *total = all;
  __syncthreads();
  return base + incl - v;
}

// HardThreshold support of n complex values: the rho largest keys |v|^2 (FP32,
// as c_abs2_key), lower index first on ties, written ascending to idx[0..rho).
// Thread t owns the contiguous elements [t c, t c + c), c = ceil(n / 1024).
// Byte-wise radix selection with a 256-bin LDS histogram.  Returns the number of
// NaN keys seen.  hist holds 256 + 8 ints, tmp kFWaves + 1 ints.
template <class Val>
__device__ int fselect(Val val, int n, int rho, int* idx, int* hist, int* tmp) {
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
  const int per = (n + kFThreads - 1) / kFThreads;
  const int j0 = tid * per;
  const int j1 = min(n, j0 + per);
  int* ctl = hist + 256;
  unsigned prefix = 0u, pmask = 0u;
  int remaining = rho;
  int nanc = 0;
  for (int d = 3; d >= 0; --d) {
    const int shift = 8 * d;
    for (int b = tid; b < 256; b += kFThreads) hist[b] = 0;
    if (d == 3 && tid == 0) ctl[2] = 0;
    __syncthreads();
    for (int j = j0; j < j1; ++j) {
      const unsigned key = __float_as_uint(c_abs2_key(val(j)));
      if (d == 3) nanc += key > 0x7f800000u ? 1 : 0;
      if ((key & pmask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1);
    }
    if (d == 3 && nanc) atomicAdd(&ctl[2], nanc);
    __syncthreads();
    if (wave == 0) {
      const int h0 = hist[4 * lane], h1 = hist[4 * lane + 1], h2 = hist[4 * lane + 2], h3 = hist[4 * lane + 3];
      const int lsum = h0 + h1 + h2 + h3;
      int incl = lsum;   // inclusive suffix sum over lanes >= lane
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_down(incl, o);
        if (lane + o < 64) incl += t;
      }
      int acc = incl - lsum;
      const int hb[4] = {h3, h2, h1, h0};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (acc < remaining && remaining <= acc + hb[q]) {
          ctl[0] = 4 * lane + 3 - q;
          ctl[1] = remaining - acc;
        }
        acc += hb[q];
      }
    }
    __syncthreads();
    remaining = ctl[1];
    prefix |= (unsigned)ctl[0] << shift;
    pmask |= 255u << shift;
    __syncthreads();
  }
  const unsigned T = prefix;
  int ngt = 0, neq = 0;
  for (int j = j0; j < j1; ++j) {
    const unsigned key = __float_as_uint(c_abs2_key(val(j)));
    ngt += key > T ? 1 : 0;
    neq += key == T ? 1 : 0;
  }
  int tot;
  const int eq_base = fblock_exscan(neq, tmp, &tot);
  const int take_eq = max(0, min(neq, remaining - eq_base));
  const int nsel = ngt + take_eq;
  const int pos0 = fblock_exscan(nsel, tmp, &tot);
  int pos = pos0, eqs = 0;
  for (int j = j0; j < j1; ++j) {
    const unsigned key = __float_as_uint(c_abs2_key(val(j)));
    bool sel = key > T;
    if (key == T) {
      sel = eqs < take_eq;
      ++eqs;
    }
    if (sel && pos < rho) idx[pos++] = j;
  }
  const int nan_total = ctl[2];
  __syncthreads();
  return nan_total;
}

// G^{-1} of a Hermitian positive definite r x r matrix (complex FP64, row-major
// double2 = re, im), by the workgroup: Cholesky G = L L^H (real positive
// diagonal) column by column, thread j + 1 + t computing L[j + 1 + t][j]; then
// thread c solves L y = e_c and L^H x = y for column c.  Returns false (identity
// in Ginv) if a pivot is not positive.
__device__ bool fblock_chol_inverse(const double2* G, double2* L, double2* Ginv, double2* Y, int r) {
  const int tid = threadIdx.x;
  for (int j = 0; j < r; ++j) {
    double s = G[j * r + j].x;
    for (int p = 0; p < j; ++p) s -= L[j * r + p].x * L[j * r + p].x + L[j * r + p].y * L[j * r + p].y;
    if (!(s > 0.0)) {
      for (int i = tid; i < r * r; i += kFThreads) Ginv[i] = make_double2((i % (r + 1) == 0) ? 1.0 : 0.0, 0.0);
      __syncthreads();
      return false;
    }
    const double d = sqrt(s);
    const int i = j + 1 + tid;
    if (i < r) {
      double tr = G[i * r + j].x, ti = G[i * r + j].y;
      for (int p = 0; p < j; ++p) {   // t -= L[i][p] conj(L[j][p])
        const double2 a = L[i * r + p], b = L[j * r + p];
        tr -= a.x * b.x + a.y * b.y;
        ti -= a.y * b.x - a.x * b.y;
      }
      L[i * r + j] = make_double2(tr / d, ti / d);
    }
    if (tid == 0) L[j * r + j] = make_double2(d, 0.0);
    if (tid < j) L[tid * r + j] = make_double2(0.0, 0.0);
    __syncthreads();
  }
  if (tid < r) {
    const int c = tid;
    for (int i = c; i < r; ++i) {
      double tr = (i == c) ? 1.0 : 0.0, ti = 0.0;
      for (int p = c; p < i; ++p) {   // t -= L[i][p] y[p]
        const double2 a = L[i * r + p], y = Y[p * r + c];
        tr -= a.x * y.x - a.y * y.y;
        ti -= a.x * y.y + a.y * y.x;
      }
      const double dd = L[i * r + i].x;
      Y[i * r + c] = make_double2(tr / dd, ti / dd);
    }
    for (int i = r - 1; i >= 0; --i) {
      double tr = i >= c ? Y[i * r + c].x : 0.0, ti = i >= c ? Y[i * r + c].y : 0.0;
      for (int p = i + 1; p < r; ++p) {   // t -= conj(L[p][i]) x[p]
        const double2 a = L[p * r + i], x = Ginv[p * r + c];
        tr -= a.x * x.x + a.y * x.y;
        ti -= a.x * x.y - a.y * x.x;
      }
      const double dd = L[i * r + i].x;
      Ginv[i * r + c] = make_double2(tr / dd, ti / dd);
    }
  }
  __syncthreads();
  return true;
}

}  // namespace

// ---------------------------------------------------------------- k_fcol

// LDS layout of the column kernel (bytes)
struct FColLayout {
  size_t gridA, gridB, tw, red, gi, dsum, gx, sidx, sval, gT, hist, tmp, total;
  // grid: complex elements of each of the two frame grids; ntw: twiddles
  __host__ __device__ FColLayout(int rho, int r, int grid = kFGrid, int ntw = kFN) {
    size_t o = 0;
    gridA = o; o = align16(o + 8 * (size_t)grid);
    gridB = o; o = align16(o + 8 * (size_t)grid);
    tw = o;    o = align16(o + 8 * (size_t)ntw);
    red = o;   o = align16(o + 8 * (size_t)kFWaves * (2 * kFRMax + 2));
    gi = o;    o = align16(o + 16 * (size_t)r * r);
    dsum = o;  o = align16(o + 8 * (size_t)(2 * kFRMax + 2));
    gx = o;    o = align16(o + 16 * (size_t)kFRMax);
    sidx = o;  o = align16(o + 4 * (size_t)rho);
    sval = o;  o = align16(o + 8 * (size_t)rho);
    gT = o;    o = align16(o + 8 * (size_t)rho);
    hist = o;  o = align16(o + 4 * (size_t)(256 + 8));
    tmp = o;   o = align16(o + 4 * (size_t)(kFWaves + 1));
    total = o;
  }
};

// Grid elements of a generic frame: the frame (n), or the rows of P_k staged for
// the Gram (m rows of kFRMax + 1 complex values over both grids), whichever is more.
__host__ __device__ inline int fgen_grid(int n, int m) {
  int need = (m * (kFRMax + 1) + 1) / 2;
  // grid B also holds the Cholesky work arrays: 2 kFRMax^2 double2 = 4 kFRMax^2 complex slots
  if (need < 4 * kFRMax * kFRMax) need = 4 * kFRMax * kFRMax;
  return ((n > need ? n : need) + 3) / 4 * 4;
}

size_t fcol_lds_bytes(int rho, int r, int n, int m, int n1, int n2) {
  if (n1 == kFN && n2 == kFN) return FColLayout(rho, r).total;
  return FColLayout(rho, r, fgen_grid(n, m), n1 + n2).total;
}

template <int R, bool GEN>
__global__ __launch_bounds__(kFThreads) void k_fcol(FColArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int tid = threadIdx.x, k = blockIdx.x;
  const int n = a.n, m = a.m, r = a.r, rho = a.rho;
  const bool gd = a.mode == FCOL_GD;
  const int gsize = GEN ? n : kFGrid;              // grid slots a transform touches
  const int ntw = GEN ? a.n1 + a.n2 : kFN;
  const FColLayout lay = GEN ? FColLayout(rho, r, fgen_grid(n, m), ntw) : FColLayout(rho, r);
  const float gscale = GEN ? (float)(1.0 / sqrt((double)n)) : 0.f;
  // element j -> grid slot (the 96 x 96 grid has a pad column)
  auto pos = [&](int j) { return GEN ? j : fpos(j); };
  auto dft2 = [&](float2* g, const float2* t, bool inv) {
    if constexpr (GEN) {
      if (inv) dft2_gen<true>(g, t, a.n1, a.n2, gscale);
      else dft2_gen<false>(g, t, a.n1, a.n2, gscale);
    } else {
      if (inv) fft2_grid<true>(g, t);
      else fft2_grid<false>(g, t);
    }
  };
  float2* gA = reinterpret_cast<float2*>(smem + lay.gridA);
  float2* gB = reinterpret_cast<float2*>(smem + lay.gridB);
  float2* tw = reinterpret_cast<float2*>(smem + lay.tw);
  double* red = reinterpret_cast<double*>(smem + lay.red);
  double2* Gi = reinterpret_cast<double2*>(smem + lay.gi);
  double* dsum = reinterpret_cast<double*>(smem + lay.dsum);
  double2* gx = reinterpret_cast<double2*>(smem + lay.gx);
  int* sidx = reinterpret_cast<int*>(smem + lay.sidx);
  float2* sval = reinterpret_cast<float2*>(smem + lay.sval);
  float2* gT = reinterpret_cast<float2*>(smem + lay.gT);
  int* hist = reinterpret_cast<int*>(smem + lay.hist);
  int* tmp = reinterpret_cast<int*>(smem + lay.tmp);

  for (int t = tid; t < ntw; t += kFThreads) tw[t] = a.tw[t];
  // the measurement rows i = tid, tid + 1024 of this thread, in registers
  int mi[2];
  bool ok[2];
  float2 yv[2];
  int flags = 0;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int i = tid + kFThreads * e;
    const int raw = i < m ? a.mask[(long long)k * m + i] : 0;
    const bool inr = raw >= 0 && raw < n;
    if (i < m && !inr) flags |= 4;   // a frequency index out of range: the row is left out
    ok[e] = i < m && inr;
    mi[e] = ok[e] ? raw : 0;
    yv[e] = ok[e] ? a.Y[(long long)k * a.ldy + i] : make_float2(0.f, 0.f);
  }
  // rows i of P_k = rows mask_k[i] of F U, read once into registers (the GD
  // steps use them about a dozen times; each re-read from L2 was a round trip
  // on the critical path).  At R = 6, 8 this costs a few spilled registers.
  float2 Pc[2][R];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const float2* src = a.FU + (long long)mi[e] * r;
#pragma unroll
    for (int c = 0; c < R; ++c) Pc[e][c] = (gd && ok[e] && c < r) ? src[c] : make_float2(0.f, 0.f);
  }
  auto Prow = [&](int e, float2 (&p)[R]) {
#pragma unroll
    for (int c = 0; c < R; ++c) p[c] = Pc[e][c];
  };
  int nz = 0;
  for (int e = tid; e < rho; e += kFThreads) {
    int j = e;   // s = 0 on the support 0 .. rho - 1 when there is no start (kept if tau = 0)
    float2 v = make_float2(0.f, 0.f);
    if (gd) {
      j = a.Sidx[(long long)k * rho + e];
      v = a.Sval[(long long)k * rho + e];
      if (j < 0 || j >= n) {   // invalid state: flag it and keep every access in bounds
        flags |= 4;
        j = 0;
        v = make_float2(0.f, 0.f);
      }
    }
    sidx[e] = j;
    sval[e] = v;
    nz |= v.x != 0.f || v.y != 0.f;
  }
  // a start whose values are all zero (an initialisation with tau0 = 0) is s = 0
  // with no support yet: T then comes from HardThreshold(g), as for no start
  const bool start = fblock_any(nz, tmp);

  // G_k = P_k^H P_k (FP64) and its inverse.  The rows of P_k are staged in the
  // two grids (free at this point); wave w sums the entries w, w + 16, ... of
  // the upper triangle with its lanes over the rows (fixed DPP order).
  if (gd) {
    constexpr int PS = R + 1;   // LDS row stride of P_k (complex values)
    float2* Pl = gA;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int i = tid + kFThreads * e;
      if (i < m) {
        float2 p[R];
        Prow(e, p);
#pragma unroll
        for (int c = 0; c < R; ++c) Pl[i * PS + c] = p[c];
      }
    }
    __syncthreads();
    double2* Gl = reinterpret_cast<double2*>(red);   // r x r
    {
      const int lane = tid & 63, wave = wave_id();
      const int E = r * (r + 1) / 2;
      for (int e = wave; e < E; e += kFWaves) {
        int ra = 0, base = 0;
        while (e >= base + (r - ra)) {
          base += r - ra;
          ++ra;
        }
        const int rb = ra + (e - base);
        double sr = 0.0, si = 0.0;
        for (int i = lane; i < m; i += 64) {   // conj(P[i][ra]) P[i][rb]
          const float2 pa = Pl[i * PS + ra], pb = Pl[i * PS + rb];
          sr = fma((double)pa.x, (double)pb.x, fma((double)pa.y, (double)pb.y, sr));
          si = fma((double)pa.x, (double)pb.y, fma(-(double)pa.y, (double)pb.x, si));
        }
        sr = wave_sum_dpp(sr);
        si = wave_sum_dpp(si);
        if (lane == 0) {
          Gl[ra * r + rb] = make_double2(sr, si);
          Gl[rb * r + ra] = make_double2(sr, -si);
        }
      }
    }
    __syncthreads();
    double2* Ll = reinterpret_cast<double2*>(gB);   // the staged rows are no longer needed
    double2* Yl = Ll + kFRMax * kFRMax;
    if (!fblock_chol_inverse(Gl, Ll, Gi, Yl, r)) flags |= 2;
  }

  // gx = G_k^{-1} x for the complex x in dsum[0 .. 2r), entry ra by thread ra
  // (one 36-term FP64 chain per workgroup rather than per thread); one barrier.
  auto ginv_apply = [&]() {
    if (tid < r) {
      double dr = 0.0, di = 0.0;
      for (int cb = 0; cb < r; ++cb) {
        const double2 g = Gi[tid * r + cb];
        const double xr = dsum[2 * cb], xi = dsum[2 * cb + 1];
        dr += g.x * xr - g.y * xi;
        di += g.x * xi + g.y * xr;
      }
      gx[tid] = make_double2(dr, di);
    }
    __syncthreads();
  };

  // v <- v - P_k G_k^{-1} P_k^H v for the two rows of this thread
  auto project = [&](float2 (&v)[2]) {
    double c[2 * R];
#pragma unroll
    for (int cc = 0; cc < 2 * R; ++cc) c[cc] = 0.0;
#pragma unroll
    for (int e = 0; e < 2; ++e) {   // conj(P[i][cc]) v[i]
      float2 p[R];
      Prow(e, p);
#pragma unroll
      for (int cc = 0; cc < R; ++cc) {
        c[2 * cc] += (double)p[cc].x * v[e].x + (double)p[cc].y * v[e].y;
        c[2 * cc + 1] += (double)p[cc].x * v[e].y - (double)p[cc].y * v[e].x;
      }
    }
    fblock_sum<2 * R>(c, red, dsum);
    ginv_apply();
    float2 d[R];
#pragma unroll
    for (int ra = 0; ra < R; ++ra) d[ra] = ra < r ? make_float2((float)gx[ra].x, (float)gx[ra].y) : make_float2(0.f, 0.f);
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      float2 p[R];
      Prow(e, p);
      float2 s = v[e];
#pragma unroll
      for (int ra = 0; ra < R; ++ra) s = c_sub(s, c_mul(p[ra], d[ra]));
      v[e] = ok[e] ? s : make_float2(0.f, 0.f);
    }
  };

  auto sum_sq = [&](float2 (&v)[2]) -> double {
    double s[1] = {0.0};
#pragma unroll
    for (int e = 0; e < 2; ++e) s[0] += (double)v[e].x * v[e].x + (double)v[e].y * v[e].y;
    fblock_sum<1>(s, red, dsum);
    return dsum[0];
  };

  // A_k s (the sparse s in sidx/sval) into grid B, gathered at this thread's rows
  auto apply_sparse = [&](const int* id, const float2* vl, int cnt, float2 (&out)[2]) {
    zero_grid(gB, gsize);
    __syncthreads();
    for (int e = tid; e < cnt; e += kFThreads) gB[pos(id[e])] = vl[e];
    __syncthreads();
    dft2(gB, tw, false);
#pragma unroll
    for (int e = 0; e < 2; ++e) out[e] = ok[e] ? gB[pos(mi[e])] : make_float2(0.f, 0.f);
    __syncthreads();
  };
  // A_k^H v into grid A
  auto apply_adj = [&](float2 (&v)[2]) {
    zero_grid(gA, gsize);
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 2; ++e)
      if (ok[e]) gA[pos(mi[e])] = v[e];
    __syncthreads();
    dft2(gA, tw, true);
  };

  // A_k s at this thread's rows.  When a HardThreshold step keeps the support
  // T, the new s is s - mu g_T, so A_k s moves by -mu A_k g_T = -mu w, which is
  // already at hand: the next transform of s is skipped (equal up to rounding
  // order).  mark is a bitmap of T over n, kept in grid B between transforms.
  float2 as[2] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
  bool have = start, known = !start;   // without a start s = 0, so A_k s = 0
  unsigned* mark = reinterpret_cast<unsigned*>(gB);
  const int words = (n + 31) >> 5;
  const int tau = rho > 0 ? a.tau : 0;
  for (int it = 0; it < tau; ++it) {
    // u = M s - z: A s - y (projected in the GD iterations)
    float2 u[2];
    if (!known) apply_sparse(sidx, sval, rho, as);
#pragma unroll
    for (int e = 0; e < 2; ++e) u[e] = ok[e] ? c_sub(as[e], yv[e]) : make_float2(0.f, 0.f);
    if (gd) project(u);
    // g = M^H u = A^H u (u lies in the range of the projector)
    apply_adj(u);
    // T: the current support, or that of HardThreshold(g) when s = 0
    if (!have) {
      flags |= fselect([&](int j) { return gA[pos(j)]; }, n, rho, sidx, hist, tmp) ? 1 : 0;
      for (int e = tid; e < rho; e += kFThreads) sval[e] = make_float2(0.f, 0.f);
      __syncthreads();
    }
    double gg_part = 0.0;
    for (int e = tid; e < rho; e += kFThreads) {
      const float2 g = gA[pos(sidx[e])];
      gT[e] = g;
      gg_part += (double)g.x * g.x + (double)g.y * g.y;
    }
    // w = M g_T: only ||w||^2 is needed.  With the projector, ||Pi w||^2 =
    // ||w||^2 - Re(c^H G^{-1} c) with c = P_k^H w, one reduction together with
    // ||g_T||^2.
    float2 w[2];
    apply_sparse(sidx, gT, rho, w);
    double gg, ww;
    {
      double v[2 * R + 2];
#pragma unroll
      for (int cc = 0; cc < 2 * R + 2; ++cc) v[cc] = 0.0;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        v[2 * R] += (double)w[e].x * w[e].x + (double)w[e].y * w[e].y;
        if (gd) {
          float2 p[R];
          Prow(e, p);
#pragma unroll
          for (int cc = 0; cc < R; ++cc) {
            v[2 * cc] += (double)p[cc].x * w[e].x + (double)p[cc].y * w[e].y;
            v[2 * cc + 1] += (double)p[cc].x * w[e].y - (double)p[cc].y * w[e].x;
          }
        }
      }
      v[2 * R + 1] = gg_part;
      fblock_sum<2 * R + 2>(v, red, dsum);
      gg = dsum[2 * R + 1];
      ww = dsum[2 * R];
      if (gd) {
        ginv_apply();
        double q = 0.0;   // Re(c^H G^{-1} c)
        for (int ra = 0; ra < r; ++ra) q += dsum[2 * ra] * gx[ra].x + dsum[2 * ra + 1] * gx[ra].y;
        ww = fmax(ww - q, 0.0);
      }
    }
    const bool okmu = ww > 0.0 && isfinite(ww) && isfinite(gg);
    const float mu = okmu ? (float)(gg / ww) : 0.f;
    // v = s - mu g in grid A, then HardThreshold
    for (int t = tid; t < gsize; t += kFThreads) gA[t] = c_scale(gA[t], -mu);
    for (int t = tid; t < words; t += kFThreads) mark[t] = 0u;
    __syncthreads();
    for (int e = tid; e < rho; e += kFThreads) {
      const int j = sidx[e];
      gA[pos(j)] = c_add(gA[pos(j)], sval[e]);
      atomicOr(&mark[j >> 5], 1u << (j & 31));
    }
    __syncthreads();
    // most steps keep T: then sidx (ascending) is already the selection
    if (!fsupport_kept([&](int j) { return gA[pos(j)]; }, n, mark, reinterpret_cast<unsigned*>(red)))
      flags |= fselect([&](int j) { return gA[pos(j)]; }, n, rho, sidx, hist, tmp) ? 1 : 0;
    int moved = 0;
    for (int e = tid; e < rho; e += kFThreads) {
      const int j = sidx[e];
      sval[e] = gA[pos(j)];
      moved |= ((mark[j >> 5] >> (j & 31)) & 1u) ^ 1u;
    }
    known = !fblock_any(moved, tmp);
    if (known && mu != 0.f)
#pragma unroll
      for (int e = 0; e < 2; ++e) as[e] = c_sub(as[e], c_scale(w[e], mu));
    have = true;
  }

  // A_k s_k and e_k = y_k - A_k s_k
  float2 ev[2];
  if (rho > 0 && !known) apply_sparse(sidx, sval, rho, as);
#pragma unroll
  for (int e = 0; e < 2; ++e) ev[e] = ok[e] ? c_sub(yv[e], as[e]) : make_float2(0.f, 0.f);

  float2* Hk = a.H + (long long)k * n;
  if (gd) {
    // b_k = G_k^{-1} P_k^H e_k; r_k = P_k b_k - e_k; h_k = A_k^H r_k
    double c[2 * R + 1];
#pragma unroll
    for (int cc = 0; cc < 2 * R + 1; ++cc) c[cc] = 0.0;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      float2 p[R];
      Prow(e, p);
#pragma unroll
      for (int cc = 0; cc < R; ++cc) {
        c[2 * cc] += (double)p[cc].x * ev[e].x + (double)p[cc].y * ev[e].y;
        c[2 * cc + 1] += (double)p[cc].x * ev[e].y - (double)p[cc].y * ev[e].x;
      }
      c[2 * R] += (double)ev[e].x * ev[e].x + (double)ev[e].y * ev[e].y;
    }
    fblock_sum<2 * R + 1>(c, red, dsum);
    ginv_apply();
    float2 b[R];
#pragma unroll
    for (int ra = 0; ra < R; ++ra) b[ra] = ra < r ? make_float2((float)gx[ra].x, (float)gx[ra].y) : make_float2(0.f, 0.f);
    if (tid < r) {
      float2 bo = b[0];
#pragma unroll
      for (int ra = 0; ra < R; ++ra)
        if (ra == tid) bo = b[ra];
      a.Bt[(long long)k * r + tid] = bo;
    }
    // ||r_k||^2 = ||e_k||^2 - Re(c^H b_k), since G_k b_k = c = P_k^H e_k
    double cb_re = 0.0;
    for (int ra = 0; ra < r; ++ra) cb_re += dsum[2 * ra] * gx[ra].x + dsum[2 * ra + 1] * gx[ra].y;
    const double d_rr = dsum[2 * R] - cb_re;
    const double rr = d_rr < 0.0 ? 0.0 : d_rr;   // rounding below zero clamped; a NaN stays NaN
    if (tid == 0) a.colrr[k] = rr;
    __syncthreads();   // dsum is read above by every thread
    float2 rv[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      float2 p[R];
      Prow(e, p);
      float2 s = make_float2(-ev[e].x, -ev[e].y);
#pragma unroll
      for (int ra = 0; ra < R; ++ra) s = c_add(s, c_mul(p[ra], b[ra]));
      rv[e] = ok[e] ? s : make_float2(0.f, 0.f);
    }
    apply_adj(rv);
  } else {
    // initialisation: ||y_k||^2 and the column A_k^H (y_k - A_k s_k) of L_0
    const double yy = sum_sq(yv);
    if (tid == 0) a.colrr[k] = yy;
    apply_adj(ev);
  }
  for (int j = tid; j < n; j += kFThreads) Hk[j] = gA[pos(j)];
  for (int e = tid; e < rho; e += kFThreads) {
    a.Sidx[(long long)k * rho + e] = sidx[e];
    a.Sval[(long long)k * rho + e] = sval[e];
  }
  if (flags) atomicOr(&a.flags[k], flags);
}

// ---------------------------------------------------------------- U side

// F U, the unitary 2D DFT of each of U's r columns (n x r, row-major; frame
// element (j1, j2) at row j1 * 96 + j2), in two launches that each give one
// 96-point line to a group of 32 lanes: PASS 0 transforms the rows (j1, c) of U
// into FU, PASS 1 the columns (u2, c) of FU in place, with the 1/96 scale (the
// same transform and scaling as fft2_grid).  A group reads its whole line before
// it writes (the lane exchanges need every lane's loads), and no two groups share
// an element, so the column pass can run in place.  kFN r is even, so a wave's
// two groups exit together.
template <int PASS>
__global__ __launch_bounds__(64) void k_fu(const float2* U, int r, const float2* tw, float2* FU) {
  const int gid = blockIdx.x * 2 + (threadIdx.x >> 5), l = threadIdx.x & 31;
  if (gid >= kFN * r) return;
  const int line = gid / r, c = gid - line * r;
  const int k1 = (int)(__builtin_bitreverse32((unsigned)l) >> 27);
  const long long stride = PASS == 0 ? (long long)r : (long long)kFN * r;
  const long long base = PASS == 0 ? (long long)line * kFN * r + c : (long long)line * r + c;
  const float2* src = (PASS == 0 ? U : FU) + base;
  float2 v[3] = {src[l * stride], src[(l + 32) * stride], src[(l + 64) * stride]};
  fft96<false>(v, l, tw);
  float2* dst = FU + base;
  const float s = 1.0f / kFN;
#pragma unroll
  for (int a = 0; a < 3; ++a) dst[(3 * k1 + a) * stride] = PASS == 0 ? v[a] : c_scale(v[a], s);
}

// F U for a generic frame: one workgroup per column c of U; the column is staged
// in LDS, transformed by dft2_gen and written back (the same transform and scale
// as the column kernel's).
__global__ __launch_bounds__(kFThreads) void k_fu_gen(const float2* U, int n, int r, int n1, int n2,
                                                      const float2* tw, float2* FU) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  float2* grid = reinterpret_cast<float2*>(smem);
  float2* twl = grid + n;
  const int c = blockIdx.x;
  for (int t = threadIdx.x; t < n1 + n2; t += kFThreads) twl[t] = tw[t];
  for (int j = threadIdx.x; j < n; j += kFThreads) grid[j] = U[(long long)j * r + c];
  __syncthreads();
  dft2_gen<false>(grid, twl, n1, n2, (float)(1.0 / sqrt((double)n)));
  for (int j = threadIdx.x; j < n; j += kFThreads) FU[(long long)j * r + c] = grid[j];
}

// Tc[k][c] = sum_j H[k][j] conj(U[j][c]) (so that L_0 (L_0^H U) = sum_k h_k conj(Tc[k]) ^ T).
template <int R>
__global__ __launch_bounds__(kFThreads) void k_fltu(const float2* H, const float2* U, int n, int r, float2* Tc,
                                                    const int* skip) {
  if (skip && *skip) return;
  __shared__ double red[kFWaves * 2 * kFRMax];
  __shared__ double out[2 * kFRMax];
  const int k = blockIdx.x, tid = threadIdx.x;
  double v[2 * R];
#pragma unroll
  for (int i = 0; i < 2 * R; ++i) v[i] = 0.0;
  for (int j = tid; j < n; j += kFThreads) {
    const float2 h = H[(long long)k * n + j];
#pragma unroll
    for (int c = 0; c < R; ++c)
      if (c < r) {
        const float2 u = U[(long long)j * r + c];
        v[2 * c] += (double)h.x * u.x + (double)h.y * u.y;
        v[2 * c + 1] += (double)h.y * u.x - (double)h.x * u.y;
      }
  }
  fblock_sum<2 * R>(v, red, out);
  if (tid < r) Tc[(long long)k * r + tid] = make_float2((float)out[2 * tid], (float)out[2 * tid + 1]);
}

// Rows of Gsum[j][c] = sum_k H[k][j] conj(B[k][c]) (grad_U f with B = B_t;
// L_0 (L_0^H U) with B = Tc) for the 256 rows j of block blockIdx.x, by 1024
// threads: thread t takes row t % 256 and the k range of split s = t / 256 (the
// four quarters of 0 .. q - 1, each summed in order); the splits are added as
// (s0 + s2) + (s1 + s3) through buf (2 x 256 x R float2 of LDS).  Threads of
// split 0 return true and hold the row in acc.
constexpr int kFGradSplits = 4;

template <int R>
__device__ bool fgrad_rows(const float2* H, const float2* B, int n, int q, int r, float2 (&acc)[R], float2* buf) {
  const int tid = threadIdx.x, row = tid & 255, sp = tid >> 8;
  const int j = blockIdx.x * 256 + row;
  const int jc = j < n ? j : n - 1;
  const int k0 = q * sp / kFGradSplits, k1 = q * (sp + 1) / kFGradSplits;
#pragma unroll
  for (int c = 0; c < R; ++c) acc[c] = make_float2(0.f, 0.f);
  constexpr int KU = 8;   // loads in flight per thread; the k order of the sum does not depend on it
  for (int kb = k0; kb < k1; kb += KU) {
    float2 h[KU];
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int k = kb + u < k1 ? kb + u : k0;
      h[u] = H[(long long)k * n + jc];
    }
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      if (kb + u < k1) {
        const int k = kb + u;
#pragma unroll
        for (int c = 0; c < R; ++c)
          if (c < r) {
            const float2 b = B[(long long)k * r + c];
            acc[c].x = fmaf(h[u].x, b.x, fmaf(h[u].y, b.y, acc[c].x));
            acc[c].y = fmaf(h[u].y, b.x, fmaf(-h[u].x, b.y, acc[c].y));
          }
      }
    }
  }
  auto put = [&](int slot) {
#pragma unroll
    for (int c = 0; c < R; ++c) buf[(slot * 256 + row) * R + c] = acc[c];
  };
  auto add = [&](int slot) {
#pragma unroll
    for (int c = 0; c < R; ++c) {
      const float2 o = buf[(slot * 256 + row) * R + c];
      acc[c].x += o.x;
      acc[c].y += o.y;
    }
  };
  if (sp >= 2) put(sp - 2);
  __syncthreads();
  if (sp < 2) add(sp);
  __syncthreads();
  if (sp == 1) put(0);
  __syncthreads();
  if (sp == 0) add(0);
  __syncthreads();   // buf is free again
  return sp == 0;
}

namespace {

// Largest eigenvalue of a real symmetric N x N matrix (row-major, destroyed) by
// cyclic Jacobi rotations; one thread.
__device__ double jacobi_lmax(double* A, int N) {
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) {
        tot += A[i * N + j] * A[i * N + j];
        if (i != j) off += A[i * N + j] * A[i * N + j];
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < N - 1; ++p)
      for (int q = p + 1; q < N; ++q) {
        const double apq = A[p * N + q];
        if (apq == 0.0) continue;
        const double theta = (A[q * N + q] - A[p * N + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < N; ++k) {
          const double akp = A[k * N + p], akq = A[k * N + q];
          A[k * N + p] = cs * akp - sn * akq;
          A[k * N + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < N; ++k) {
          const double apk = A[p * N + k], aqk = A[q * N + k];
          A[p * N + k] = cs * apk - sn * aqk;
          A[q * N + k] = sn * apk + cs * aqk;
        }
      }
  }
  double l = A[0];
  for (int i = 1; i < N; ++i) l = fmax(l, A[i * N + i]);
  return l;
}

// W (r x r, complex FP64) = X^H Y over the n rows of the row-major n x r X and Y
// (global memory).  Whole rows are staged through LDS 256 at a time (coalesced
// copies; the next chunk is loaded into registers while the current one is
// summed), so each element is read from memory once.  Wave w computes the
// entries e = w, w + 16, ... (with sym, the entries a <= b only, the others by
// conjugation); per entry the lanes stride over the rows j = lane, lane + 64, ...
// in order and the lane sums are added by the fixed DPP tree.  stage holds
// 2 x 256 x kFRMax float2.  Ends with a barrier.  (Not inlined: inlined at its
// three call sites it pushed k_fqr<6> past 128 VGPRs.)
template <int R>
__device__ __noinline__ void fgram(const float2* X, const float2* Y, int n, int r, float2* stage, double2* W,
                                   bool sym = true) {
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
  constexpr int CH = 256;
  constexpr int kEW = (kFRMax * kFRMax + kFWaves - 1) / kFWaves;   // entries of one wave, at most
  const bool same = X == Y;
  float2* Xs = stage;
  float2* Ys = same ? stage : stage + CH * kFRMax;
  const int E = sym ? r * (r + 1) / 2 : r * r;
  int ra[kEW], rb[kEW];
  double sr[kEW], si[kEW];
#pragma unroll
  for (int t = 0; t < kEW; ++t) {
    const int e = wave + t * kFWaves;
    int a = 0, b = 0;
    if (e < E) {
      if (sym) {
        int base = 0;
        while (e >= base + (r - a)) {
          base += r - a;
          ++a;
        }
        b = a + (e - base);
      } else {
        a = e / r;
        b = e - a * r;
      }
    }
    ra[t] = a;
    rb[t] = b;
    sr[t] = 0.0;
    si[t] = 0.0;
  }
  const int nch = (n + CH - 1) / CH;
  float2 xv[2], yv[2];   // this thread's share of a chunk: at most 256 x 8 / 1024 = 2 elements
  auto fetch = [&](int c) {
    const long long o = (long long)c * CH * r;
    const int cnt = min(CH, n - c * CH) * r;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int i = tid + u * kFThreads;
      if (i < cnt) {
        xv[u] = X[o + i];
        if (!same) yv[u] = Y[o + i];
      }
    }
  };
  fetch(0);
  for (int c = 0; c < nch; ++c) {
    const int rows = min(CH, n - c * CH);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int i = tid + u * kFThreads;
      if (i < rows * r) {
        Xs[i] = xv[u];
        if (!same) Ys[i] = yv[u];
      }
    }
    __syncthreads();
    if (c + 1 < nch) fetch(c + 1);
#pragma unroll
    for (int t = 0; t < kEW; ++t) {
      if (wave + t * kFWaves < E) {
        for (int jl = lane; jl < rows; jl += 64) {   // conj(X[j][ra]) Y[j][rb]
          const float2 x = Xs[jl * r + ra[t]], y = Ys[jl * r + rb[t]];
          sr[t] = fma((double)x.x, (double)y.x, fma((double)x.y, (double)y.y, sr[t]));
          si[t] = fma((double)x.x, (double)y.y, fma(-(double)x.y, (double)y.x, si[t]));
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < kEW; ++t) {
    if (wave + t * kFWaves < E) {
      const double vr = wave_sum_dpp(sr[t]);
      const double vi = wave_sum_dpp(si[t]);
      if (lane == 0) {
        W[ra[t] * r + rb[t]] = make_double2(vr, vi);
        if (sym) W[rb[t] * r + ra[t]] = make_double2(vr, -vi);
      }
    }
  }
  __syncthreads();
}

// Cholesky W = L L^H of a Hermitian positive definite r x r matrix (complex FP64,
// row-major in LDS), real positive diagonal, by one wave in LDS, right-looking:
// the lower triangle of W is copied to L; at step j column j is scaled by
// lane-parallel products with 1 / L_jj and the trailing lower triangle is
// updated by all lanes.  Returns false (wave-uniform) if a pivot is not
// positive.  All 64 lanes call it; the LDS accesses of one wave complete in order.
__device__ bool wave_chol_c(const double2* W, double2* L, int r) {
  const int lane = threadIdx.x & 63;
  for (int e = lane; e < r * r; e += 64)
    if (e % r <= e / r) L[e] = W[e];
  __builtin_amdgcn_s_waitcnt(0);
  __builtin_amdgcn_wave_barrier();
  for (int j = 0; j < r; ++j) {
    const double piv = L[j * r + j].x;
    if (!(piv > 0.0)) return false;
    const double d = sqrt(piv);
    const double inv = 1.0 / d;
    if (lane == j) {
      L[j * r + j] = make_double2(d, 0.0);
    } else if (lane > j && lane < r) {
      const double2 v = L[lane * r + j];
      L[lane * r + j] = make_double2(v.x * inv, v.y * inv);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    const int t = r - j - 1;   // trailing size
    for (int e = lane; e < t * t; e += 64) {
      const int i = j + 1 + e / t, k = j + 1 + e % t;
      if (k <= i) {   // L[i][k] -= L[i][j] conj(L[k][j])
        const double2 a = L[i * r + j], b = L[k * r + j], w = L[i * r + k];
        L[i * r + k] = make_double2(w.x - (a.x * b.x + a.y * b.y), w.y - (a.y * b.x - a.x * b.y));
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
  }
  return true;
}

// Rinv = (L^H)^{-1} (upper triangular, complex FP64) from the factor of
// wave_chol_c, by one wave: lane c solves L m = e_c by forward substitution (the
// rows of L read from LDS) and writes Rinv[c][i] = conj(m[i]) to dst (r x r,
// row-major).  All 64 lanes of the wave that factored call it.
template <int R>
__device__ void wave_rinv_c(const double2* L, double2* dst, int r) {
  const int c = threadIdx.x & 63;
  if (c < r) {
    double2 mc[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      double mr = 0.0, mi = 0.0;
      if (i < r && i >= c) {
        mr = (i == c) ? 1.0 : 0.0;
#pragma unroll
        for (int p = 0; p < R; ++p)
          if (p >= c && p < i) {   // - L[i][p] m[p]
            const double2 a = L[i * r + p];
            mr -= a.x * mc[p].x - a.y * mc[p].y;
            mi -= a.x * mc[p].y + a.y * mc[p].x;
          }
        const double dd = L[i * r + i].x;
        mr /= dd;
        mi /= dd;
      }
      mc[i] = make_double2(mr, mi);
    }
#pragma unroll
    for (int i = 0; i < R; ++i)
      if (i < r) dst[c * r + i] = make_double2(mc[i].x, -mc[i].y);
  }
}

// dst[0 .. count) = src[0 .. count) (complex values, 16-byte aligned arrays) by the
// workgroup with 16-byte accesses, 8 in flight per thread.
__device__ __forceinline__ void block_copy_c(float2* dst, const float2* src, int count) {
  const int tid = threadIdx.x;
  const int n4 = count >> 1;   // two complex values per float4
  typedef float f32x4_c __attribute__((ext_vector_type(4)));
  const f32x4_c* s4 = reinterpret_cast<const f32x4_c*>(src);
  f32x4_c* d4 = reinterpret_cast<f32x4_c*>(dst);
  constexpr int U = 8;
  int i = tid;
  for (; i + (U - 1) * kFThreads < n4; i += U * kFThreads) {
    f32x4_c v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = s4[i + u * kFThreads];
#pragma unroll
    for (int u = 0; u < U; ++u) d4[i + u * kFThreads] = v[u];
  }
  for (; i < n4; i += kFThreads) d4[i] = s4[i];
  if ((count & 1) && tid == 0) dst[count - 1] = src[count - 1];
}

// One CholeskyQR pass on X (n x r in global memory): X <- X R^{-1}, R = L^H from
// X^H X = L L^H.  Returns false if X^H X is not positive definite.
template <int R>
__device__ bool fcholqr_pass(float2* X, int n, int r, float2* stage, double2* W, double2* Lm, int* okf) {
  const int tid = threadIdx.x;
  fgram<R>(X, X, n, r, stage, W);
  if (tid < 64) {
    const bool ok = wave_chol_c(W, Lm, r);
    if (tid == 0) *okf = ok ? 1 : 0;
  }
  __syncthreads();
  if (!*okf) return false;
  // row x <- x R^{-1}: q[c] = (x[c] - sum_{p<c} q[p] R[p][c]) / R[c][c], R[p][c] = conj(L[c][p])
  for (int j = tid; j < n; j += kFThreads) {
    float2 x[R];
    double2 qd[R];
#pragma unroll
    for (int c = 0; c < R; ++c) x[c] = c < r ? X[(long long)j * r + c] : make_float2(0.f, 0.f);
#pragma unroll
    for (int c = 0; c < R; ++c) {
      double tr = x[c].x, ti = x[c].y;
#pragma unroll
      for (int p = 0; p < c; ++p) {   // q[p] * conj(L[c][p])
        const double2 l = c < r ? Lm[c * r + p] : make_double2(0.0, 0.0);
        tr -= qd[p].x * l.x + qd[p].y * l.y;
        ti -= qd[p].y * l.x - qd[p].x * l.y;
      }
      const double d = c < r ? Lm[c * r + c].x : 1.0;
      qd[c] = make_double2(tr / d, ti / d);
    }
#pragma unroll
    for (int c = 0; c < R; ++c)
      if (c < r) X[(long long)j * r + c] = make_float2((float)qd[c].x, (float)qd[c].y);
  }
  __syncthreads();
  return true;
}

}  // namespace

// U <- QR(Utmp) (CholeskyQR2, real positive diagonal): the orthonormal start of
// the subspace iteration.  One workgroup.  (The GD update and the subspace steps
// run over many workgroups: k_fqr_a .. k_fqr_f.)
template <int R>
__global__ __launch_bounds__(kFThreads) void k_fqr(FQRArgs a) {
  __shared__ float2 stage[2 * 256 * kFRMax];   // rows staged by fgram
  __shared__ double2 W[kFRMax * kFRMax];
  __shared__ double2 Lm[kFRMax * kFRMax];
  __shared__ int okf;
  const int tid = threadIdx.x, n = a.n, r = a.r, nr = n * r;
  float2* X = a.Utmp;
  bool ok = fcholqr_pass<R>(X, n, r, stage, W, Lm, &okf);
  if (ok) ok = fcholqr_pass<R>(X, n, r, stage, W, Lm, &okf);
  if (!ok) {
    if (tid == 0) atomicOr(&a.ctl->err, 2);
    return;
  }
  block_copy_c(a.U, X, nr);
}

__global__ void k_ftwiddle(float2* tw) {
  const int t = threadIdx.x;
  if (t < kFN) {
    double s, c;
    sincospi(-2.0 * t / kFN, &s, &c);
    tw[t] = make_float2((float)c, (float)s);
  }
}

// Twiddles of a generic frame: W_n1^t (t < n1), then W_n2^t (t < n2), W_N = exp(-2 pi i / N).
__global__ void k_ftwiddle_gen(float2* tw, int n1, int n2) {
  for (int t = threadIdx.x + blockIdx.x * blockDim.x; t < n1 + n2; t += blockDim.x * gridDim.x) {
    const int N = t < n1 ? n1 : n2, e = t < n1 ? t : t - n1;
    double s, c;
    sincospi(-2.0 * e / N, &s, &c);
    tw[t] = make_float2((float)c, (float)s);
  }
}

__global__ void k_fbasis(float2* U, int n, int r) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < (long long)n * r;
       i += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(i / r), c = (int)(i % r);
    U[i] = make_float2((j % r == c) ? 1.f : 0.f, 0.f);
  }
}

// ---------------------------------------------------------------- GD update over many workgroups
//
// The projected GD step U+ = QR(U - eta grad) of Alg. 1 for the Fourier form,
// split so that the n x r arrays are streamed by many CUs:
//   k_fgrad_gd : rows of grad (four column splits per 1024-thread workgroup,
//                added in a fixed order) and, per 256-row block, the partial
//                Grams U^H U, U^H G, G^H G (wave per entry, lanes over rows);
//   k_fqr_a    : one workgroup: sums the partials in block order, eta at t = 1,
//                the Gram of X = U - eta G by expansion, its Cholesky factor and
//                R1^{-1} (one wave); the residual and the iteration counter;
//   k_fqr_b    : X = (U - eta G) R1^{-1} row by row, partial Grams of X;
//   k_fqr_c    : one workgroup: R2^{-1} from the Gram of X;
//   k_fqr_d    : U_prev = U, U = X R2^{-1}.
// CholeskyQR2 as in k_fqr, with the first Gram taken from the expansion
// U^H U - eta (U^H G + G^H U) + eta^2 G^H G of the unrounded U - eta G.
//
// The initialisation's subspace iteration (mode QR_POWER) runs the same chain
// on G = L_0 (L_0^H U): k_fqr_a takes the first Gram as G^H G, k_fqr_b forms
// X = G R1^{-1}, and k_fqr_d adds per-block partial Grams U_prev^H U; then
//   k_fqr_e    : W = U_prev^H U from the partials, per-block sums of
//                |U - U_prev W|^2 over the rows (the subspace change);
//   k_fqr_f    : one thread: the change, the step counter and the stop rule.
// Every kernel of the chain returns at once after the stop rule has fired.

namespace {

// sum over b = 0 .. nb - 1 of p[b * stride], in that order; the loads go out 8 at a time.
__device__ __forceinline__ double2 sum_blocks(const double2* p, long long stride, int nb) {
  double sr = 0.0, si = 0.0;
  int b = 0;
  for (; b + 8 <= nb; b += 8) {
    double2 v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = p[(long long)(b + u) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      sr += v[u].x;
      si += v[u].y;
    }
  }
  for (; b < nb; ++b) {
    const double2 v = p[(long long)b * stride];
    sr += v.x;
    si += v.y;
  }
  return make_double2(sr, si);
}

// Partial Gram of the 256 LDS rows Xl, Yl (rows x r complex): dst[a * r + b] =
// sum_rows conj(X[a]) Y[b]; the workgroup's waves take entries w, w + waves, ...;
// with sym only a <= b are summed and the rest mirrored.
__device__ void rows_gram(const float2* Xl, const float2* Yl, int r, bool sym, double2* dst) {
  const int lane = threadIdx.x & 63, wave = wave_id(), waves = blockDim.x >> 6;
  const int E = sym ? r * (r + 1) / 2 : r * r;
  for (int e = wave; e < E; e += waves) {
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
    double sr = 0.0, si = 0.0;
    for (int j = lane; j < 256; j += 64) {
      const float2 x = Xl[j * r + ra], y = Yl[j * r + rb];
      sr = fma((double)x.x, (double)y.x, fma((double)x.y, (double)y.y, sr));
      si = fma((double)x.x, (double)y.y, fma(-(double)x.y, (double)y.x, si));
    }
    sr = wave_sum_dpp(sr);
    si = wave_sum_dpp(si);
    if (lane == 0) {
      dst[ra * r + rb] = make_double2(sr, si);
      if (sym) dst[rb * r + ra] = make_double2(sr, -si);
    }
  }
}

}  // namespace

template <int R>
__global__ __launch_bounds__(kFThreads) void k_fgrad_gd(const float2* H, const float2* B, const float2* U, int n, int q,
                                                        int r, float2* Gsum, double2* part, const int* skip) {
  if (skip && *skip) return;
  __shared__ float2 sm[2 * 256 * R];   // the split sums first, then U and grad rows
  float2* Ul = sm;
  float2* Gl = sm + 256 * R;
  float2 acc[R];
  const bool mine = fgrad_rows<R>(H, B, n, q, r, acc, sm);
  const int tid = threadIdx.x, j = blockIdx.x * 256 + (tid & 255);
  if (mine) {
#pragma unroll
    for (int c = 0; c < R; ++c)
      if (c < r) {
        const bool in = j < n;
        if (in) Gsum[(long long)j * r + c] = acc[c];
        Gl[tid * r + c] = in ? acc[c] : make_float2(0.f, 0.f);
        Ul[tid * r + c] = in ? U[(long long)j * r + c] : make_float2(0.f, 0.f);
      }
  }
  __syncthreads();
  double2* slot = part + (long long)blockIdx.x * 3 * r * r;
  rows_gram(Ul, Ul, r, true, slot);
  rows_gram(Ul, Gl, r, false, slot + r * r);
  rows_gram(Gl, Gl, r, true, slot + 2 * r * r);
}

__global__ __launch_bounds__(256) void k_fqr_a(FQRArgs a) {
  __shared__ double2 S[3 * kFRMax * kFRMax], Lm[kFRMax * kFRMax];
  __shared__ double Mr[4 * kFRMax * kFRMax];
  __shared__ double red[4];
  __shared__ double eta_s;
  if (a.mode == QR_POWER && a.ctl->conv) return;
  const int tid = threadIdx.x, r = a.r, rr = r * r;
  double2* W = reinterpret_cast<double2*>(Mr);
  for (int e = tid; e < 3 * rr; e += 256) S[e] = sum_blocks(a.part + e, 3 * rr, a.nb);
  __syncthreads();
  const double2* UU = S;
  const double2* UG = S + rr;
  const double2* GG = S + 2 * rr;
  if (tid == 0 && a.mode == QR_POWER) {
    for (int e = 0; e < rr; ++e) W[e] = GG[e];   // X = G: its Gram
  } else if (tid == 0) {
    double eta;
    if (!a.ctl->eta_set) {
      const int N = 2 * r;   // Hermitian GG = A + iB -> real symmetric [[A, -B], [B, A]]
      for (int i = 0; i < r; ++i)
        for (int jj = 0; jj < r; ++jj) {
          const double2 w = GG[i * r + jj];
          Mr[i * N + jj] = w.x;
          Mr[(i + r) * N + jj + r] = w.x;
          Mr[i * N + jj + r] = -w.y;
          Mr[(i + r) * N + jj] = w.y;
        }
      const double lam = jacobi_lmax(Mr, N);
      eta = lam > 0.0 ? a.eta_c / sqrt(lam) : 0.0;
      a.ctl->eta = eta;
      a.ctl->eta_set = 1;
    } else {
      eta = a.ctl->eta;
    }
    eta_s = eta;
    // Gram of X = U - eta G: UU - eta (UG + UG^H) + eta^2 GG
    for (int i = 0; i < r; ++i)
      for (int jj = 0; jj < r; ++jj) {
        const double2 uu = UU[i * r + jj], ug = UG[i * r + jj], gu = UG[jj * r + i], gg = GG[i * r + jj];
        W[i * r + jj] = make_double2(uu.x - eta * (ug.x + gu.x) + eta * eta * gg.x,
                                     uu.y - eta * (ug.y - gu.y) + eta * eta * gg.y);
      }
  }
  __syncthreads();
  if (tid < 64) {
    const bool ok = wave_chol_c(W, Lm, r);
    if (ok) wave_rinv_c<kFRMax>(Lm, a.rinv, r);
    if (!ok && tid == 0) {
      atomicOr(&a.ctl->err, 2);
      for (int e = 0; e < rr; ++e) a.rinv[e] = make_double2((e % (r + 1) == 0) ? 1.0 : 0.0, 0.0);
    }
  }
  if (a.mode == QR_POWER) return;
  // the residual of the iteration (colrr in column order) and the counters
  double s = 0.0;
  int fl = 0;
  for (int k = tid; k < a.q; k += 256) {
    s += a.colrr[k];
    fl |= a.colflags[k];
  }
  s = wave_sum_dpp(s);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  if (fl) atomicOr(&a.ctl->err, fl);
  __syncthreads();
  if (tid == 0) {
    const double ss = (red[0] + red[1]) + (red[2] + red[3]);
    const double resid = a.ctl->ynorm2 > 0.0 ? sqrt(ss / a.ctl->ynorm2) : sqrt(ss);
    const int t = a.ctl->t;
    if (a.rlog && t < a.rlog_len) a.rlog[t] = resid;
    a.ctl->resid = resid;
    a.ctl->t = t + 1;
    a.ctl->prev_resid = resid;
  }
}

// X = (U - eta G) R1^{-1} (FP64 per row, stored FP32) and the partial Grams of X.
template <int R>
__global__ __launch_bounds__(256) void k_fqr_b(FQRArgs a) {
  __shared__ float2 Xl[256 * kFRMax];
  if (a.mode == QR_POWER && a.ctl->conv) return;
  const int tid = threadIdx.x, j = blockIdx.x * 256 + tid, r = a.r;
  const bool power = a.mode == QR_POWER;
  const double eta = power ? -1.0 : a.ctl->eta;   // POWER: X = G
  double2 x[R];
#pragma unroll
  for (int c = 0; c < R; ++c) {
    x[c] = make_double2(0.0, 0.0);
    if (c < r && j < a.n) {
      const float2 u = power ? make_float2(0.f, 0.f) : a.U[(long long)j * r + c], g = a.G[(long long)j * r + c];
      x[c] = make_double2(fma(-eta, (double)g.x, (double)u.x), fma(-eta, (double)g.y, (double)u.y));
    }
  }
#pragma unroll
  for (int c = 0; c < R; ++c)
    if (c < r) {
      double tr = 0.0, ti = 0.0;
#pragma unroll
      for (int aa = 0; aa < R; ++aa)
        if (aa <= c) {   // x[aa] Rinv[aa][c]
          const double2 m = a.rinv[aa * r + c];
          tr += x[aa].x * m.x - x[aa].y * m.y;
          ti += x[aa].x * m.y + x[aa].y * m.x;
        }
      const float2 v = make_float2((float)tr, (float)ti);
      if (j < a.n) a.Utmp[(long long)j * r + c] = v;
      Xl[tid * r + c] = j < a.n ? v : make_float2(0.f, 0.f);
    }
  __syncthreads();
  rows_gram(Xl, Xl, r, true, a.part + (long long)blockIdx.x * r * r);
}

__global__ __launch_bounds__(256) void k_fqr_c(FQRArgs a) {
  __shared__ double2 W[kFRMax * kFRMax], Lm[kFRMax * kFRMax];
  if (a.mode == QR_POWER && a.ctl->conv) return;
  const int tid = threadIdx.x, rr = a.r * a.r;
  for (int e = tid; e < rr; e += 256) W[e] = sum_blocks(a.part + e, rr, a.nb);
  __syncthreads();
  if (tid < 64) {
    const bool ok = wave_chol_c(W, Lm, a.r);
    if (ok) wave_rinv_c<kFRMax>(Lm, a.rinv + rr, a.r);
    if (!ok && tid == 0) {
      atomicOr(&a.ctl->err, 2);
      for (int e = 0; e < rr; ++e) a.rinv[rr + e] = make_double2((e % (a.r + 1) == 0) ? 1.0 : 0.0, 0.0);
    }
  }
}

// U_prev = U; U = X R2^{-1}.  POWER: also the per-block partial Grams U_prev^H U.
template <int R>
__global__ __launch_bounds__(256) void k_fqr_d(FQRArgs a) {
  __shared__ float2 Ol[256 * R], Nl[256 * R];
  const bool power = a.mode == QR_POWER;
  if (power && a.ctl->conv) return;
  const int tid = threadIdx.x, j = blockIdx.x * 256 + tid, r = a.r;
  const bool in = j < a.n;
  const double2* Ri = a.rinv + r * r;
  double2 x[R];
#pragma unroll
  for (int c = 0; c < R; ++c) {
    const float2 v = (in && c < r) ? a.Utmp[(long long)j * r + c] : make_float2(0.f, 0.f);
    x[c] = make_double2(v.x, v.y);
  }
#pragma unroll
  for (int c = 0; c < R; ++c)
    if (c < r) {
      double tr = 0.0, ti = 0.0;
#pragma unroll
      for (int aa = 0; aa < R; ++aa)
        if (aa <= c) {
          const double2 m = Ri[aa * r + c];
          tr += x[aa].x * m.x - x[aa].y * m.y;
          ti += x[aa].x * m.y + x[aa].y * m.x;
        }
      const float2 un = make_float2((float)tr, (float)ti);
      const float2 uo = in ? a.U[(long long)j * r + c] : make_float2(0.f, 0.f);
      if (in) {
        a.Uprev[(long long)j * r + c] = uo;
        a.U[(long long)j * r + c] = un;
      }
      if (power) {
        Ol[tid * r + c] = uo;
        Nl[tid * r + c] = in ? un : make_float2(0.f, 0.f);
      }
    }
  if (!power) return;
  __syncthreads();
  rows_gram(Ol, Nl, r, false, a.part + (long long)blockIdx.x * r * r);
}

// POWER: W = U_prev^H U summed from the per-block partials (in block order, by
// every workgroup), then the block's sum of |U[j] - U_prev[j] W|^2 over its rows
// (FP64 per row, the 256 row sums added by the fixed DPP tree and the 4 wave
// totals in order) into part[nb r^2 + block].x.
template <int R>
__global__ __launch_bounds__(256) void k_fqr_e(FQRArgs a) {
  __shared__ double2 Wl[kFRMax * kFRMax];
  __shared__ double wsum[4];
  if (a.ctl->conv) return;
  const int tid = threadIdx.x, j = blockIdx.x * 256 + tid, r = a.r, rr = r * r;
  for (int e = tid; e < rr; e += 256) Wl[e] = sum_blocks(a.part + e, rr, a.nb);
  __syncthreads();
  double acc = 0.0;
  if (j < a.n) {
    float2 u[R];
#pragma unroll
    for (int e = 0; e < R; ++e) u[e] = e < r ? a.Uprev[(long long)j * r + e] : make_float2(0.f, 0.f);
#pragma unroll
    for (int c = 0; c < R; ++c)
      if (c < r) {
        const float2 xv = a.U[(long long)j * r + c];
        double dx = (double)xv.x, dy = (double)xv.y;
#pragma unroll
        for (int e = 0; e < R; ++e)
          if (e < r) {
            const double2 w = Wl[e * r + c];
            dx -= (double)u[e].x * w.x - (double)u[e].y * w.y;
            dy -= (double)u[e].x * w.y + (double)u[e].y * w.x;
          }
        acc += dx * dx + dy * dy;
      }
  }
  acc = wave_sum_dpp(acc);
  if ((tid & 63) == 0) wsum[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) a.part[(long long)a.nb * rr + blockIdx.x] = make_double2((wsum[0] + wsum[1]) + (wsum[2] + wsum[3]), 0.0);
}

// POWER: the subspace change from the block sums (in block order), the step
// counter and the stop rule.
__global__ void k_fqr_f(FQRArgs a) {
  if (threadIdx.x != 0 || a.ctl->conv) return;
  const double f = sum_blocks(a.part + (long long)a.nb * a.r * a.r, 1, a.nb).x;
  const double sd = sqrt(f);
  const double prev = a.ctl->power_sd;   // 0 before the first step
  a.ctl->power_sd = sd;
  a.ctl->power_it += 1;
  // as in k_fqr: converged at power_tol, or once the change has stopped
  // shrinking below 1e-3 (by less than 1 % in a step)
  if (sd <= a.power_tol || (sd <= 1e-3 && prev > 0.0 && sd >= 0.99 * prev)) a.ctl->conv = 1;
}

// ---------------------------------------------------------------- launchers

#define FR_SWITCH(R_, CALL)  \
  switch (R_) {              \
    case 2: CALL(2); break;  \
    case 4: CALL(4); break;  \
    case 6: CALL(6); break;  \
    default: CALL(8); break; \
  }

static int fr_bucket(int r) { return r <= 2 ? 2 : (r <= 4 ? 4 : (r <= 6 ? 6 : 8)); }

template <int RR, bool GEN>
static hipError_t launch_fcol_inst(const FColArgs& a, size_t lds, hipStream_t st) {
  static bool attr_set = false;   // the LDS limit is raised once, before any graph capture
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)k_fcol<RR, GEN>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)kFLdsMax);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL((k_fcol<RR, GEN>), dim3(a.q), dim3(kFThreads), lds, st, a);
  return hipSuccess;
}

hipError_t launch_fcol(const FColArgs& a, hipStream_t st) {
  const bool gen = !(a.n1 == kFN && a.n2 == kFN);
  const size_t lds = fcol_lds_bytes(a.rho, a.r, a.n, a.m, a.n1, a.n2);
  if (lds > kFLdsMax) return hipErrorInvalidValue;
  (void)hipGetLastError();
  hipError_t e;
#define FCOL_CALL(RR) e = gen ? launch_fcol_inst<RR, true>(a, lds, st) : launch_fcol_inst<RR, false>(a, lds, st)
  FR_SWITCH(fr_bucket(a.r), FCOL_CALL)
#undef FCOL_CALL
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch_fu_gen(const float2* U, int n, int r, int n1, int n2, const float2* tw, float2* FU,
                         hipStream_t st) {
  (void)hipGetLastError();
  const size_t lds = 8 * (size_t)(n + n1 + n2);
  hipLaunchKernelGGL(k_fu_gen, dim3(r), dim3(kFThreads), lds, st, U, n, r, n1, n2, tw, FU);
  return hipGetLastError();
}

hipError_t launch_ftwiddle_gen(float2* tw, int n1, int n2, hipStream_t st) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_ftwiddle_gen, dim3((n1 + n2 + 255) / 256), dim3(256), 0, st, tw, n1, n2);
  return hipGetLastError();
}

hipError_t launch_fu(const float2* U, int r, const float2* tw, float2* FU, hipStream_t st) {
  (void)hipGetLastError();
  const int blocks = kFN * r / 2;   // two 32-lane groups per 64-thread workgroup
  hipLaunchKernelGGL(k_fu<0>, dim3(blocks), dim3(64), 0, st, U, r, tw, FU);
  hipLaunchKernelGGL(k_fu<1>, dim3(blocks), dim3(64), 0, st, U, r, tw, FU);
  return hipGetLastError();
}

hipError_t launch_fltu(const float2* H, const float2* U, int n, int q, int r, float2* Tc, const int* skip,
                       hipStream_t st) {
  (void)hipGetLastError();
#define FLTU_CALL(RR) hipLaunchKernelGGL(k_fltu<RR>, dim3(q), dim3(kFThreads), 0, st, H, U, n, r, Tc, skip)
  FR_SWITCH(fr_bucket(r), FLTU_CALL)
#undef FLTU_CALL
  return hipGetLastError();
}

hipError_t launch_fqr(const FQRArgs& a, hipStream_t st) {
  (void)hipGetLastError();
#define FQR_CALL(RR) hipLaunchKernelGGL(k_fqr<RR>, dim3(1), dim3(kFThreads), 0, st, a)
  FR_SWITCH(fr_bucket(a.r), FQR_CALL)
#undef FQR_CALL
  return hipGetLastError();
}

hipError_t launch_fgrad_gd(const float2* H, const float2* B, const float2* U, int n, int q, int r, float2* Gsum,
                           double2* part, const int* skip, hipStream_t st) {
  (void)hipGetLastError();
#define FGD_CALL(RR) \
  hipLaunchKernelGGL(k_fgrad_gd<RR>, dim3((n + 255) / 256), dim3(kFThreads), 0, st, H, B, U, n, q, r, Gsum, part, skip)
  FR_SWITCH(fr_bucket(r), FGD_CALL)
#undef FGD_CALL
  return hipGetLastError();
}

hipError_t launch_fqr_gd(const FQRArgs& a, hipStream_t st) {
  const int nb = (a.n + 255) / 256;
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_fqr_a, dim3(1), dim3(256), 0, st, a);
#define FQB_CALL(RR) hipLaunchKernelGGL(k_fqr_b<RR>, dim3(nb), dim3(256), 0, st, a)
  FR_SWITCH(fr_bucket(a.r), FQB_CALL)
#undef FQB_CALL
  hipLaunchKernelGGL(k_fqr_c, dim3(1), dim3(256), 0, st, a);
#define FQD_CALL(RR) hipLaunchKernelGGL(k_fqr_d<RR>, dim3(nb), dim3(256), 0, st, a)
  FR_SWITCH(fr_bucket(a.r), FQD_CALL)
#undef FQD_CALL
  if (a.mode == QR_POWER) {
#define FQE_CALL(RR) hipLaunchKernelGGL(k_fqr_e<RR>, dim3(nb), dim3(256), 0, st, a)
    FR_SWITCH(fr_bucket(a.r), FQE_CALL)
#undef FQE_CALL
    hipLaunchKernelGGL(k_fqr_f, dim3(1), dim3(64), 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_ftwiddle(float2* tw, hipStream_t st) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_ftwiddle, dim3(1), dim3(128), 0, st, tw);
  return hipGetLastError();
}

hipError_t launch_fbasis(float2* U, int n, int r, hipStream_t st) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_fbasis, dim3(64), dim3(256), 0, st, U, n, r);
  return hipGetLastError();
}

}  // namespace altg
