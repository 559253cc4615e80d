// Column kernels of AltGDmin-LR+S for gfx950.
//
// One workgroup owns one column k and streams its A_k (m x n, column-major, row
// index fastest) with coalesced 16-byte loads.  Lane l of every wave holds rows
// 4*(l + 64c) .. +3 for c < NC, so a column j of A_k is read by one wave as NC
// contiguous 1 KiB segments.  The column kernel comes in workgroups of W = 4, 8
// or 16 waves: the wave count sets the order of the cross-wave sums (and so the
// bits), so it is a property of the problem; problems with few columns, whose
// workgroups cannot fill the chip, take the wider ones.
//
//  k_au  : P_k = A_k U (m x r), G_k = P_k^T P_k in FP64, G_k^{-1} by Gauss-Jordan in one wave
//          (the pieces of (A_k U)^dagger, eq. (bk_LS)).  The rows of U are
//          staged in LDS 64 at a time and read back as broadcasts; waves split
//          the columns j of A_k and their partial P_k are summed in LDS in a
//          fixed order.
//  k_col : tau iterations of IHT (Alg. 2) on column k, then the LS solve for
//          b_k (eq. (bk_LS)), the residual r_k = A_k(U b_k + s_k) - y_k and
//          h_k = A_k^T r_k for grad_U f (Sec. 2.1), or the back-projection
//          A_k^T (y_k - A_k s_k) of the initialisation (Sec. 2.3).
//
// One IHT iteration costs one gather of the rho support columns of A_k
// (A_k s_k), one streaming pass over A_k that forms g_j = A_j^T u and, for the
// columns j of the current support T, accumulates w = sum_{j in T} g_j A_j
// (the M g_T of the normalised step) while A_j is still in registers, and a
// block-wide exact top-rho selection.  In the GDmin loop the projector
// Pi_k v = v - P_k G_k^{-1} P_k^T v supplies z_k and M_k = Pi_k A_k of Sec. 2.2
// without forming M_k; since Pi_k is symmetric and idempotent,
// M_k^T (M_k s - z_k) = A_k^T Pi_k (A_k s - y_k).
#include <mutex>

#include "launch.h"

namespace altg {

// ---------------------------------------------------------------- helpers

template <int NC>
struct Lane {
  int ch[NC];   // 4-row chunk index held by this lane
  int chc[NC];  // the same, clamped to the last chunk that holds a row below m (always a legal address)
  int nv[NC];   // number of rows of that chunk below m (0 when the chunk lies beyond m)
  __device__ Lane(int lane, int m) {
    const int chmax = (m - 1) >> 2;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      ch[c] = lane + 64 * c;
      chc[c] = ch[c] < chmax ? ch[c] : chmax;
      const int v = m - 4 * ch[c];
      nv[c] = v < 0 ? 0 : (v > 4 ? 4 : v);
    }
  }
};

// Sum the per-wave partial vectors of all waves (fixed order 0..W-1); every
// wave ends with the same total.  Two barriers.
template <int NC, int W = kWaves>
__device__ __forceinline__ void xwave_sum(float4 (&v)[NC], const Lane<NC>& ln, float* wpart, int mq,
                                          int wave) {
#pragma unroll
  for (int c = 0; c < NC; ++c)
    if (ln.nv[c] > 0) *reinterpret_cast<float4*>(wpart + wave * mq + 4 * ln.ch[c]) = v[c];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    if (ln.nv[c] > 0) {
      float4 s = *reinterpret_cast<const float4*>(wpart + 4 * ln.ch[c]);
#pragma unroll
      for (int w = 1; w < W; ++w) s = add4(s, *reinterpret_cast<const float4*>(wpart + w * mq + 4 * ln.ch[c]));
      v[c] = s;
    }
  }
  __syncthreads();
}

template <int W = kWaves>
__device__ __forceinline__ double xwave_sum_scalar(double x, double* redd, int lane, int wave) {
  if (lane == 0) redd[wave] = x;
  __syncthreads();
  double s = redd[0];
#pragma unroll
  for (int w = 1; w < W; ++w) s += redd[w];
  __syncthreads();
  return s;
}

// out = sum_{t < cnt} coef[t] * A_k[:, idx[t]]  (idx, coef in LDS), all waves get the total.
// Each wave keeps up to 8 support columns in flight when A_k has at most 256 rows
// (4 otherwise, and in the Philox form, where they are generated, not loaded).
template <int FMT, int NC, int W = kWaves, int POL = POL_STREAM>
__device__ __forceinline__ void gather(const ALoader<FMT, POL>& L, const Lane<NC>& ln, const int* idx,
                                       const float* coef, int cnt, float4 (&out)[NC], float* wpart,
                                       int mq, int wave) {
  constexpr int GU = (NC == 1 && FMT != FMT_PHILOX) ? 8 : 4;   // support columns in flight per wave
  float4 acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int t0 = wave; t0 < cnt; t0 += W * GU) {
    // every load is issued before any is used: clamped, always legal addresses,
    // invalid rows and slots are zeroed afterwards
    typename ALoader<FMT, POL>::raw_t av[GU][NC];
    float cf[GU];
#pragma unroll
    for (int g = 0; g < GU; ++g) {
      const int t = t0 + g * W;
      const int j = idx[t < cnt ? t : t0];
      cf[g] = t < cnt ? coef[t] : 0.f;
#pragma unroll
      for (int c = 0; c < NC; ++c) av[g][c] = L.fetch(j, ln.chc[c]);
    }
#pragma unroll
    for (int g = 0; g < GU; ++g) {
      const bool ok = t0 + g * W < cnt;
#pragma unroll
      for (int c = 0; c < NC; ++c)
        acc[c] = axpy4(cf[g], mask_rows(ALoader<FMT, POL>::expand(av[g][c]), ok ? ln.nv[c] : 0), acc[c]);
    }
  }
  xwave_sum<NC, W>(acc, ln, wpart, mq, wave);
#pragma unroll
  for (int c = 0; c < NC; ++c) out[c] = acc[c];
}

// v <- v - P_k d with d = G_k^{-1} P_k^T v (FP64 products and solve).  The r
// reductions of P_k^T v are split across the waves and exchanged through cbuf
// (LDS, r doubles); every wave then applies the same d to its own copy of v.
// If bl != nullptr, lane i < r receives b_i = -d_i (the LS coefficients when
// v = A_k s_k - y_k).  One barrier; cbuf may be rewritten only after another.
template <int NC, int W = kWaves>
__device__ __forceinline__ void project(float4 (&v)[NC], const Lane<NC>& ln, const float* Pl,
                                        const double* Gi, int r, int lane, int wave, double* cbuf,
                                        double* bl) {
  for (int rr = wave; rr < r; rr += W) {
    double part = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (e < ln.nv[c]) part = fma((double)Pl[(4 * ln.ch[c] + e) * r + rr], (double)get4(v[c], e), part);
    const double tot = wave_sum_dpp(part);
    if (lane == 0) cbuf[rr] = tot;
  }
  __syncthreads();
  double myd = 0.0;
  if (lane < r)
    for (int jj = 0; jj < r; ++jj) myd = fma(Gi[lane * r + jj], cbuf[jj], myd);
  double acc[NC][4];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[c][e] = (double)get4(v[c], e);
  for (int rr = 0; rr < r; ++rr) {
    const double drr = readlane_f64(myd, __builtin_amdgcn_readfirstlane(rr));
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (e < ln.nv[c]) acc[c][e] = fma(-(double)Pl[(4 * ln.ch[c] + e) * r + rr], drr, acc[c][e]);
  }
#pragma unroll
  for (int c = 0; c < NC; ++c)
    v[c] = make_float4((float)acc[c][0], (float)acc[c][1], (float)acc[c][2], (float)acc[c][3]);
  if (bl) *bl = -myd;
}

template <int NC>
__device__ __forceinline__ double sumsq(const float4 (&v)[NC]) {
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    s = fma((double)v[c].x, (double)v[c].x, s);
    s = fma((double)v[c].y, (double)v[c].y, s);
    s = fma((double)v[c].z, (double)v[c].z, s);
    s = fma((double)v[c].w, (double)v[c].w, s);
  }
  return wave_sum_dpp(s);
}

// Totals over the 64 lanes of JU per-lane partial sums at once (JU = 1, 2, 4, 8):
// on return lane i < JU holds the total of x[i].  A butterfly: lanes l and
// l ^ 1, l ^ 2 (quad permutations), l ^ 4, l ^ 8 (row shifts restricted to the
// banks whose partner lies that way), then rows r ^ 1 and the two halves
// (permlane swaps).  Both lanes of a pair add the same two numbers, so a
// column's total has the same bits in every lane; with JU > 1 each lane
// carries, from the first step on, the column it ends with, so every JU gives
// the same bits.
template <int SH>
__device__ __forceinline__ float lanes_xor(float v) {   // value of lane l ^ SH (SH = 4 or 8)
  static_assert(SH == 4 || SH == 8, "row butterflies by 4 and 8 only");
  const int iv = __float_as_int(v);
  int t = __builtin_amdgcn_update_dpp(iv, iv, 0x100 + SH, 0xF, SH == 4 ? 0x5 : 0x3, false);   // row_shl
  t = __builtin_amdgcn_update_dpp(t, iv, 0x110 + SH, 0xF, SH == 4 ? 0xA : 0xC, false);       // row_shr
  return __int_as_float(t);
}

template <int JU>
__device__ __forceinline__ float col_totals(const float (&x)[JU], int lane) {
  static_assert(JU == 1 || JU == 2 || JU == 4 || JU == 8, "JU must be 1, 2, 4 or 8");
  auto qp = [](float v, int ctrl) -> float {
    return ctrl == 0xB1 ? __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false))
                        : __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
  };
  float v;
  if constexpr (JU == 1) {
    v = x[0] + qp(x[0], 0xB1);
    v = v + qp(v, 0x4E);
    v = v + lanes_xor<4>(v);
  } else if constexpr (JU == 2) {
    const bool odd = lane & 1;
    const float a = odd ? x[1] : x[0], b = odd ? x[0] : x[1];
    v = a + qp(b, 0xB1);                 // lane parity p: column p
    v = v + qp(v, 0x4E);
    v = v + lanes_xor<4>(v);
  } else if constexpr (JU == 4) {
    const bool odd = lane & 1, two = lane & 2;
    const float a = odd ? x[1] : x[0], b = odd ? x[0] : x[1];
    const float c = odd ? x[3] : x[2], d = odd ? x[2] : x[3];
    const float ab = a + qp(b, 0xB1);    // even lanes: column 0, odd: column 1
    const float cd = c + qp(d, 0xB1);    // even lanes: column 2, odd: column 3
    const float e = two ? cd : ab, f = two ? ab : cd;
    v = e + qp(f, 0x4E);                 // lane & 3: column
    v = v + lanes_xor<4>(v);
  } else {
    const bool odd = lane & 1, two = lane & 2, four = lane & 4;
    float h[4];
#pragma unroll
    for (int pq = 0; pq < 4; ++pq) {     // pairs (2pq, 2pq + 1): lane parity picks the column kept
      const float a = odd ? x[2 * pq + 1] : x[2 * pq], b = odd ? x[2 * pq] : x[2 * pq + 1];
      h[pq] = a + qp(b, 0xB1);
    }
    const float e0 = two ? h[1] : h[0], f0 = two ? h[0] : h[1];   // columns 0..3
    const float e1 = two ? h[3] : h[2], f1 = two ? h[2] : h[3];   // columns 4..7
    const float g0 = e0 + qp(f0, 0x4E), g1 = e1 + qp(f1, 0x4E);
    const float k = four ? g1 : g0, gv = four ? g0 : g1;
    v = k + lanes_xor<4>(gv);            // lane & 7: column
  }
  v = v + lanes_xor<8>(v);
  const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  v = __uint_as_float(p[0]) + __uint_as_float(p[1]);     // rows r and r ^ 1
  const auto h = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(h[0]) + __uint_as_float(h[1]);  // lanes l and l ^ 32
}

// Streaming pass over A_k: gl[j] = A_j^T u for every column j; for j in the
// support bitmap inT (if given) also wacc += gl[j] * A_j and gT2 += gl[j]^2.
// Wave w takes columns j = w, w + W, ...; groups of JU columns are loaded one
// group ahead of the one being reduced, and reduced together (col_totals).
// u must be zero on rows >= m (and A finite there): the products are then not
// masked.  The order in which a wave visits the columns and every column's
// reduction tree do not depend on JU, so every JU gives the same bits.
// default loads in flight (autotuned variants pass another JU); wider workgroups
// have more waves in flight and take fewer columns per group
// Default loads in flight of the column passes (columns per wave per group).
// The mixed BF16 form streams 2-byte elements, so its 8-wave workgroups keep
// twice the columns in flight at two row chunks (0.191 -> 0.180 ms at q = 125).
// The FP32 plane at two row chunks in 4-wave workgroups takes one column per
// group: with two it needs a 16-byte spill under its 128-register cap (0.982
// against 1.02 ms at n = q = 1000, m = 400, r = 10).
constexpr int default_ju(int nc, int w = kWaves, int fmt = FMT_F32) {
  return w >= 16 ? (nc == 1 ? 2 : 1)
                 : (w == 8 && nc == 2 && fmt == FMT_BF16MIX ? 4
                                                            : (nc == 1 ? 4 : (w == 4 && nc == 2 && fmt == FMT_F32 ? 1 : 2)));
}

template <int FMT, int NC, int JU, int W = kWaves, int POL = POL_STREAM>
__device__ __forceinline__ void fused_pass(const ALoader<FMT, POL>& L, const Lane<NC>& ln, const float4 (&u)[NC],
                                           int n, float* gl, const unsigned* inT, float4 (&wacc)[NC],
                                           double& gT2, int lane, int wave) {
  // the support bits of a group's columns j0, j0 + W, ... must lie in the two
  // bitmap words read per group
  static_assert((JU - 1) * W <= 32, "a group's support bits span more than two bitmap words");
  constexpr int step = W * JU;
  // loads are unconditional (column clamped to n-1, chunk clamped to a legal
  // one) so that a whole group is in flight at once; consume() drops them
  typedef typename ALoader<FMT, POL>::raw_t raw_t;
  auto load = [&](int j0, raw_t (&ar)[JU][NC]) {
#pragma unroll
    for (int ju = 0; ju < JU; ++ju) {
      const int j = j0 + ju * W;
      const int jc = j < n ? j : n - 1;
#pragma unroll
      for (int c = 0; c < NC; ++c) ar[ju][c] = L.fetch(jc, ln.chc[c]);
    }
  };
  auto consume = [&](int j0, const raw_t (&ar)[JU][NC]) {
    // support bits of columns j0 .. j0 + W (JU - 1) (at most 63 bits from
    // j0 - j0 % 32): two bitmap words, read before the reduction hides their latency
    unsigned long long tb = 0ull;
    if (inT) {
      const int wb = j0 >> 5;
      const unsigned w0 = inT[wb];
      const unsigned w1 = 32 * (wb + 1) < n ? inT[wb + 1] : 0u;
      tb = (((unsigned long long)w1 << 32) | w0) >> (j0 & 31);
    }
    float4 av[JU][NC];
    float d[JU];
#pragma unroll
    for (int ju = 0; ju < JU; ++ju) {
      av[ju][0] = ALoader<FMT, POL>::expand(ar[ju][0]);
      float s = dot4(av[ju][0], u[0]);
#pragma unroll
      for (int c = 1; c < NC; ++c) {
        av[ju][c] = ALoader<FMT, POL>::expand(ar[ju][c]);
        s += dot4(av[ju][c], u[c]);
      }
      d[ju] = s;
    }
    const float tot = col_totals<JU>(d, lane);
    const int jl = j0 + lane * W;
    if (lane < JU && jl < n) gl[jl] = tot;
    if (inT) {
#pragma unroll
      for (int ju = 0; ju < JU; ++ju) {
        const int j = j0 + ju * W;
        if (j < n && ((tb >> (W * ju)) & 1ull)) {
          const float dj = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(tot), ju));
#pragma unroll
          for (int c = 0; c < NC; ++c) wacc[c] = axpy4(dj, mask_rows(av[ju][c], ln.nv[c]), wacc[c]);
          gT2 = fma((double)dj, (double)dj, gT2);
        }
      }
    }
  };
  // Two groups in flight: the next group is loaded before the current one is
  // reduced.  The loop has one exit and loads without a condition (past the
  // end they re-read column n - 1 and are dropped): with a load under a branch,
  // or a second exit, the compiler waits for the newer loads as well before
  // the older group is reduced, and the two groups no longer overlap.
  const int groups = wave < n ? (n - wave + step - 1) / step : 0;
  raw_t a0[JU][NC], a1[JU][NC];
  load(wave, a0);
  int g = 0;
  for (; g + 1 < groups; g += 2) {
    const int j0 = wave + g * step;
    load(j0 + step, a1);
    consume(j0, a0);
    load(j0 + 2 * step, a0);
    consume(j0 + step, a1);
  }
  if (g < groups) consume(wave + g * step, a0);
}

// HardThreshold of Alg. 2 on vals[0..n) (LDS): the rho entries of largest
// |v|, lower index first on ties, written ascending to idx/val (LDS).
// Exact: the rho-th largest magnitude T is found by a radix select on the FP32
// magnitude bits (monotone in |v|), one byte per round from the top, with a
// 256-bin LDS histogram; ties at T are then resolved in index order by one
// wave.  hist: 256 + 8 ints of LDS.  Returns the number of NaNs (block-uniform).
template <int W = kWaves>
static __device__ int block_select(const float* vals, int n, int rho, int* idx, float* val, int* hist) {
  constexpr int T = 64 * W;   // threads of the workgroup
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
  if (rho <= 0) return 0;
  int* ctl = hist + 256;   // [0] digit, [1] rank left, [2] NaN count
  unsigned prefix = 0u, pmask = 0u;
  int remaining = rho;
  for (int d = 3; d >= 0; --d) {
    const int shift = 8 * d;
    for (int b = tid; b < 256; b += T) hist[b] = 0;
    if (d == 3 && tid == 0) ctl[2] = 0;
    __syncthreads();
    int nanc = 0;
    for (int j = tid; j < n; j += T) {
      const unsigned key = __float_as_uint(vals[j]) & 0x7fffffffu;
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
      int acc = incl - lsum;   // elements in bins above 4*lane+3
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
  }
  const unsigned thr = prefix;
  const int need_eq = remaining;
  if (wave == 0) {
    const unsigned long long lt = (1ull << lane) - 1ull;
    int base_eq = 0, base_pos = 0;
    for (int j0 = 0; j0 < n; j0 += 64) {
      const int j = j0 + lane;
      const bool valid = j < n;
      const float x = valid ? vals[j] : 0.f;
      const unsigned key = __float_as_uint(x) & 0x7fffffffu;
      const bool eq = valid && key == thr;
      const bool gtb = valid && key > thr;
      const unsigned long long meq = __ballot(eq);
      const int eq_rank = base_eq + __popcll(meq & lt);
      const bool sel = gtb || (eq && eq_rank < need_eq);
      const unsigned long long msel = __ballot(sel);
      const int pos = base_pos + __popcll(msel & lt);
      if (sel) {
        idx[pos] = j;
        val[pos] = x;
      }
      base_eq += __popcll(meq);
      base_pos += __popcll(msel);
    }
  }
  __syncthreads();
  return ctl[2];
}

// Whether HardThreshold of vals[0..n) keeps the support marked in the bitmap
// inT: it does when every magnitude on it is larger than every magnitude off it
// (with a tie or a NaN the full select decides).  slot: 2 W words of LDS;
// barriers inside, the last one after the slot is read.
template <int W = kWaves>
static __device__ bool block_support_kept(const float* vals, int n, const unsigned* inT, unsigned* slot) {
  const int lane = threadIdx.x & 63, wave = wave_id();
  unsigned kmin = 0xffffffffu, kmax = 0u;
  bool bad = false;
  for (int j = threadIdx.x; j < n; j += 64 * W) {
    const unsigned key = __float_as_uint(vals[j]) & 0x7fffffffu;
    bad |= key > 0x7f800000u;
    if ((inT[j >> 5] >> (j & 31)) & 1u)
      kmin = min(kmin, key);
    else
      kmax = max(kmax, key);
  }
  if (bad) kmin = 0u;   // fails the test below for the whole block
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    kmin = min(kmin, __shfl_xor(kmin, o));
    kmax = max(kmax, __shfl_xor(kmax, o));
  }
  if (lane == 0) {
    slot[2 * wave] = kmin;
    slot[2 * wave + 1] = kmax;
  }
  __syncthreads();
  unsigned mn = 0xffffffffu, mx = 0u;
#pragma unroll
  for (int w = 0; w < W; ++w) {
    mn = min(mn, slot[2 * w]);
    mx = max(mx, slot[2 * w + 1]);
  }
  __syncthreads();
  return mn > mx;
}

// ---------------------------------------------------------------- k_col

template <int FMT, int NC, int JU, int W, int POL = POL_STREAM>
__device__ __forceinline__ void col_body(const ColArgs& a, int k, unsigned char* smem) {
  constexpr int kT = 64 * W;   // threads of the workgroup
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
  const int n = a.n, m = a.m, r = a.r, rho = a.rho;
  const ColLayout lay(n, m, r, rho, a.project, FMT == FMT_PHILOX, W);
  double* Gi = reinterpret_cast<double*>(smem + lay.ginv);
  // P_k in LDS when it fits, else read from the workspace copy in global memory
  float* Pl = lay.p_in_lds ? reinterpret_cast<float*>(smem + lay.P) : const_cast<float*>(a.P + (long long)k * m * r);
  float* wpart = reinterpret_cast<float*>(smem + lay.wpart);
  float* gl = reinterpret_cast<float*>(smem + lay.g);
  float* sd = reinterpret_cast<float*>(smem + lay.sd);
  unsigned* inT = reinterpret_cast<unsigned*>(smem + lay.inT);
  int* Ti = reinterpret_cast<int*>(smem + lay.Ti);
  float* Tv = reinterpret_cast<float*>(smem + lay.Tv);
  double* redd = reinterpret_cast<double*>(smem + lay.red);
  int* hist = reinterpret_cast<int*>(smem + lay.hist);
  double* cbuf = reinterpret_cast<double*>(smem + lay.cbuf);
  const int mq = lay.mq;
  const int nwords = (n + 31) >> 5;

  constexpr int GF = gather_fmt(FMT), SF = stream_fmt(FMT);
  ALoader<GF, POL> L(a, k);    // A_k s_k: exact
  ALoader<SF, POL> Ls(a, k);   // A_k^T u and the step length: the streaming view
  if constexpr (FMT == FMT_PHILOX) {
    float* tab = reinterpret_cast<float*>(smem + lay.tab);
    for (int t = tid; t < kNormalTable; t += kT) tab[t] = a.table[t];
    L.tab = tab;   // read only after the barrier that ends the LDS set-up below
    Ls.tab = tab;
  }
  const Lane<NC> ln(lane, m);

  float4 yv[NC];
  {
    const float* yk = a.Y + (long long)k * a.ldy;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      float t[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) t[e] = (e < ln.nv[c]) ? yk[4 * ln.ch[c] + e] : 0.f;
      yv[c] = make_float4(t[0], t[1], t[2], t[3]);
    }
  }

  for (int j = tid; j < n; j += kT) sd[j] = 0.f;
  for (int w = tid; w < nwords; w += kT) inT[w] = 0u;
  if (a.project) {
    const float* Pk = a.P + (long long)k * m * r;
    if (lay.p_in_lds)
      for (int t = tid; t < m * r; t += kT) Pl[t] = Pk[t];
    const double* Gk = a.Ginv + (long long)k * r * r;
    for (int t = tid; t < r * r; t += kT) Gi[t] = Gk[t];
  }
  __syncthreads();
  // A start support must hold rho distinct in-range indices in ascending order
  // (every support this library writes does).  Any other start is invalid caller
  // state: the column is flagged (bit 2) and starts from s = 0 with no support.
  int nz = 0, bad = 0;
  if (a.has_support) {
    for (int t = tid; t < rho; t += kT) {
      const int j = a.Tidx[(long long)k * rho + t];
      const int jp = t > 0 ? a.Tidx[(long long)k * rho + t - 1] : -1;
      const float v = a.Tval[(long long)k * rho + t];
      bad |= (j < 0 || j >= n || j <= jp) ? 1 : 0;
      Ti[t] = j;
      Tv[t] = v;
      nz |= v != 0.f;
    }
  }
  // one reduction tells both whether some start value is nonzero and whether the
  // start is invalid (weights 1 and 64 per wave, at most 16 waves)
  const double vote = xwave_sum_scalar<W>((__ballot(nz != 0) != 0ull ? 1.0 : 0.0) + (__ballot(bad != 0) != 0ull ? 64.0 : 0.0),
                                       redd, lane, wave);
  const bool invalid = vote >= 64.0;
  if (a.has_support && !invalid) {
    for (int t = tid; t < rho; t += kT) {   // each thread reads back only its own entries
      const int j = Ti[t];
      sd[j] = Tv[t];
      atomicOr(&inT[j >> 5], 1u << (j & 31));
    }
  } else {
    for (int t = tid; t < rho; t += kT) {   // s = 0 on the support 0 .. rho - 1 (kept if tau = 0)
      Ti[t] = t;
      Tv[t] = 0.f;
    }
    if (invalid && tid == 0 && a.flags) atomicOr(&a.flags[k], 4);
  }
  // a start whose values are all zero (an initialisation with tau0 = 0) is s = 0
  // with no support yet: T then comes from HardThreshold(g), as for no start
  bool hasT = !invalid && vote > 0.0;
  int nan_seen = 0;

  for (int it = 0; it < a.tau; ++it) {
    // u = Pi (A_k s - y_k)   (Pi = I in the initialisation)
    float4 v[NC];
    gather<GF, NC, W>(L, ln, Ti, Tv, hasT ? rho : 0, v, wpart, mq, wave);
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = sub4(v[c], yv[c]);
    if (a.project) project<NC, W>(v, ln, Pl, Gi, r, lane, wave, cbuf, nullptr);

    // g = A_k^T u; w = A_k g_T on the current support
    float4 w[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) w[c] = make_float4(0.f, 0.f, 0.f, 0.f);
    double gT2 = 0.0;
    fused_pass<SF, NC, JU, W>(Ls, ln, v, n, gl, hasT ? inT : nullptr, w, gT2, lane, wave);
    __syncthreads();
    if (hasT) {
      xwave_sum<NC, W>(w, ln, wpart, mq, wave);
      gT2 = xwave_sum_scalar<W>(gT2, redd, lane, wave);
    } else {
      // no support yet (s = 0): restrict to the support of HardThreshold(g, rho)
      nan_seen += block_select<W>(gl, n, rho, Ti, Tv, hist);
      gather<SF, NC, W>(Ls, ln, Ti, Tv, rho, w, wpart, mq, wave);
      gT2 = 0.0;
      for (int t = 0; t < rho; ++t) gT2 = fma((double)Tv[t], (double)Tv[t], gT2);
    }
    if (a.project) project<NC, W>(w, ln, Pl, Gi, r, lane, wave, cbuf, nullptr);
    const double ww = sumsq<NC>(w);
    const double mu = (ww > 0.0 && isfinite(ww) && isfinite(gT2)) ? gT2 / ww : 0.0;
    const bool last = (it == a.tau - 1);
    if (last && a.G_out)
      for (int j = tid; j < n; j += kT) a.G_out[(long long)k * n + j] = gl[j];
    if (last && a.mu_out && tid == 0) a.mu_out[k] = mu;
    // s - mu g, then HardThreshold
    for (int j = tid; j < n; j += kT) gl[j] = (float)fma(-mu, (double)gl[j], (double)sd[j]);
    __syncthreads();
    if (hasT && block_support_kept<W>(gl, n, inT, reinterpret_cast<unsigned*>(hist))) {
      // most steps keep T: Ti (ascending) and inT stand, s takes the new values on T
      for (int t = tid; t < rho; t += kT) {
        const int j = Ti[t];
        Tv[t] = gl[j];
        sd[j] = gl[j];
      }
    } else {
      nan_seen += block_select<W>(gl, n, rho, Ti, Tv, hist);
      for (int j = tid; j < n; j += kT) sd[j] = 0.f;
      for (int wd = tid; wd < nwords; wd += kT) inT[wd] = 0u;
      __syncthreads();
      for (int t = tid; t < rho; t += kT) {
        const int j = Ti[t];
        sd[j] = Tv[t];
        atomicOr(&inT[j >> 5], 1u << (j & 31));
      }
    }
    __syncthreads();
    hasT = true;
  }

  if (a.tail != TAIL_NONE) {
    float4 v[NC];
    gather<GF, NC, W>(L, ln, Ti, Tv, hasT ? rho : 0, v, wpart, mq, wave);
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = sub4(v[c], yv[c]);   // A_k s_k - y_k
    if (a.tail == TAIL_LSGRAD) {
      // b_k = G^{-1} P^T (y - A s); r_k = P b + A s - y = Pi (A s - y)
      double b = 0.0;
      project<NC, W>(v, ln, Pl, Gi, r, lane, wave, cbuf, &b);
      const double rr = sumsq<NC>(v);
      if (wave == 0 && lane < r) a.Bt[(long long)k * r + lane] = (float)b;
      if (tid == 0 && a.rr) a.rr[k] = rr;
    } else {
#pragma unroll
      for (int c = 0; c < NC; ++c) v[c] = make_float4(-v[c].x, -v[c].y, -v[c].z, -v[c].w);   // y - A s
      const double yy = sumsq<NC>(yv);
      if (tid == 0 && a.rr) a.rr[k] = yy;
    }
    float4 w[NC];
    double dummy = 0.0;
    fused_pass<SF, NC, JU, W>(Ls, ln, v, n, gl, nullptr, w, dummy, lane, wave);
    __syncthreads();
    for (int j = tid; j < n; j += kT) a.H[(long long)k * n + j] = gl[j];
  }

  for (int t = tid; t < rho; t += kT) {
    a.Tidx[(long long)k * rho + t] = Ti[t];
    a.Tval[(long long)k * rho + t] = Tv[t];
  }
  if (tid == 0 && nan_seen > 0 && a.flags) a.flags[k] |= 1;
}

// Minimum waves per SIMD asked of the register allocator (4 waves: at most 128
// VGPRs): as many as the column pass fits without spilling.  The loads in
// flight grow with NC and JU; the two BF16 planes and the Philox rounds need
// more registers than one FP32 or hi plane.
constexpr int col_min_waves(int fmt, int nc, int ju) {
  if (ju == 8) return nc == 1 ? 2 : 1;
  if (fmt == FMT_PHILOX) return nc <= 2 ? 2 : 1;
  if (nc == 1) return 4;
  if (nc == 2) return ju == 1 ? 4 : (ju == 2 ? (fmt == FMT_BF16X2 ? 3 : 4) : (fmt == FMT_BF16X2 ? 2 : 3));
  return ju == 4 ? 1 : 2;
}

// Wider workgroups: W / 4 waves per SIMD at least (the workgroup must fit).
constexpr int col_min_waves_w(int fmt, int nc, int ju, int w) {
  return col_min_waves(fmt, nc, ju) > w / 4 ? col_min_waves(fmt, nc, ju) : w / 4;
}

template <int FMT, int NC, int JU = default_ju(NC, kWaves, FMT), int W = kWaves, int POL = POL_STREAM>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(col_min_waves_w(FMT, NC, JU, W), 8))) void k_col(ColArgs a) {
  if (a.gate && *a.gate != a.gate_want) return;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  col_body<FMT, NC, JU, W, POL>(a, blockIdx.x, smem);
}

// Several problems in one launch: block b works on column map[b].y of problem map[b].x.
template <int FMT, int NC, int W = kWaves, int POL = POL_STREAM>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(col_min_waves_w(FMT, NC, default_ju(NC, W, FMT), W), 8))) void k_col_grp(
    const ColArgs* tab, const int2* map) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int2 mp = map[blockIdx.x];
  const ColArgs a = tab[mp.x];
  if (a.gate && *a.gate != a.gate_want) return;
  col_body<FMT, NC, default_ju(NC, W, FMT), W, POL>(a, mp.y, smem);
}

// ---------------------------------------------------------------- k_au

// One column k of A_k U by a workgroup of W waves.  Waves split the 256-row
// chunks of A_k first and the columns j second: with nch = ceil(m / 256) chunks,
// wave w takes chunk w / js and columns j = w % js, w % js + js, ... where
// js = max(1, W / nch); each lane holds 4 rows x R accumulators.  Partial P_k of
// the waves sharing a chunk are added in a fixed order (in LDS when P_k fits,
// else in global memory), so W sets the summation order: it is a property of the
// problem (8 waves up to 512 columns), the same in a solo and a batched launch.
// The Gram and the inverse use the first 4 waves whatever W.
template <int FMT, int R, int AUD, int POL = POL_STREAM, int W = kWaves>
__device__ __forceinline__ void au_body(const AUArgs& a, int k, unsigned char* smem) {
  constexpr int kT = 64 * W;
  const int tid = threadIdx.x, lane = tid & 63, wave = wave_id();
  const int n = a.n, m = a.m, r = a.r;
  const AULayout lay(m, r, FMT == FMT_PHILOX, W);
  float* Pk = a.P + (long long)k * m * r;
  float* Pp = lay.p_in_lds ? reinterpret_cast<float*>(smem + lay.P) : Pk;
  double* gpart = reinterpret_cast<double*>(smem + lay.gpart);
  double* Gl = reinterpret_cast<double*>(smem + lay.G);
  double* Wl = reinterpret_cast<double*>(smem + lay.W);
  double* Gil = reinterpret_cast<double*>(smem + lay.Gi);
  ALoader<FMT, POL> L(a, k);
  if constexpr (FMT == FMT_PHILOX) {
    float* tab = reinterpret_cast<float*>(smem + lay.tab);
    for (int t = tid; t < kNormalTable; t += kT) tab[t] = a.table[t];
    L.tab = tab;
    __syncthreads();
  }
  const int nch = (m + 255) >> 8;
  const int js = W / nch > 1 ? W / nch : 1;
  const int cs = wave / js, jw = wave % js;
  const bool active = cs < nch;
  const int ch = lane + 64 * cs;
  const int chmax = (m - 1) >> 2;
  const int chc = ch < chmax ? ch : chmax;
  const int nvr = m - 4 * ch;
  const int nv = nvr < 0 ? 0 : (nvr > 4 ? 4 : nvr);

  float acc[4][R];
#pragma unroll
  for (int e = 0; e < 4; ++e)
#pragma unroll
    for (int rr = 0; rr < R; ++rr) acc[e][rr] = 0.f;

  // software pipeline, AUD columns deep: the A_k loads of the next AUD columns
  // of this wave are in flight while the 4R FMAs of the current column are
  // issued.  The rows of U this wave needs are staged 64 at a time in its own
  // LDS slice (lane t loads the row of the wave's t-th next column) and read back
  // as broadcast 16-byte LDS loads, so the FMAs take plain register operands.
  constexpr int RP = (R + 3) / 4 * 4;
  float* Uw = reinterpret_cast<float*>(smem + lay.P) + wave * 64 * RP;   // shares the P region
  const float* U = a.U;
  typedef typename ALoader<FMT, POL>::raw_t raw_t;
  auto fetch = [&](int j, raw_t& a4) {
    const int jc = j < n ? j : n - 1;   // clamped: always a legal address
    a4 = L.fetch(jc, chc);
  };
  float un[RP];
  auto load_rows = [&](int t0) {        // rows of columns jw + js (t0 + t), t = lane
    const int jrow = jw + js * (t0 + lane);
    const int jr = jrow < n ? jrow : n - 1;
    const float* row = U + (long long)jr * r;
    // one address register for the row and fixed offsets; r is uniform over the
    // wave (a batched launch's R is its largest rank, so r may be far below R),
    // and entries at or beyond r are never read
#pragma unroll
    for (int rr = 0; rr < RP; ++rr) un[rr] = rr < r ? row[rr] : 0.f;
  };
  auto store_rows = [&](int t0) {
    const int jrow = jw + js * (t0 + lane);
#pragma unroll
    for (int rr = 0; rr < RP; ++rr) Uw[lane * RP + rr] = (jrow < n && rr < r) ? un[rr] : 0.f;
  };
  auto fma_col = [&](float4 a4, int t) {  // t: slot of the column in the staged block
    float u[RP];
#pragma unroll
    for (int q4 = 0; q4 < RP / 4; ++q4) {
      const float4 w4 = *reinterpret_cast<const float4*>(Uw + t * RP + 4 * q4);
      u[4 * q4] = w4.x; u[4 * q4 + 1] = w4.y; u[4 * q4 + 2] = w4.z; u[4 * q4 + 3] = w4.w;
    }
    a4 = mask_rows(a4, nv);
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int rr = 0; rr < R; ++rr) acc[e][rr] = fmaf(get4(a4, e), u[rr], acc[e][rr]);
  };
  auto stage = [&](int t) {             // wave-local: the LDS accesses of one wave complete in order
    __builtin_amdgcn_wave_barrier();
    load_rows(t);
    store_rows(t);
    __builtin_amdgcn_wave_barrier();
  };
  if (active) {
    // t-th column of this wave: j = jw + t js.  AUD + 1 slots in rotation: the
    // slot refilled at step t is the one consumed at step t - 1, so that no
    // register holding a load in flight is ever copied (a copy would wait for
    // it).  Refills in the main loop are not under a condition (past the end
    // they re-read column n - 1 and are dropped).
    constexpr int NB = AUD + 1;
    const int cols = jw < n ? (n - jw + js - 1) / js : 0;
    raw_t buf[NB];
#pragma unroll
    for (int d = 0; d < AUD; ++d) fetch(jw + d * js, buf[d]);
    int t = 0;
    for (; t + NB <= cols; t += NB) {
#pragma unroll
      for (int d = 0; d < NB; ++d) {
        const int tt = t + d;
        if ((tt & 63) == 0) stage(tt);
        fetch(jw + (tt + AUD) * js, buf[(d + AUD) % NB]);
        fma_col(ALoader<FMT, POL>::expand(buf[d]), tt & 63);
      }
    }
#pragma unroll
    for (int d = 0; d < NB; ++d) {
      const int tt = t + d;
      if (tt < cols) {
        if ((tt & 63) == 0) stage(tt);
        if (d + AUD < NB) fetch(jw + (tt + AUD) * js, buf[d + AUD]);
        fma_col(ALoader<FMT, POL>::expand(buf[d]), tt & 63);
      }
    }
  }
  __syncthreads();   // the staged rows of U share LDS with P

  // partial P of the waves sharing a chunk, added in column-split order.  In
  // LDS, P is column-major with row stride mp (lane-contiguous 16-byte stores);
  // in global memory it is row-major m x r.
  const int mp = lay.mp;
  for (int s = 0; s < js; ++s) {
    if (active && jw == s && nv > 0) {
      if (lay.p_in_lds) {
#pragma unroll
        for (int rr = 0; rr < R; ++rr)
          if (rr < r) {
            float4* dst = reinterpret_cast<float4*>(Pp + rr * mp + 4 * ch);
            float4 v = make_float4(acc[0][rr], acc[1][rr], acc[2][rr], acc[3][rr]);
            if (s > 0) {
              const float4 o = *dst;
              v = make_float4(o.x + v.x, o.y + v.y, o.z + v.z, o.w + v.w);
            }
            *dst = v;
          }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (e < nv) {
            const int i = 4 * ch + e;
#pragma unroll
            for (int rr = 0; rr < R; ++rr)
              if (rr < r) Pp[i * r + rr] = (s == 0) ? acc[e][rr] : Pp[i * r + rr] + acc[e][rr];
          }
      }
    }
    __syncthreads();
  }
  if (lay.p_in_lds)
    for (int t = tid; t < m * r; t += kT) {
      const int i = t / r, rr = t - i * r;
      Pk[t] = Pp[rr * mp + i];
    }
  auto pval = [&](int i, int c) -> double {
    return (double)(lay.p_in_lds ? Pp[c * mp + i] : Pp[i * r + c]);
  };

  // G = P^T P in FP64.  Thread (blk, part) accumulates the 2 x 2 block
  // (2ba .. 2ba+1) x (2bb .. 2bb+1), ba <= bb, over rows part, part + parts, ...;
  // the parts are then added in order.  Columns beyond r read as zero.
  const int RB = (r + 1) >> 1;
  const int nb = RB * (RB + 1) / 2;
  const int parts = kThreads / nb;
  if (tid < kThreads) {
    const int blk = tid % nb, part = tid / nb;
    int ba = 0, base = 0;
    while (blk >= base + (RB - ba)) { base += RB - ba; ++ba; }
    const int bb = ba + (blk - base);
    const int c0 = 2 * ba, c1 = 2 * ba + 1, d0 = 2 * bb, d1 = 2 * bb + 1;
    double g00 = 0.0, g01 = 0.0, g10 = 0.0, g11 = 0.0;
    if (part < parts)
      for (int i = part; i < m; i += parts) {
        const double x0 = pval(i, c0), x1 = c1 < r ? pval(i, c1) : 0.0;
        const double y0 = pval(i, d0), y1 = d1 < r ? pval(i, d1) : 0.0;
        g00 = fma(x0, y0, g00); g01 = fma(x0, y1, g01);
        g10 = fma(x1, y0, g10); g11 = fma(x1, y1, g11);
      }
    gpart[4 * tid] = g00; gpart[4 * tid + 1] = g01; gpart[4 * tid + 2] = g10; gpart[4 * tid + 3] = g11;
  }
  __syncthreads();
  if (tid < 4 * nb) {
    const int blk = tid >> 2, w = tid & 3;
    int ba = 0, base = 0;
    while (blk >= base + (RB - ba)) { base += RB - ba; ++ba; }
    const int bb = ba + (blk - base);
    const int ra = 2 * ba + (w >> 1), rb = 2 * bb + (w & 1);
    double t = 0.0;
    for (int p = 0; p < parts; ++p) t += gpart[4 * (p * nb + blk) + w];
    if (ra < r && rb < r) {
      Gl[ra * r + rb] = t;
      Gl[rb * r + ra] = t;
    }
  }
  __syncthreads();
  // G^{-1} by wave 0 (tid 0, which raises the flag, is in it)
  if (wave == 0) {
    const bool spd = wave_spd_inverse(Gl, Wl, Gil, r);
    if (!spd && tid == 0 && a.flags) a.flags[k] |= 2;
  }
  __syncthreads();
  double* Gk = a.Ginv + (long long)k * r * r;
  for (int t = tid; t < r * r; t += kT) Gk[t] = Gil[t];
}

// A_k loads of the next AUD columns in flight per wave (autotuned variants differ).
// The r accumulators per row compete with the loads for registers: at R = 14 one
// column in flight keeps four waves per SIMD (0.311 against 0.377 ms with two at
// n = q = 1000, m = 400, FP32), at R = 16 four in flight hide the latency best
// (0.382 against 0.409 ms); two elsewhere.  The BF16 hi + lo planes take two loads
// per group of elements and one group in flight is best up to R = 14 (0.308
// against 0.319 ms at r = 10, 0.273 against 0.292 at r = 4), three at R = 16
// (0.423 against 0.457 with two).
constexpr int default_aud(int R, int FMT = FMT_F32) {
  if (FMT == FMT_BF16X2) return R == 16 ? 3 : 1;
  return R == 14 ? 1 : (R == 16 ? 4 : 2);
}

// Launches of at most kDeepAuColumns columns (the MI355X's 256 CUs: one column
// workgroup per CU, one wave per SIMD) take the deep variants: three loads in
// flight at every rank, four at R <= 4 (cached loads at q = 125, n = 1000,
// m = 400, FP32: 0.091 against 0.105 ms at r = 10, 0.121 against 0.149 at
// r = 14, 0.068 against 0.081 at r = 4).  With several workgroups per CU the
// default depths keep more waves resident.  The depth only moves loads: the
// arithmetic, and so every bit, is the same.
constexpr int deep_aud(int R, int = FMT_F32) { return R <= 4 ? 4 : 3; }
constexpr int kDeepAuColumns = 256;

template <int FMT, int R, int AUD = default_aud(R, FMT), int POL = POL_STREAM, int W = kWaves>
__global__ __launch_bounds__(64 * W) void k_au(AUArgs a) {
  if (a.gate && *a.gate != a.gate_want) return;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  au_body<FMT, R, AUD, POL, W>(a, blockIdx.x, smem);
}

// Several problems in one launch: block b works on column map[b].y of problem map[b].x.
template <int FMT, int R, int POL = POL_STREAM, int AUD = default_aud(R, FMT), int W = kWaves>
__global__ __launch_bounds__(64 * W) void k_au_grp(const AUArgs* tab, const int2* map) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  const int2 mp = map[blockIdx.x];
  const AUArgs a = tab[mp.x];
  if (a.gate && *a.gate != a.gate_want) return;
  au_body<FMT, R, AUD, POL, W>(a, mp.y, smem);
}

#if !defined(ALTG_PART) || ALTG_PART == 1
// HardThreshold of one vector per workgroup (the step-level select entry point).
__global__ __launch_bounds__(kThreads) void k_select(const float* V, int n, long long ldv, int rho, int* idx,
                                                     float* val, int* flags) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  float* vl = reinterpret_cast<float*>(smem);
  int* Ti = reinterpret_cast<int*>(smem + align16(4 * (size_t)n));
  float* Tv = reinterpret_cast<float*>(smem + align16(4 * (size_t)n) + align16(4 * (size_t)rho));
  int* hist = reinterpret_cast<int*>(smem + align16(4 * (size_t)n) + 2 * align16(4 * (size_t)rho));
  const int c = blockIdx.x, tid = threadIdx.x;
  for (int j = tid; j < n; j += kThreads) vl[j] = V[(long long)c * ldv + j];
  __syncthreads();
  const int nan = block_select(vl, n, rho, Ti, Tv, hist);
  for (int t = tid; t < rho; t += kThreads) {
    idx[(long long)c * rho + t] = Ti[t];
    val[(long long)c * rho + t] = Tv[t];
  }
  if (tid == 0 && flags) flags[c] = nan > 0 ? 1 : 0;
}

size_t select_lds_bytes(int n, int rho) { return align16(4 * (size_t)n) + 2 * align16(4 * (size_t)rho) + 4 * (256 + 8); }

hipError_t launch_select(const float* V, int n, int count, long long ldv, int rho, int* idx, float* val,
                         int* flags, hipStream_t st) {
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  hipLaunchKernelGGL(k_select, dim3(count), dim3(kThreads), select_lds_bytes(n, rho), st, V, n, ldv, rho, idx, val,
                     flags);
  return hipGetLastError();
}

// ---------------------------------------------------------------- dispatch tables

typedef void (*col_fn)(ColArgs);
typedef void (*au_fn)(AUArgs);
typedef void (*colg_fn)(const ColArgs*, const int2*);
typedef void (*aug_fn)(const AUArgs*, const int2*);

#define COL_ROW(F) {k_col<F, 1>, k_col<F, 2>, k_col<F, 3>, k_col<F, 4>}
static const col_fn kColTable[5][kNCMax] = {COL_ROW(FMT_F32), COL_ROW(FMT_BF16X2), COL_ROW(FMT_BF16HI),
                                            COL_ROW(FMT_PHILOX), COL_ROW(FMT_BF16MIX)};
#define COLG_ROW(F) {k_col_grp<F, 1>, k_col_grp<F, 2>, k_col_grp<F, 3>, k_col_grp<F, 4>}
static const colg_fn kColGrpTable[5][kNCMax] = {COLG_ROW(FMT_F32), COLG_ROW(FMT_BF16X2), COLG_ROW(FMT_BF16HI),
                                                COLG_ROW(FMT_PHILOX), COLG_ROW(FMT_BF16MIX)};
#define AU_ROW(F) {k_au<F, 2>, k_au<F, 4>, k_au<F, 6>, k_au<F, 8>, k_au<F, 10>, k_au<F, 12>, k_au<F, 14>, k_au<F, 16>}
static const au_fn kAUTable[4][kRMax / 2] = {AU_ROW(FMT_F32), AU_ROW(FMT_BF16X2), AU_ROW(FMT_BF16HI), AU_ROW(FMT_PHILOX)};
#define AUG_ROW(F) {k_au_grp<F, 2>, k_au_grp<F, 4>, k_au_grp<F, 6>, k_au_grp<F, 8>, k_au_grp<F, 10>, k_au_grp<F, 12>, \
                    k_au_grp<F, 14>, k_au_grp<F, 16>}
static const aug_fn kAUGrpTable[4][kRMax / 2] = {AUG_ROW(FMT_F32), AUG_ROW(FMT_BF16X2), AUG_ROW(FMT_BF16HI),
                                                 AUG_ROW(FMT_PHILOX)};
// the deep depths of the plane formats, for launches of at most kDeepAuColumns columns
// (the Philox form regenerates A and is bound by its ALU work: it keeps the defaults)
#define AUD_ROW(F) {k_au<F, 2, deep_aud(2)>, k_au<F, 4, deep_aud(4)>, k_au<F, 6, deep_aud(6)>, k_au<F, 8, deep_aud(8)>, \
                    k_au<F, 10, deep_aud(10)>, k_au<F, 12, deep_aud(12)>, k_au<F, 14, deep_aud(14)>,              \
                    k_au<F, 16, deep_aud(16)>}
static const au_fn kAUDeep[3][kRMax / 2] = {AUD_ROW(FMT_F32), AUD_ROW(FMT_BF16X2), AUD_ROW(FMT_BF16HI)};
#define AUGD_ROW(F) {k_au_grp<F, 2, POL_STREAM, deep_aud(2)>, k_au_grp<F, 4, POL_STREAM, deep_aud(4)>,   \
                     k_au_grp<F, 6, POL_STREAM, deep_aud(6)>, k_au_grp<F, 8, POL_STREAM, deep_aud(8)>,   \
                     k_au_grp<F, 10, POL_STREAM, deep_aud(10)>, k_au_grp<F, 12, POL_STREAM, deep_aud(12)>, \
                     k_au_grp<F, 14, POL_STREAM, deep_aud(14)>, k_au_grp<F, 16, POL_STREAM, deep_aud(16)>}
static const aug_fn kAUGrpDeep[3][kRMax / 2] = {AUGD_ROW(FMT_F32), AUGD_ROW(FMT_BF16X2), AUGD_ROW(FMT_BF16HI)};
// 8-wave workgroups (problems of at most 512 columns, with the deep depths; every
// format, so that the width, and with it the bits, do not depend on how A is held)
#define AU8_ROW(F) {k_au<F, 2, deep_aud(2), POL_STREAM, 8>, k_au<F, 4, deep_aud(4), POL_STREAM, 8>,     \
                    k_au<F, 6, deep_aud(6), POL_STREAM, 8>, k_au<F, 8, deep_aud(8), POL_STREAM, 8>,     \
                    k_au<F, 10, deep_aud(10), POL_STREAM, 8>, k_au<F, 12, deep_aud(12), POL_STREAM, 8>, \
                    k_au<F, 14, deep_aud(14), POL_STREAM, 8>, k_au<F, 16, deep_aud(16), POL_STREAM, 8>}
static const au_fn kAU8[4][kRMax / 2] = {AU8_ROW(FMT_F32), AU8_ROW(FMT_BF16X2), AU8_ROW(FMT_BF16HI), AU8_ROW(FMT_PHILOX)};
#define AUG8_ROW(F) {k_au_grp<F, 2, POL_STREAM, deep_aud(2), 8>, k_au_grp<F, 4, POL_STREAM, deep_aud(4), 8>,     \
                     k_au_grp<F, 6, POL_STREAM, deep_aud(6), 8>, k_au_grp<F, 8, POL_STREAM, deep_aud(8), 8>,     \
                     k_au_grp<F, 10, POL_STREAM, deep_aud(10), 8>, k_au_grp<F, 12, POL_STREAM, deep_aud(12), 8>, \
                     k_au_grp<F, 14, POL_STREAM, deep_aud(14), 8>, k_au_grp<F, 16, POL_STREAM, deep_aud(16), 8>}
static const aug_fn kAUGrp8[4][kRMax / 2] = {AUG8_ROW(FMT_F32), AUG8_ROW(FMT_BF16X2), AUG8_ROW(FMT_BF16HI),
                                             AUG8_ROW(FMT_PHILOX)};

// the workgroup width of the A_k U kernels for a launch: 8 waves when asked for, else 4
static inline int au_width(int waves) { return waves == 8 ? 8 : kWaves; }

bool au_supported(int m, int r) { return m >= 1 && m <= 256 * kNCMax && r >= 1 && r <= kRMax; }

hipError_t launch_col(int fmt, const ColArgs& a, hipStream_t st, int pol) {
  if (fmt < FMT_F32 || fmt > FMT_BF16MIX) return hipErrorInvalidValue;
  if (pol == POL_CACHED) {   // the cached-load instantiation when one is built, else the streaming one
    const hipError_t e = launch_col_cached(fmt, a, st);
    if (e != hipErrorNotSupported) return e;
  }
  if (a.waves == 8 || a.waves == 16) return launch_col_wide(fmt, a, st);
  if (a.waves != 0 && a.waves != kWaves) return hipErrorInvalidValue;
  const int nc = (a.m + 255) / 256;
  const ColLayout lay(a.n, a.m, a.r, a.rho, a.project, fmt == FMT_PHILOX);
  if (lay.total > kColLdsDefault) {
    const hipError_t e = col_allow_big_lds();
    if (e != hipSuccess) return e;
  }
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  hipLaunchKernelGGL(kColTable[fmt][nc - 1], dim3(a.q), dim3(kThreads), lay.total, st, a);
  return hipGetLastError();
}

hipError_t launch_au(int fmt, const AUArgs& a, hipStream_t st, int pol) {
  if (fmt < FMT_F32 || fmt > FMT_PHILOX) return hipErrorInvalidValue;   // A_k U is exact in every form
  if (pol == POL_CACHED) {
    const hipError_t e = launch_au_cached(fmt, a, st);
    if (e != hipErrorNotSupported) return e;
  }
  const int ri = (a.r + 1) / 2 - 1, w = au_width(a.waves);
  const AULayout lay(a.m, a.r, fmt == FMT_PHILOX, w);
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  const au_fn f = w == 8 ? kAU8[fmt][ri]
                         : ((fmt != FMT_PHILOX && a.q <= kDeepAuColumns) ? kAUDeep[fmt][ri] : kAUTable[fmt][ri]);
  hipLaunchKernelGGL(f, dim3(a.q), dim3(64 * w), lay.total, st, a);
  return hipGetLastError();
}

hipError_t launch_col_grp(int fmt, int nc, int waves, const ColArgs* tab, const int2* map, int blocks, size_t lds,
                          hipStream_t st, int pol) {
  if (fmt < FMT_F32 || fmt > FMT_BF16MIX) return hipErrorInvalidValue;
  if (pol == POL_CACHED) {
    const hipError_t e = launch_col_grp_cached(fmt, nc, waves, tab, map, blocks, lds, st);
    if (e != hipErrorNotSupported) return e;
  }
  if (waves == 8 || waves == 16) return launch_col_grp_wide(fmt, nc, waves, tab, map, blocks, lds, st);
  if (waves != kWaves) return hipErrorInvalidValue;
  if (lds > kColLdsDefault) {
    const hipError_t e = col_allow_big_lds();
    if (e != hipSuccess) return e;
  }
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  hipLaunchKernelGGL(kColGrpTable[fmt][nc - 1], dim3(blocks), dim3(kThreads), lds, st, tab, map);
  return hipGetLastError();
}

hipError_t launch_au_grp(int fmt, int rmax, int waves, const AUArgs* tab, const int2* map, int blocks, size_t lds,
                         hipStream_t st, int pol) {
  if (fmt < FMT_F32 || fmt > FMT_PHILOX) return hipErrorInvalidValue;
  if (pol == POL_CACHED) {
    const hipError_t e = launch_au_grp_cached(fmt, rmax, waves, tab, map, blocks, lds, st);
    if (e != hipErrorNotSupported) return e;
  }
  const int ri = (rmax + 1) / 2 - 1, w = au_width(waves);
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  const aug_fn f = w == 8 ? kAUGrp8[fmt][ri]
                          : ((fmt != FMT_PHILOX && blocks <= kDeepAuColumns) ? kAUGrpDeep[fmt][ri]
                                                                              : kAUGrpTable[fmt][ri]);
  hipLaunchKernelGGL(f, dim3(blocks), dim3(64 * w), lds, st, tab, map);
  return hipGetLastError();
}

size_t col_lds_bytes(int n, int m, int r, int rho, int project, int philox, int waves) {
  return ColLayout(n, m, r, rho, project, philox, waves).total;
}

// Raise the dynamic LDS limit of each kernel in `fns` to kColLdsMax (null entries skipped).
template <class F>
static hipError_t raise_lds(const F* fns, size_t count) {
  for (size_t i = 0; i < count; ++i)
    if (fns[i]) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fns[i]),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kColLdsMax);
      if (e != hipSuccess) return e;
    }
  return hipSuccess;
}

hipError_t col_allow_big_lds() {
  static std::mutex mu;
  static bool done = false;
  std::lock_guard<std::mutex> lk(mu);
  if (done) return hipSuccess;
  hipError_t e = raise_lds(&kColTable[0][0], sizeof(kColTable) / sizeof(kColTable[0][0]));
  if (e == hipSuccess) e = raise_lds(&kColGrpTable[0][0], sizeof(kColGrpTable) / sizeof(kColGrpTable[0][0]));
  if (e == hipSuccess) e = col_allow_big_lds_tuned();
  if (e == hipSuccess) e = col_allow_big_lds_cached();
  if (e == hipSuccess) done = true;
  return e;
}
size_t au_lds_bytes(int m, int r, int philox, int waves) { return AULayout(m, r, philox, waves).total; }

// Materialises the Philox form of A into the FP32 layout (one thread per 4-row chunk).
__global__ __launch_bounds__(256) void k_philox_fill(unsigned long long seed, const float* table, int q, int n, int m,
                                                     long long lda, float* A) {
  __shared__ float tab[kNormalTable];
  for (int t = threadIdx.x; t < kNormalTable; t += blockDim.x) tab[t] = table[t];
  __syncthreads();
  const int nch = (m + 3) / 4;
  const long long total = (long long)q * n * nch;
  AUArgs dummy;
  dummy.seed = seed;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total; e += (long long)gridDim.x * blockDim.x) {
    const int ch = (int)(e % nch);
    const int j = (int)((e / nch) % n);
    const int k = (int)(e / ((long long)nch * n));
    ALoader<FMT_PHILOX> L(dummy, k);
    L.tab = tab;
    const float4 v = L.load(j, ch);
    float* dst = A + (long long)k * n * lda + (long long)j * lda + 4 * ch;
    const float vv[4] = {v.x, v.y, v.z, v.w};
    for (int c = 0; c < 4; ++c)
      if (4 * ch + c < m) dst[c] = vv[c];
  }
}

hipError_t launch_philox_fill(unsigned long long seed, const float* table, int q, int n, int m, long long lda, float* A,
                              hipStream_t st) {
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  hipLaunchKernelGGL(k_philox_fill, dim3(1024), dim3(256), 0, st, seed, table, q, n, m, lda, A);
  return hipGetLastError();
}

#endif  // part 1

#if ALTG_PART == 2
// Autotuned variants of the plane formats: k_col with JU in {1, 2, 4, 8} (FP32,
// BF16X2 and the mixed BF16 form) and k_au with AUD in {1, 2, 3, 4, 8} (FP32,
// BF16X2).  JU = 8 and AUD = 8 keep many loads in flight per wave at one or two
// waves per SIMD: for problems with few columns, where each CU holds one or two
// column workgroups.  Every variant gives the same bits as the default one.
typedef void (*col_fn2)(ColArgs);
typedef void (*au_fn2)(AUArgs);
// JU = 8 for at most two row chunks (its loads need every register at more)
#define COLT_NC(F, NC) {k_col<F, NC, 1>, k_col<F, NC, 2>, k_col<F, NC, 4>, k_col<F, NC, 8>}
#define COLT_NC4(F, NC) {k_col<F, NC, 1>, k_col<F, NC, 2>, k_col<F, NC, 4>, nullptr}
#define COLT_F(F) {COLT_NC(F, 1), COLT_NC(F, 2), COLT_NC4(F, 3), COLT_NC4(F, 4)}
static const col_fn2 kColTuned[3][kNCMax][4] = {COLT_F(FMT_F32), COLT_F(FMT_BF16X2), COLT_F(FMT_BF16MIX)};
#define AUT_R(F, R) {k_au<F, R, 1>, k_au<F, R, 2>, k_au<F, R, 3>, k_au<F, R, 4>, k_au<F, R, 8>}
#define AUT_F(F) {AUT_R(F, 2), AUT_R(F, 4), AUT_R(F, 6), AUT_R(F, 8), AUT_R(F, 10), AUT_R(F, 12), AUT_R(F, 14), AUT_R(F, 16)}
static const au_fn2 kAUTuned[2][kRMax / 2][5] = {AUT_F(FMT_F32), AUT_F(FMT_BF16X2)};

template <int N>
static int tuned_slot(int v, const int (&vals)[N]) {
  for (int i = 0; i < N; ++i)
    if (vals[i] == v) return i;
  return -1;
}

// Wide column workgroups (8 and 16 waves) with the default loads in flight of
// their width; 16 waves are built for at most two row chunks (m <= 512).
#define COLW_F(F, W) {k_col<F, 1, default_ju(1, W, F), W>, k_col<F, 2, default_ju(2, W, F), W>, \
                      k_col<F, 3, default_ju(3, W, F), W>, k_col<F, 4, default_ju(4, W, F), W>}
#define COLW16_F(F) {k_col<F, 1, default_ju(1, 16), 16>, k_col<F, 2, default_ju(2, 16), 16>, nullptr, nullptr}
static const col_fn2 kColWide[2][5][kNCMax] = {
    {COLW_F(FMT_F32, 8), COLW_F(FMT_BF16X2, 8), COLW_F(FMT_BF16HI, 8), COLW_F(FMT_PHILOX, 8), COLW_F(FMT_BF16MIX, 8)},
    {COLW16_F(FMT_F32), COLW16_F(FMT_BF16X2), COLW16_F(FMT_BF16HI), COLW16_F(FMT_PHILOX), COLW16_F(FMT_BF16MIX)}};
typedef void (*colg_fn2)(const ColArgs*, const int2*);
#define COLGW_F(F, W) {k_col_grp<F, 1, W>, k_col_grp<F, 2, W>, k_col_grp<F, 3, W>, k_col_grp<F, 4, W>}
#define COLGW16_F(F) {k_col_grp<F, 1, 16>, k_col_grp<F, 2, 16>, nullptr, nullptr}
static const colg_fn2 kColGrpWide[2][5][kNCMax] = {
    {COLGW_F(FMT_F32, 8), COLGW_F(FMT_BF16X2, 8), COLGW_F(FMT_BF16HI, 8), COLGW_F(FMT_PHILOX, 8),
     COLGW_F(FMT_BF16MIX, 8)},
    {COLGW16_F(FMT_F32), COLGW16_F(FMT_BF16X2), COLGW16_F(FMT_BF16HI), COLGW16_F(FMT_PHILOX), COLGW16_F(FMT_BF16MIX)}};

bool col_wide_built(int waves, int nc) { return waves == 8 || (waves == 16 && nc <= 2); }

hipError_t launch_col_wide(int fmt, const ColArgs& a, hipStream_t st) {
  const int nc = (a.m + 255) / 256;
  const int wi = a.waves == 16 ? 1 : 0;
  if (fmt < FMT_F32 || fmt > FMT_BF16MIX || nc < 1 || nc > kNCMax || !kColWide[wi][fmt][nc - 1])
    return hipErrorNotSupported;
  const ColLayout lay(a.n, a.m, a.r, a.rho, a.project, fmt == FMT_PHILOX, a.waves);
  if (lay.total > kColLdsDefault) {
    const hipError_t e = col_allow_big_lds();
    if (e != hipSuccess) return e;
  }
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  hipLaunchKernelGGL(kColWide[wi][fmt][nc - 1], dim3(a.q), dim3(64 * a.waves), lay.total, st, a);
  return hipGetLastError();
}

hipError_t launch_col_grp_wide(int fmt, int nc, int waves, const ColArgs* tab, const int2* map, int blocks,
                               size_t lds, hipStream_t st) {
  const int wi = waves == 16 ? 1 : 0;
  if (fmt < FMT_F32 || fmt > FMT_BF16MIX || nc < 1 || nc > kNCMax || !kColGrpWide[wi][fmt][nc - 1])
    return hipErrorNotSupported;
  if (lds > kColLdsDefault) {
    const hipError_t e = col_allow_big_lds();
    if (e != hipSuccess) return e;
  }
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  hipLaunchKernelGGL(kColGrpWide[wi][fmt][nc - 1], dim3(blocks), dim3(64 * waves), lds, st, tab, map);
  return hipGetLastError();
}

template <class F>
static hipError_t raise_lds(const F* fns, size_t count) {
  for (size_t i = 0; i < count; ++i)
    if (fns[i]) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fns[i]),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kColLdsMax);
      if (e != hipSuccess) return e;
    }
  return hipSuccess;
}

hipError_t col_allow_big_lds_tuned() {
  hipError_t e = raise_lds(&kColTuned[0][0][0], sizeof(kColTuned) / sizeof(kColTuned[0][0][0]));
  if (e == hipSuccess) e = raise_lds(&kColWide[0][0][0], sizeof(kColWide) / sizeof(kColWide[0][0][0]));
  if (e == hipSuccess) e = raise_lds(&kColGrpWide[0][0][0], sizeof(kColGrpWide) / sizeof(kColGrpWide[0][0][0]));
  return e;
}

hipError_t launch_col_tuned(int fmt, int ju, const ColArgs& a, hipStream_t st) {
  static const int kJU[4] = {1, 2, 4, 8};
  const int slot = tuned_slot(ju, kJU);
  const int row = fmt == FMT_F32 ? 0 : fmt == FMT_BF16X2 ? 1 : fmt == FMT_BF16MIX ? 2 : -1;
  if (row < 0 || slot < 0) return hipErrorInvalidValue;
  const int nc = (a.m + 255) / 256;
  if (!kColTuned[row][nc - 1][slot]) return hipErrorNotSupported;   // variant not built
  const ColLayout lay(a.n, a.m, a.r, a.rho, a.project, 0);
  if (lay.total > kColLdsDefault) {
    const hipError_t e = col_allow_big_lds();
    if (e != hipSuccess) return e;
  }
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  hipLaunchKernelGGL(kColTuned[row][nc - 1][slot], dim3(a.q), dim3(kThreads), lay.total, st, a);
  return hipGetLastError();
}

hipError_t launch_au_tuned(int fmt, int aud, const AUArgs& a, hipStream_t st) {
  static const int kAUD[5] = {1, 2, 3, 4, 8};
  const int slot = tuned_slot(aud, kAUD);
  if ((fmt != FMT_F32 && fmt != FMT_BF16X2) || slot < 0) return hipErrorInvalidValue;
  const int ri = (a.r + 1) / 2 - 1;
  const AULayout lay(a.m, a.r, 0);
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  hipLaunchKernelGGL(kAUTuned[fmt == FMT_F32 ? 0 : 1][ri][slot], dim3(a.q), dim3(kThreads), lay.total, st, a);
  return hipGetLastError();
}
#endif  // ALTG_PART == 2

#if ALTG_PART == 3
// Cached-load (POL_CACHED) instantiations of the default column and A_k U
// kernels, for problems whose streamed plane fits in the Infinity Cache: 4- and
// 8-wave column workgroups, the single-problem and the batched launches.  The
// Philox form loads no A and has none (its launches take the streaming kernels).
typedef void (*col_fn3)(ColArgs);
typedef void (*colg_fn3)(const ColArgs*, const int2*);
typedef void (*au_fn3)(AUArgs);
typedef void (*aug_fn3)(const AUArgs*, const int2*);
#define COLC_F(F, W) {k_col<F, 1, default_ju(1, W, F), W, POL_CACHED>, k_col<F, 2, default_ju(2, W, F), W, POL_CACHED>, \
                      k_col<F, 3, default_ju(3, W, F), W, POL_CACHED>, k_col<F, 4, default_ju(4, W, F), W, POL_CACHED>}
#define COLC_NONE {nullptr, nullptr, nullptr, nullptr}
static const col_fn3 kColCached[2][5][kNCMax] = {
    {COLC_F(FMT_F32, 4), COLC_F(FMT_BF16X2, 4), COLC_F(FMT_BF16HI, 4), COLC_NONE, COLC_F(FMT_BF16MIX, 4)},
    {COLC_F(FMT_F32, 8), COLC_F(FMT_BF16X2, 8), COLC_F(FMT_BF16HI, 8), COLC_NONE, COLC_F(FMT_BF16MIX, 8)}};
#define COLGC_F(F, W) {k_col_grp<F, 1, W, POL_CACHED>, k_col_grp<F, 2, W, POL_CACHED>, \
                       k_col_grp<F, 3, W, POL_CACHED>, k_col_grp<F, 4, W, POL_CACHED>}
static const colg_fn3 kColGrpCached[2][5][kNCMax] = {
    {COLGC_F(FMT_F32, 4), COLGC_F(FMT_BF16X2, 4), COLGC_F(FMT_BF16HI, 4), COLC_NONE, COLGC_F(FMT_BF16MIX, 4)},
    {COLGC_F(FMT_F32, 8), COLGC_F(FMT_BF16X2, 8), COLGC_F(FMT_BF16HI, 8), COLC_NONE, COLGC_F(FMT_BF16MIX, 8)}};
// [0]: the default depths; [1]: the deep ones, for launches of at most kDeepAuColumns columns
#define AUC_F(F, D) {k_au<F, 2, D(2, F), POL_CACHED>, k_au<F, 4, D(4, F), POL_CACHED>, k_au<F, 6, D(6, F), POL_CACHED>,     \
                     k_au<F, 8, D(8, F), POL_CACHED>, k_au<F, 10, D(10, F), POL_CACHED>, k_au<F, 12, D(12, F), POL_CACHED>, \
                     k_au<F, 14, D(14, F), POL_CACHED>, k_au<F, 16, D(16, F), POL_CACHED>}
static const au_fn3 kAUCached[2][3][kRMax / 2] = {
    {AUC_F(FMT_F32, default_aud), AUC_F(FMT_BF16X2, default_aud), AUC_F(FMT_BF16HI, default_aud)},
    {AUC_F(FMT_F32, deep_aud), AUC_F(FMT_BF16X2, deep_aud), AUC_F(FMT_BF16HI, deep_aud)}};
#define AUGC_F(F, D) {k_au_grp<F, 2, POL_CACHED, D(2, F)>, k_au_grp<F, 4, POL_CACHED, D(4, F)>,   \
                      k_au_grp<F, 6, POL_CACHED, D(6, F)>, k_au_grp<F, 8, POL_CACHED, D(8, F)>,   \
                      k_au_grp<F, 10, POL_CACHED, D(10, F)>, k_au_grp<F, 12, POL_CACHED, D(12, F)>, \
                      k_au_grp<F, 14, POL_CACHED, D(14, F)>, k_au_grp<F, 16, POL_CACHED, D(16, F)>}
static const aug_fn3 kAUGrpCached[2][3][kRMax / 2] = {
    {AUGC_F(FMT_F32, default_aud), AUGC_F(FMT_BF16X2, default_aud), AUGC_F(FMT_BF16HI, default_aud)},
    {AUGC_F(FMT_F32, deep_aud), AUGC_F(FMT_BF16X2, deep_aud), AUGC_F(FMT_BF16HI, deep_aud)}};
// 8-wave workgroups (deep depths), as in the streaming tables
#define AUC8_F(F) {k_au<F, 2, deep_aud(2), POL_CACHED, 8>, k_au<F, 4, deep_aud(4), POL_CACHED, 8>,     \
                   k_au<F, 6, deep_aud(6), POL_CACHED, 8>, k_au<F, 8, deep_aud(8), POL_CACHED, 8>,     \
                   k_au<F, 10, deep_aud(10), POL_CACHED, 8>, k_au<F, 12, deep_aud(12), POL_CACHED, 8>, \
                   k_au<F, 14, deep_aud(14), POL_CACHED, 8>, k_au<F, 16, deep_aud(16), POL_CACHED, 8>}
static const au_fn3 kAUCached8[3][kRMax / 2] = {AUC8_F(FMT_F32), AUC8_F(FMT_BF16X2), AUC8_F(FMT_BF16HI)};
#define AUGC8_F(F) {k_au_grp<F, 2, POL_CACHED, deep_aud(2), 8>, k_au_grp<F, 4, POL_CACHED, deep_aud(4), 8>,     \
                    k_au_grp<F, 6, POL_CACHED, deep_aud(6), 8>, k_au_grp<F, 8, POL_CACHED, deep_aud(8), 8>,     \
                    k_au_grp<F, 10, POL_CACHED, deep_aud(10), 8>, k_au_grp<F, 12, POL_CACHED, deep_aud(12), 8>, \
                    k_au_grp<F, 14, POL_CACHED, deep_aud(14), 8>, k_au_grp<F, 16, POL_CACHED, deep_aud(16), 8>}
static const aug_fn3 kAUGrpCached8[3][kRMax / 2] = {AUGC8_F(FMT_F32), AUGC8_F(FMT_BF16X2), AUGC8_F(FMT_BF16HI)};

static int cached_width_row(int waves) { return waves == 8 ? 1 : (waves == 0 || waves == kWaves ? 0 : -1); }

hipError_t col_allow_big_lds_cached() {
  for (size_t i = 0; i < sizeof(kColCached) / sizeof(kColCached[0][0][0]); ++i) {
    const col_fn3 f = (&kColCached[0][0][0])[i];
    if (!f) continue;
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(f),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)kColLdsMax);
    if (e != hipSuccess) return e;
  }
  for (size_t i = 0; i < sizeof(kColGrpCached) / sizeof(kColGrpCached[0][0][0]); ++i) {
    const colg_fn3 f = (&kColGrpCached[0][0][0])[i];
    if (!f) continue;
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(f),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)kColLdsMax);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_col_cached(int fmt, const ColArgs& a, hipStream_t st) {
  const int nc = (a.m + 255) / 256, wi = cached_width_row(a.waves);
  if (fmt < FMT_F32 || fmt > FMT_BF16MIX || wi < 0 || nc < 1 || nc > kNCMax || !kColCached[wi][fmt][nc - 1])
    return hipErrorNotSupported;
  const int w = wi ? 8 : kWaves;
  const ColLayout lay(a.n, a.m, a.r, a.rho, a.project, 0, w);
  if (lay.total > kColLdsDefault) {
    const hipError_t e = col_allow_big_lds();
    if (e != hipSuccess) return e;
  }
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  hipLaunchKernelGGL(kColCached[wi][fmt][nc - 1], dim3(a.q), dim3(64 * w), lay.total, st, a);
  return hipGetLastError();
}

hipError_t launch_col_grp_cached(int fmt, int nc, int waves, const ColArgs* tab, const int2* map, int blocks,
                                 size_t lds, hipStream_t st) {
  const int wi = cached_width_row(waves);
  if (fmt < FMT_F32 || fmt > FMT_BF16MIX || wi < 0 || nc < 1 || nc > kNCMax || !kColGrpCached[wi][fmt][nc - 1])
    return hipErrorNotSupported;
  if (lds > kColLdsDefault) {
    const hipError_t e = col_allow_big_lds();
    if (e != hipSuccess) return e;
  }
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  hipLaunchKernelGGL(kColGrpCached[wi][fmt][nc - 1], dim3(blocks), dim3(64 * (wi ? 8 : kWaves)), lds, st, tab, map);
  return hipGetLastError();
}

hipError_t launch_au_cached(int fmt, const AUArgs& a, hipStream_t st) {
  if (fmt < FMT_F32 || fmt > FMT_BF16HI) return hipErrorNotSupported;
  const int ri = (a.r + 1) / 2 - 1, w = a.waves == 8 ? 8 : kWaves;
  const AULayout lay(a.m, a.r, 0, w);
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  const au_fn3 f = w == 8 ? kAUCached8[fmt][ri] : kAUCached[a.q <= kDeepAuColumns][fmt][ri];
  hipLaunchKernelGGL(f, dim3(a.q), dim3(64 * w), lay.total, st, a);
  return hipGetLastError();
}

hipError_t launch_au_grp_cached(int fmt, int rmax, int waves, const AUArgs* tab, const int2* map, int blocks,
                                size_t lds, hipStream_t st) {
  if (fmt < FMT_F32 || fmt > FMT_BF16HI) return hipErrorNotSupported;
  const int ri = (rmax + 1) / 2 - 1, w = waves == 8 ? 8 : kWaves;
  (void)hipGetLastError();   // clear a stale error of an earlier, unrelated call
  const aug_fn3 f = w == 8 ? kAUGrpCached8[fmt][ri] : kAUGrpCached[blocks <= kDeepAuColumns][fmt][ri];
  hipLaunchKernelGGL(f, dim3(blocks), dim3(64 * w), lds, st, tab, map);
  return hipGetLastError();
}
#endif  // ALTG_PART == 3

}  // namespace altg
