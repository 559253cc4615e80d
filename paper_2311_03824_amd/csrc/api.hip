// C ABI of the AltGDmin-LR+S hot path (declarations and contracts in include/altgdmin.h).
//
// Host side only: validation, workspace carving, launch sequencing and the HIP
// graph of one GDmin iteration.  Every step of the method runs in the kernels
// of k_column.hip and k_small.hip.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "altgdmin.h"
#include "launch.h"

using namespace altg;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define HIPCHK(x)                                                                         \
  do {                                                                                    \
    hipError_t e_ = (x);                                                                  \
    if (e_ != hipSuccess) return fail(ALTGDMIN_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Every entry point that enqueues work takes the caller's stream; the library
// never enqueues on the null (legacy default) stream.
#define NEED_STREAM(s)                                                                     \
  do {                                                                                     \
    if (!(s)) return fail(ALTGDMIN_EINVAL, "stream is NULL: pass a created HIP stream"); \
  } while (0)

// Events that are destroyed on every exit path.
struct EventPair {
  hipEvent_t e[2] = {nullptr, nullptr};
  hipError_t create() {
    hipError_t r = hipEventCreate(&e[0]);
    return r == hipSuccess ? hipEventCreate(&e[1]) : r;
  }
  ~EventPair() {
    for (hipEvent_t x : e)
      if (x) (void)hipEventDestroy(x);
  }
};

constexpr size_t kAlign = 256;
constexpr size_t kMaxLds = 64 * 1024;

// Lays arrays out in the workspace at 256-byte boundaries.  A null base only
// measures (the addresses are formed as integers, never as offsets of null).
struct Carver {
  uintptr_t base;
  size_t off = 0;
  explicit Carver(void* b) : base(reinterpret_cast<uintptr_t>(b)) {}
  template <class T>
  T* take(size_t count) {
    off = (off + kAlign - 1) / kAlign * kAlign;
    T* p = reinterpret_cast<T*>(base + off);
    off += count * sizeof(T);
    return p;
  }
};

// column splits of the gradient reduction: enough workgroups to fill the
// chip for small n, one split when every split would hold few columns
int grad_splits(int q) { return q >= 512 ? 4 : (q >= 64 ? 2 : 1); }

// Automatic rank (Sec. 2.6): K = max(1, floor(min(n, q, m) / 10)) leading singular
// values of L_0 decide r; the block subspace iteration carries b = K + 8 columns
// (capped by the LDS of its b x b FP64 matrices and by min(n, q)).
int rank_budget(int n, int q, int m) { return std::max(1, std::min(n, std::min(q, m)) / 10); }
int rank_block(int n, int q, int m) {
  return std::min(rank_budget(n, q, m) + 8, std::min(kRankBlockMax, std::min(n, q)));
}
// the rank the workspace is laid out for: r, or with r = 0 the largest the automatic rule may pick
int r_eff(const altgdmin_problem& p) {
  if (p.r > 0) return p.r;
  const int cap = p.a_format == ALTGDMIN_A_PFOURIER ? kFRMax : kRMax;
  return std::min(std::min(rank_budget(p.n, p.q, p.m), cap), std::min(p.m, p.n));
}

// The matrix the rank estimate runs on and its sizes: L_0 itself for the real
// forms (n x q; K values, a block of b columns); for the Fourier form the real
// embedding [[X, -Y], [Y, X]] of L_0 = X + iY (2n x 2q), whose singular values are
// those of L_0 twice each, so K and the block double.
struct RankShape {
  int n, q, K, b;
};
RankShape rank_shape(int n, int q, int m) { return {n, q, rank_budget(n, q, m), rank_block(n, q, m)}; }
RankShape rank_shape_complex(int n, int q, int m) {
  const int K = rank_budget(n, q, m);
  return {2 * n, 2 * q, 2 * K, std::min(2 * K + 8, std::min(kRankBlockMax, std::min(2 * n, 2 * q)))};
}

// Scratch of the automatic rank: the block U and Z = L_0 L_0^T U (n x b), T = L_0^T U
// (q x b), the FP64 Gram and R^{-1} (b x b), R^{-1} in FP32, the K values, r, a flag.
struct RankScratch {
  float* Ub;
  float* Z;
  float* T;
  double* W;
  double* Xinv;
  float* Xf;
  double* sv;
  int* r;
  int* flag;
  size_t bytes;
};

RankScratch rank_scratch(void* base, const RankShape& sh) {
  const size_t n = sh.n, q = sh.q, b = sh.b, K = sh.K;
  RankScratch s;
  Carver c(base);
  s.Ub = c.take<float>((size_t)n * b);
  s.Z = c.take<float>((size_t)n * b);
  s.T = c.take<float>((size_t)q * b);
  s.W = c.take<double>(b * b);
  s.Xinv = c.take<double>(b * b);
  s.Xf = c.take<float>(b * b);
  s.sv = c.take<double>(K);
  s.r = c.take<int>(1);
  s.flag = c.take<int>(1);
  s.bytes = (c.off + kAlign - 1) / kAlign * kAlign;
  return s;
}

// Enqueues the automatic rank on L_0 (given as L0t, q x n): `iters` steps of the
// block subspace iteration from a fixed orthonormal start, each Z = L_0 (L_0^T U)
// and CholeskyQR2, then the Rayleigh-Ritz values and the rank (device outputs r,
// sv).  Returns the buffer that holds the final orthonormal block (n x b).
hipError_t enqueue_rank(const float* L0t, const RankShape& sh, double energy, int iters, RankScratch& s,
                        float** block, hipStream_t st) {
  const int n = sh.n, q = sh.q, b = sh.b, K = sh.K;
  float* U = s.Ub;
  float* Z = s.Z;
  hipError_t e = launch_fill_int(s.flag, 0, 1, st);
  if (e == hipSuccess) e = launch_fill_basis(U, n, b, st);
  for (int it = 0; it < iters && e == hipSuccess; ++it) {
    e = launch_rank_mm(false, L0t, n, U, b, s.T, b, q, b, n, st);                 // T = L_0^T U
    if (e == hipSuccess) e = launch_rank_mm(true, L0t, n, s.T, b, Z, b, n, b, q, st);   // Z = L_0 T
    for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {                     // CholeskyQR2: Z -> U -> Z
      e = launch_rank_gram(Z, n, b, s.W, st);
      if (e == hipSuccess) e = launch_rank_chol(s.W, b, s.Xinv, s.Xf, s.flag, st);
      if (e == hipSuccess) e = launch_rank_mm(false, Z, b, s.Xf, b, U, b, n, b, b, st);
      std::swap(U, Z);
    }
    std::swap(U, Z);   // after two passes the orthonormal block is in Z: name it U again
  }
  if (e == hipSuccess) e = launch_rank_mm(false, L0t, n, U, b, s.T, b, q, b, n, st);   // T = L_0^T U
  if (e == hipSuccess) e = launch_rank_gram(s.T, q, b, s.W, st);                       // M = T^T T
  if (e == hipSuccess) e = launch_rank_jacobi(s.W, b, K, energy, s.sv, s.r, st);
  *block = U;
  return e;
}

int fmt_of(const altgdmin_problem* p) {
  switch (p->a_format) {
    case ALTGDMIN_A_BF16X2: return FMT_BF16X2;
    case ALTGDMIN_A_PHILOX: return FMT_PHILOX;
    case ALTGDMIN_A_PFOURIER: return FMT_PFOURIER;
    default: return FMT_F32;
  }
}

}  // namespace

struct altgdmin_handle {
  altgdmin_problem prob;
  altgdmin_params par;
  int fmt;
  float* P;
  double* Ginv;
  int* Tidx;
  float* Tval;
  float* Bt;
  float* H;
  double* colrr;
  int* colflags;
  float* gpart;
  int KS;
  float* U;
  float* Uprev;
  float* Utmp;
  float* Tpow;
  Ctl* ctl;
  double* rlog;
  int rlog_len;
  // partial Fourier form: complex buffers (float pairs); Tval, Bt, H, gpart (the
  // gradient or L_0 L_0^H U), U, Uprev, Utmp and Tpow hold complex values there
  float* FU = nullptr;     // n x r: the 2D DFT of U's columns
  float* tw = nullptr;     // 96 twiddles
  double* fpart = nullptr; // per-256-row-block partial Grams of the GD update
  double* frinv = nullptr; // R1^{-1}, R2^{-1} of the GD update
  void* rank_ws = nullptr; // r = 0 (automatic rank): scratch of the rank estimate
  float* rank_embed = nullptr;  // Fourier form, r = 0: the real embedding of L_0 (2q x 2n)
  int col_waves = kWaves;  // waves of the column workgroup (a property of the problem, see choose_col_waves)
  int col_unroll = 0;      // autotuned JU of the column kernel (0: the default instantiation)
  int au_depth = 0;        // autotuned AUD of the A_k U kernel (0: the default instantiation)
  int colfmt = 0;          // format of the column kernel: fmt, or the mixed BF16 form
  bool hi_phase = false;   // BF16X2 with a hi-only phase
  bool auto_rank = false;  // the problem asked for r = 0: r is chosen at init (Sec. 2.6)
  bool have_graph = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int t_host = 0;
};

namespace {

// Workspace of the partial Fourier form (complex values as float pairs).
size_t carve_fourier(altgdmin_handle* h, void* base) {
  const altgdmin_problem& p = h->prob;
  const size_t n = p.n, q = p.q, r = r_eff(p), rho = p.rho;
  Carver c(base);
  h->ctl = c.take<Ctl>(1);
  h->P = nullptr;
  h->Ginv = nullptr;
  h->Tidx = c.take<int>(q * rho);
  h->Tval = c.take<float>(2 * q * rho);
  h->Bt = c.take<float>(2 * q * r);
  h->H = c.take<float>(2 * q * n);
  h->colrr = c.take<double>(q);
  h->colflags = c.take<int>(q);
  h->KS = 1;
  h->gpart = c.take<float>(2 * n * r);
  h->FU = c.take<float>(2 * n * r);
  h->U = c.take<float>(2 * n * r);
  h->Uprev = c.take<float>(2 * n * r);
  h->Utmp = c.take<float>(2 * n * r);
  h->Tpow = c.take<float>(2 * q * r);
  h->tw = c.take<float>(2 * (size_t)std::max(kFN, p.n1 + p.n2));
  h->fpart = c.take<double>(2 * 3 * r * r * ((n + 255) / 256));
  h->frinv = c.take<double>(2 * 2 * r * r);
  h->rlog_len = h->par.t_max > 0 ? h->par.t_max : 1;
  h->rlog = c.take<double>(h->rlog_len);
  if (p.r == 0) {   // automatic rank: the real embedding of L_0 and the estimate's scratch
    h->rank_embed = c.take<float>(4 * q * n);
    h->rank_ws = c.take<unsigned char>(rank_scratch(nullptr, rank_shape_complex(p.n, p.q, p.m)).bytes);
  }
  return (c.off + kAlign - 1) / kAlign * kAlign;
}

// Lays the workspace out; with base == nullptr it only measures.
size_t carve(altgdmin_handle* h, void* base) {
  if (h->prob.a_format == ALTGDMIN_A_PFOURIER) return carve_fourier(h, base);
  const altgdmin_problem& p = h->prob;
  const size_t n = p.n, q = p.q, m = p.m, r = r_eff(p), rho = p.rho;
  Carver c(base);
  h->ctl = c.take<Ctl>(1);
  h->P = c.take<float>(q * m * r);
  h->Ginv = c.take<double>(q * r * r);
  h->Tidx = c.take<int>(q * rho);
  h->Tval = c.take<float>(q * rho);
  h->Bt = c.take<float>(q * r);
  h->H = c.take<float>(q * n);
  h->colrr = c.take<double>(q);
  h->colflags = c.take<int>(q);
  h->KS = grad_splits(p.q);
  h->gpart = c.take<float>((size_t)h->KS * n * r);
  h->U = c.take<float>(n * r);
  h->Uprev = c.take<float>(n * r);
  h->Utmp = c.take<float>(n * r);
  h->Tpow = c.take<float>(q * r);
  h->rlog_len = h->par.t_max > 0 ? h->par.t_max : 1;
  h->rlog = c.take<double>(h->rlog_len);
  if (p.r == 0) h->rank_ws = c.take<unsigned char>(rank_scratch(nullptr, rank_shape(p.n, p.q, p.m)).bytes);
  return (c.off + kAlign - 1) / kAlign * kAlign;
}

int validate(const altgdmin_problem* p, const altgdmin_params* par) {
  if (!p || !par) return fail(ALTGDMIN_EINVAL, "null problem or params");
  if (p->n < 1 || p->q < 1 || p->m < 1) return fail(ALTGDMIN_EINVAL, "n, q, m must be >= 1");
  if (p->r < 0 || (p->r > 0 && (p->r > p->m || p->r > p->n)))
    return fail(ALTGDMIN_EINVAL, "need 1 <= r <= min(m, n), or r = 0 for the automatic rank");
  if (p->r == 0 && (p->a_format == ALTGDMIN_A_PFOURIER ? 2 : 1) * rank_budget(p->n, p->q, p->m) > kRankBlockMax)
    return fail(ALTGDMIN_ENOTBUILT, "automatic rank: min(n, q, m) / 10 above the largest block of the estimate");
  if (p->r == 0 && !(par->rank_energy > 0.0 && par->rank_energy <= 1.0 && par->rank_iters >= 1))
    return fail(ALTGDMIN_EINVAL, "automatic rank needs 0 < rank_energy <= 1 and rank_iters >= 1");
  if (p->rho < 0 || p->rho > p->n) return fail(ALTGDMIN_EINVAL, "need 0 <= rho <= n");
  if (par->tau0 < 0 || par->tau < 0 || par->t_max < 0 || par->power_iters < 0 || par->poll_every < 1 ||
      !(par->eta_c >= 0.0) || par->bf16_hi_max < 0 ||
      (par->flags & ~(ALTGDMIN_FLAG_EAGER | ALTGDMIN_FLAG_AUTOTUNE | ALTGDMIN_FLAG_BF16_MIXED)))
    return fail(ALTGDMIN_EINVAL, "invalid params");
  if ((par->flags & ALTGDMIN_FLAG_BF16_MIXED) && (p->a_format != ALTGDMIN_A_BF16X2 || par->bf16_hi_max > 0))
    return fail(ALTGDMIN_EINVAL, "the mixed BF16 form needs BF16X2 planes and no hi-only phase");
  if (p->a_format == ALTGDMIN_A_PFOURIER) {
    if (p->n1 < 1 || p->n2 < 1 || (int64_t)p->n1 * p->n2 != p->n) return fail(ALTGDMIN_EINVAL, "need n = n1 * n2");
    if (p->m > p->n) return fail(ALTGDMIN_EINVAL, "need m <= n");
    if (!(p->n1 == kFN && p->n2 == kFN)) {   // generic frames: direct line DFTs in LDS
      if (p->n > kFGenPer * kFThreads || p->n1 > kFGenLineMax || p->n2 > kFGenLineMax)
        return fail(ALTGDMIN_ENOTBUILT, "Fourier form: frames other than 96 x 96 are built for n <= 4096 and "
                                        "n1, n2 <= 1024");
    }
    if (p->m > 2 * kFThreads) return fail(ALTGDMIN_ENOTBUILT, "Fourier form: m > 2048 has no instantiation");
    if (p->r > kFRMax) return fail(ALTGDMIN_ENOTBUILT, "Fourier form: r > 8 has no instantiation");
    if (p->rho > kFRhoMax) return fail(ALTGDMIN_ENOTBUILT, "Fourier form: rho > 256 has no instantiation");
    if (fcol_lds_bytes(p->rho, r_eff(*p), p->n, p->m, p->n1, p->n2) > kFLdsMax)
      return fail(ALTGDMIN_ENOTBUILT, "Fourier form: the frame and the rows of P_k need more LDS than a CU has");
    if (!p->fourier_mask || !p->Y) return fail(ALTGDMIN_EINVAL, "Fourier form needs the mask and Y");
    if (p->ldy < p->m) return fail(ALTGDMIN_EINVAL, "ldy must be >= m");
    if (reinterpret_cast<uintptr_t>(p->Y) % 8 != 0) return fail(ALTGDMIN_EINVAL, "Y must be 8-byte aligned");
    return ALTGDMIN_OK;
  }
  if (p->r > kRMax) return fail(ALTGDMIN_ENOTBUILT, "r > 16 has no instantiation");
  const int re = r_eff(*p);
  if (p->m > 256 * kNCMax) return fail(ALTGDMIN_ENOTBUILT, "m > 1024 has no instantiation");
  if (p->a_format != ALTGDMIN_A_F32 && p->a_format != ALTGDMIN_A_BF16X2 && p->a_format != ALTGDMIN_A_PHILOX)
    return fail(ALTGDMIN_EINVAL, "unknown a_format");
  if (!p->Y) return fail(ALTGDMIN_EINVAL, "Y must be non-null");
  if (p->a_format == ALTGDMIN_A_PHILOX) {
    if (!p->normal_table) return fail(ALTGDMIN_EINVAL, "PHILOX needs the normal table");
  } else {
    if (!p->A) return fail(ALTGDMIN_EINVAL, "A must be non-null");
    if (p->a_format == ALTGDMIN_A_BF16X2 && !p->A_lo) return fail(ALTGDMIN_EINVAL, "BF16X2 needs A_lo");
    if (p->lda < p->m || p->lda % 4 != 0) return fail(ALTGDMIN_EINVAL, "lda must be >= m and a multiple of 4");
    if (p->a_stride_k < p->lda * (int64_t)p->n || p->a_stride_k % 4 != 0)
      return fail(ALTGDMIN_EINVAL, "a_stride_k must be >= lda*n and a multiple of 4");
    const size_t align = p->a_format == ALTGDMIN_A_F32 ? 16 : 8;
    if (reinterpret_cast<uintptr_t>(p->A) % align != 0 ||
        (p->A_lo && reinterpret_cast<uintptr_t>(p->A_lo) % align != 0))
      return fail(ALTGDMIN_EINVAL, "A planes are not aligned to 4 elements");
  }
  if (p->ldy < p->m) return fail(ALTGDMIN_EINVAL, "ldy must be >= m");
  if (!au_supported(p->m, re)) return fail(ALTGDMIN_ENOTBUILT, "no A_k U instantiation for this (m, r)");
  const int phx = p->a_format == ALTGDMIN_A_PHILOX;
  if (col_lds_bytes(p->n, p->m, re, p->rho, 1, phx) > kColLdsMax || au_lds_bytes(p->m, re, phx, 8) > kMaxLds)
    return fail(ALTGDMIN_ENOTBUILT, "problem needs more than 160 KiB of LDS per column workgroup");
  return ALTGDMIN_OK;
}

// Waves of the column workgroup of a problem.  One workgroup per column cannot
// fill the 256 CUs when q is small, and a CU then streams faster with more
// waves in flight: 8 waves up to 512 columns, 4 above; the mixed BF16 form
// (mixed) takes 8 only up to 320.  At n = 1000, m = 400, r = 10: k_col 31 %
// faster at q = 125 and 9 % at q = 250 in FP32, 45 % and 42 % in the mixed form;
// at q = 330 / 400 / 500 FP32 0.420 / 0.446 / 0.521 ms against 0.474 / 0.494 /
// 0.534 with 4, the mixed form 0.367 / 0.376 / 0.395 against 0.321 / 0.328 /
// 0.340; at q = 700 4 waves win (0.696 against 0.748); 16 waves measured slower
// than 8 at every q.  The width sets the order of the cross-wave sums, so it is
// fixed by the problem, never by timing (the FP32 plane, the exact BF16 split and
// the Philox form share it and so their bits).  A width not built for m, or
// whose LDS does not fit, falls back to the next narrower.
// ALTGDMIN_COL_WAVES=4|8|16 forces a width (measurements, tests).
int choose_col_waves(const altgdmin_problem& p, bool mixed) {
  const int phx = p.a_format == ALTGDMIN_A_PHILOX;
  // above 64 KiB of LDS (large n) a CU holds one column workgroup: 8 waves keep
  // more loads in flight whatever q
  const bool big = col_lds_bytes(p.n, p.m, r_eff(p), p.rho, 1, phx) > kColLdsDefault;
  int w = p.q <= 320 || big || (!mixed && p.q <= 512) ? 8 : kWaves;
  if (const char* f = std::getenv("ALTGDMIN_COL_WAVES")) {
    const int v = std::atoi(f);
    if (v == 4 || v == 8 || v == 16) w = v;
  }
  const int nc = (p.m + 255) / 256;
  if (phx) w = std::min(w, nc == 1 ? 16 : (nc == 2 ? 8 : kWaves));   // the generator's registers: wide only at small m
  const size_t cap = big ? kColLdsMax : kColLdsDefault;
  while (w > kWaves && (!col_wide_built(w, nc) || col_lds_bytes(p.n, p.m, r_eff(p), p.rho, 1, phx, w) > cap))
    w /= 2;
  return w;
}

// Waves of the A_k U workgroup: 8 up to 512 columns, 4 above (n = 1000, m = 400,
// r = 10: 0.065 against 0.094 ms at q = 125, 0.134 against 0.147 at q = 330 in
// FP32 and 0.159 against 0.204 with BF16 hi + lo planes, 0.157 against 0.161 at
// q = 500; 0.223 against 0.192 at q = 700).  It sets the order of the cross-wave
// sums of P_k, so, like the column width, it is a property of the problem (of q,
// not of the A format), the same in solo and batched launches.
// ALTGDMIN_AU_WAVES=4|8 forces a width (tests of the 4-wave tuned depths).
int au_waves(const altgdmin_problem& p) {
  int w = p.q <= 512 ? 8 : kWaves;
  if (const char* f = std::getenv("ALTGDMIN_AU_WAVES")) {
    const int v = std::atoi(f);
    if (v == 4 || v == 8) w = v;
  }
  return w;
}

ColArgs col_args(const altgdmin_handle* h) {
  const altgdmin_problem& p = h->prob;
  ColArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = p.n; a.q = p.q; a.m = p.m; a.r = p.r; a.rho = p.rho;
  a.A = p.A; a.Alo = p.A_lo; a.lda = p.lda; a.sA = p.a_stride_k;
  a.Y = p.Y; a.ldy = p.ldy;
  a.P = h->P; a.Ginv = h->Ginv; a.Tidx = h->Tidx; a.Tval = h->Tval;
  a.H = h->H; a.Bt = h->Bt; a.rr = h->colrr; a.flags = h->colflags;
  a.seed = p.a_seed; a.table = p.normal_table;
  a.waves = h->col_waves;
  return a;
}

QRArgs qr_args(const altgdmin_handle* h, int mode) {
  QRArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = h->prob.n; a.r = h->prob.r; a.KS = h->KS; a.mode = mode;
  a.gpart = h->gpart; a.U = h->U; a.Uprev = h->Uprev; a.Utmp = h->Utmp; a.ctl = h->ctl;
  a.eta_c = h->par.eta_c; a.power_tol = h->par.power_tol;
  a.colrr = h->colrr; a.colflags = h->colflags; a.q = h->prob.q;
  a.rlog = h->rlog; a.rlog_len = h->rlog_len;
  a.hi_max = h->par.bf16_hi_max;
  a.stall = h->par.bf16_stall;
  return a;
}

// The column and A_k U launches of a solve, through the autotuned variant when
// one was chosen for this problem's format.
hipError_t col_launch(const altgdmin_handle* h, int fmt, const ColArgs& a, hipStream_t st) {
  if (h->col_unroll > 0 && fmt == h->colfmt && a.waves == kWaves) return launch_col_tuned(fmt, h->col_unroll, a, st);
  // the FP32 default at two row chunks keeps one column per group in flight; when
  // its LDS leaves a CU three 4-wave workgroups instead of four (r >= 15 at m = 400)
  // two in flight win (1.16 against 1.42 ms at n = q = 1000, m = 400, r = 16)
  if (h->col_unroll == 0 && fmt == FMT_F32 && a.waves == kWaves && (a.m + 255) / 256 == 2 &&
      col_lds_bytes(a.n, a.m, a.r, a.rho, a.project, 0) > 160 * 1024 / 4)
    return launch_col_tuned(fmt, 2, a, st);
  return launch_col(fmt, a, st, h->col_unroll < 0 ? POL_CACHED : POL_STREAM);
}
hipError_t au_launch(const altgdmin_handle* h, int fmt, const AUArgs& a, hipStream_t st) {
  // the tuned depths are built for 4-wave workgroups
  if (h->au_depth > 0 && fmt == h->fmt && a.waves != 8) return launch_au_tuned(fmt, h->au_depth, a, st);
  return launch_au(fmt, a, st, h->au_depth < 0 ? POL_CACHED : POL_STREAM);
}

// ---- autotuner: the loads in flight of the two streaming kernels, per
// (A format, n, q, m, r, rho), chosen by timing the variants on the problem's own
// data; kept for the process and, with ALTGDMIN_TUNE_CACHE=<file>, in a JSON-lines
// file keyed by the GPU architecture.
using TuneKey = std::tuple<std::string, int, int, int, int, int, int>;
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tune;
bool g_tune_loaded = false;

std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

void tune_cache_load(const std::string& arch) {
  g_tune_loaded = true;
  const char* path = std::getenv("ALTGDMIN_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    char a[64] = {0};
    int fmt, n, q, m, r, rho, ju, aud;
    if (std::sscanf(line,
                    "{\"arch\": \"%63[^\"]\", \"fmt\": %d, \"n\": %d, \"q\": %d, \"m\": %d, \"r\": %d, "
                    "\"rho\": %d, \"col_unroll\": %d, \"au_depth\": %d",
                    a, &fmt, &n, &q, &m, &r, &rho, &ju, &aud) == 9 &&
        arch == a)
      g_tune[TuneKey(arch, fmt, n, q, m, r, rho)] = {ju, aud};
  }
  std::fclose(f);
}

void tune_cache_append(const TuneKey& k, int ju, int aud, float col_ms, float au_ms) {
  const char* path = std::getenv("ALTGDMIN_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f,
               "{\"arch\": \"%s\", \"fmt\": %d, \"n\": %d, \"q\": %d, \"m\": %d, \"r\": %d, \"rho\": %d, "
               "\"col_unroll\": %d, \"au_depth\": %d, \"col_ms\": %.4f, \"au_ms\": %.4f}\n",
               std::get<0>(k).c_str(), std::get<1>(k), std::get<2>(k), std::get<3>(k), std::get<4>(k), std::get<5>(k),
               std::get<6>(k), ju, aud, col_ms, au_ms);
  std::fclose(f);
}

ColArgs col_args(const altgdmin_handle* h);

// Load policy of A (the same bits either way): ordinary loads, which the 256 MB
// Infinity Cache keeps between the passes, when the plane the column passes
// stream fits in kCacheBudget; non-temporal loads otherwise.  The environment
// variable ALTGDMIN_LOAD_POLICY=stream|cached forces one.
constexpr size_t kCacheBudget = 200ull << 20;
size_t streamed_plane_bytes(const altgdmin_problem& p, int colfmt) {
  const size_t eb = colfmt == FMT_F32 || colfmt == FMT_BF16X2 ? 4 : colfmt == FMT_BF16MIX ? 2 : 0;
  return eb * (size_t)p.q * (size_t)p.n * (size_t)p.lda;
}
int load_policy(size_t bytes) {
  if (const char* f = std::getenv("ALTGDMIN_LOAD_POLICY")) {
    if (!std::strcmp(f, "stream")) return POL_STREAM;
    if (!std::strcmp(f, "cached")) return POL_CACHED;
  }
  return bytes > 0 && bytes <= kCacheBudget ? POL_CACHED : POL_STREAM;
}

int autotune(altgdmin_handle* h, hipStream_t st) {
  const altgdmin_problem& p = h->prob;
  // ALTGDMIN_TUNE_FORCE="JU,AUD" skips the timing and takes these variants (tests)
  if (const char* force = std::getenv("ALTGDMIN_TUNE_FORCE")) {
    int ju = 0, aud = 0;
    auto ok = [](int v) { return v == -1 || v == 1 || v == 2 || v == 4 || v == 8; };
    if (std::sscanf(force, "%d,%d", &ju, &aud) != 2 || !ok(ju) || !(ok(aud) || aud == 3))
      return fail(ALTGDMIN_EINVAL,
                  "ALTGDMIN_TUNE_FORCE must be JU,AUD with JU in {-1, 1, 2, 4, 8}, AUD in {-1, 1, 2, 3, 4, 8}");
    if (ju == 8 && p.m > 512) ju = 4;   // JU = 8 is built for at most two row chunks
    // the unrolls are built for 4-wave workgroups; -1 (the cached default) for every width
    h->col_unroll = ju < 0 || h->col_waves == kWaves ? ju : 0;
    h->au_depth = aud < 0 || au_waves(h->prob) == kWaves ? aud : 0;
    return ALTGDMIN_OK;
  }
  const std::string arch = device_arch();
  const TuneKey key(arch, h->colfmt, p.n, p.q, p.m, p.r, p.rho);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_loaded) tune_cache_load(arch);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      h->col_unroll = it->second.first;
      h->au_depth = it->second.second;
      return ALTGDMIN_OK;
    }
  }
  // the variants run on the problem's own A and y: A_k U from a fixed orthonormal
  // U, then the column kernel as in a GDmin iteration; every buffer they write
  // is rewritten by the initialisation or the first iteration
  HIPCHK(launch_fill_basis(h->Utmp, p.n, p.r, st));
  AUArgs au;
  std::memset(&au, 0, sizeof(au));
  au.n = p.n; au.q = p.q; au.m = p.m; au.r = p.r;
  au.A = p.A; au.Alo = p.A_lo; au.lda = p.lda; au.sA = p.a_stride_k;
  au.U = h->Utmp; au.P = h->P; au.Ginv = h->Ginv; au.flags = h->colflags;
  au.waves = au_waves(h->prob);
  // the column kernel in its GDmin configuration (projection by the P_k, G_k^{-1}
  // the A_k U runs just wrote, tau IHT iterations, the LS / gradient tail), from
  // an empty support
  ColArgs ca = col_args(h);
  ca.tau = h->par.tau; ca.project = 1; ca.has_support = 0; ca.tail = TAIL_LSGRAD;
  EventPair ev;
  HIPCHK(ev.create());
  hipEvent_t e0 = ev.e[0], e1 = ev.e[1];
  constexpr int kReps = 5;
  auto timed = [&](auto launch, float* ms) -> hipError_t {
    hipError_t e = launch();   // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int rep = 0; rep < kReps && e == hipSuccess; ++rep) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    *ms /= (float)kReps;
    return e;
  };
  // The default instantiation under the load policy's rule (0: streamed, -1:
  // cached) is timed first and kept unless a variant beats the best so far by
  // kMargin: the candidates run from an empty support, which is not the state of
  // the iterations they are picked for, so near-equal times are not a reason to
  // leave the default.  Candidates: the unrolls (4-wave column workgroups only)
  // and the A_k U depths.
  constexpr float kMargin = 0.02f;
  const bool cached = load_policy(streamed_plane_bytes(p, h->colfmt)) == POL_CACHED;
  const int base = cached ? -1 : 0;
  const int pol = cached ? POL_CACHED : POL_STREAM;
  int best_aud = base, best_ju = base;
  float best_au = 0.f, best_col = 0.f;
  hipError_t e = timed([&] { return launch_au(h->fmt, au, st, pol); }, &best_au);
  for (int aud : {1, 2, 3, 4, 8}) {
    if (e != hipSuccess || au.waves != kWaves) break;   // the tuned depths are built for 4 waves
    float ms = 0.f;
    e = timed([&] { return launch_au_tuned(h->fmt, aud, au, st); }, &ms);
    if (e != hipSuccess) break;
    if (ms < (1.f - kMargin) * best_au) { best_au = ms; best_aud = aud; }
  }
  if (e == hipSuccess) e = timed([&] { return launch_col(h->colfmt, ca, st, pol); }, &best_col);
  for (int ju : {1, 2, 4, 8}) {
    if (e != hipSuccess || h->col_waves != kWaves) break;
    float ms = 0.f;
    e = timed([&] { return launch_col_tuned(h->colfmt, ju, ca, st); }, &ms);
    if (e == hipErrorNotSupported) {   // no such instantiation for this row count: not a candidate
      e = hipSuccess;
      continue;
    }
    if (e != hipSuccess) break;
    if (ms < (1.f - kMargin) * best_col) { best_col = ms; best_ju = ju; }
  }
  if (e != hipSuccess) return fail(ALTGDMIN_EHIP, std::string("autotune: ") + hipGetErrorString(e));
  h->col_unroll = best_ju;
  h->au_depth = best_aud;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = {best_ju, best_aud};
  tune_cache_append(key, best_ju, best_aud, best_col, best_au);
  return ALTGDMIN_OK;
}

FColArgs fcol_args(const altgdmin_handle* h, int mode) {
  const altgdmin_problem& p = h->prob;
  FColArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = p.n; a.q = p.q; a.m = p.m; a.r = p.r; a.rho = p.rho;
  a.mode = mode;
  a.tau = mode == FCOL_GD ? h->par.tau : h->par.tau0;
  a.mask = p.fourier_mask;
  a.Y = static_cast<const float2*>(static_cast<const void*>(p.Y));
  a.ldy = p.ldy;
  a.FU = reinterpret_cast<const float2*>(h->FU);
  a.tw = reinterpret_cast<const float2*>(h->tw);
  a.n1 = p.n1;
  a.n2 = p.n2;
  a.Sidx = h->Tidx;
  a.Sval = reinterpret_cast<float2*>(h->Tval);
  a.Bt = reinterpret_cast<float2*>(h->Bt);
  a.H = reinterpret_cast<float2*>(h->H);
  a.colrr = h->colrr;
  a.flags = h->colflags;
  return a;
}

FQRArgs fqr_args(const altgdmin_handle* h, int mode) {
  FQRArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = h->prob.n; a.r = h->prob.r; a.q = h->prob.q; a.mode = mode;
  a.G = reinterpret_cast<const float2*>(h->gpart);
  a.U = reinterpret_cast<float2*>(h->U);
  a.Uprev = reinterpret_cast<float2*>(h->Uprev);
  a.Utmp = reinterpret_cast<float2*>(h->Utmp);
  a.ctl = h->ctl;
  a.eta_c = h->par.eta_c;
  a.power_tol = h->par.power_tol;
  a.colrr = h->colrr;
  a.colflags = h->colflags;
  a.rlog = h->rlog;
  a.rlog_len = h->rlog_len;
  a.part = reinterpret_cast<double2*>(h->fpart);
  a.rinv = reinterpret_cast<double2*>(h->frinv);
  a.nb = (h->prob.n + 255) / 256;
  return a;
}

#define F2(p) reinterpret_cast<float2*>(p)
#define CF2(p) reinterpret_cast<const float2*>(p)

// The four launches of one GDmin iteration of the partial Fourier form.
hipError_t fourier_launch(altgdmin_handle* h, int which, hipStream_t st) {
  const altgdmin_problem& p = h->prob;
  switch (which) {
    case 0:
      if (p.n1 == kFN && p.n2 == kFN) return launch_fu(CF2(h->U), p.r, CF2(h->tw), F2(h->FU), st);
      return launch_fu_gen(CF2(h->U), p.n, p.r, p.n1, p.n2, CF2(h->tw), F2(h->FU), st);
    case 1: return launch_fcol(fcol_args(h, FCOL_GD), st);
    case 2:
      return launch_fgrad_gd(CF2(h->H), CF2(h->Bt), CF2(h->U), p.n, p.q, p.r, F2(h->gpart),
                             reinterpret_cast<double2*>(h->fpart), nullptr, st);
    default: return launch_fqr_gd(fqr_args(h, QR_GD), st);
  }
}

// One GDmin iteration of Alg. 1 on stream st.
int enqueue_iteration(altgdmin_handle* h, hipStream_t st) {
  if (h->fmt == FMT_PFOURIER) {
    for (int w = 0; w < 4; ++w) HIPCHK(fourier_launch(h, w, st));
    return ALTGDMIN_OK;
  }
  const altgdmin_problem& p = h->prob;
  AUArgs au;
  au.n = p.n; au.q = p.q; au.m = p.m; au.r = p.r;
  au.A = p.A; au.Alo = p.A_lo; au.lda = p.lda; au.sA = p.a_stride_k;
  au.U = h->U; au.P = h->P; au.Ginv = h->Ginv; au.flags = h->colflags;
  au.gate = nullptr; au.gate_want = 0;
  au.seed = p.a_seed; au.table = p.normal_table;
  au.waves = au_waves(h->prob);
  ColArgs ca = col_args(h);
  ca.tau = h->par.tau; ca.project = 1; ca.has_support = 1; ca.tail = TAIL_LSGRAD;
  if (h->hi_phase) {
    // both variants are in the graph; the phase flag in the control block picks one
    au.gate = &h->ctl->phase; ca.gate = &h->ctl->phase;
    au.gate_want = 0; ca.gate_want = 0;
    HIPCHK(launch_au(FMT_BF16HI, au, st));
    HIPCHK(launch_col(FMT_BF16HI, ca, st));
    au.gate_want = 1; ca.gate_want = 1;
  }
  HIPCHK(au_launch(h, h->fmt, au, st));
  HIPCHK(col_launch(h, h->colfmt, ca, st));
  HIPCHK(launch_grad(h->H, h->Bt, p.n, p.q, p.r, h->KS, h->gpart, nullptr, st));
  HIPCHK(launch_qr(qr_args(h, QR_GD), st));
  return ALTGDMIN_OK;
}

}  // namespace

extern "C" {

void altgdmin_default_params(altgdmin_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->tau0 = 10;
  p->tau = 3;
  p->t_max = 200;
  p->power_iters = 100;
  p->poll_every = 10;
  p->eta_c = 0.14;
  p->power_tol = 1e-6;
  p->tol_resid = 0.0;
  p->bf16_hi_max = 0;
  p->bf16_stall = 0.9;
  p->rank_energy = 0.65;
  p->rank_iters = 30;
}

int altgdmin_workspace_bytes(const altgdmin_problem* prob, const altgdmin_params* par, size_t* bytes) {
  int rc = validate(prob, par);
  if (rc) return rc;
  if (!bytes) return fail(ALTGDMIN_EINVAL, "bytes is null");
  altgdmin_handle h;
  h.prob = *prob;
  h.par = *par;
  *bytes = carve(&h, nullptr);
  return ALTGDMIN_OK;
}

int altgdmin_init(const altgdmin_problem* prob, const altgdmin_params* par, void* workspace, size_t ws_bytes,
                  void* stream, altgdmin_handle** out) {
  int rc = validate(prob, par);
  if (rc) return rc;
  if (!workspace || !out) return fail(ALTGDMIN_EINVAL, "null workspace or out");
  NEED_STREAM(stream);
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0) return fail(ALTGDMIN_EINVAL, "workspace must be 256-byte aligned");
  altgdmin_handle* h = new altgdmin_handle();
  h->prob = *prob;
  h->par = *par;
  h->fmt = fmt_of(prob);
  h->hi_phase = (h->fmt == FMT_BF16X2 && par->bf16_hi_max > 0);
  h->colfmt = (par->flags & ALTGDMIN_FLAG_BF16_MIXED) ? FMT_BF16MIX : h->fmt;
  h->auto_rank = prob->r == 0;
  if (h->fmt != FMT_PFOURIER) {
    h->col_waves = choose_col_waves(h->prob, h->colfmt == FMT_BF16MIX);
    // a GDmin iteration's column workgroup (with P_k) may need more LDS than the
    // initialisation's: raise the kernels' limit now, before any graph capture
    if (col_lds_bytes(prob->n, prob->m, r_eff(*prob), prob->rho, 1, prob->a_format == ALTGDMIN_A_PHILOX,
                      h->col_waves) > kColLdsDefault) {
      const hipError_t le = col_allow_big_lds();
      if (le != hipSuccess) {
        delete h;
        return fail(ALTGDMIN_EHIP, std::string("column kernels' LDS limit: ") + hipGetErrorString(le));
      }
    }
    // the default instantiations with cached loads when the streamed plane fits in
    // the Infinity Cache (the autotuner, when on, times them against the unrolls)
    if (load_policy(streamed_plane_bytes(h->prob, h->colfmt)) == POL_CACHED) h->col_unroll = h->au_depth = -1;
  }
  const size_t need = carve(h, workspace);   // with r = 0, laid out for the largest rank the rule may pick
  const int r_cap = r_eff(h->prob);
  if (h->auto_rank) h->prob.r = r_cap;       // until the rank is chosen (the initialisation IHT does not use r)
  if (ws_bytes < need) {
    delete h;
    return fail(ALTGDMIN_ENOWS, "workspace too small: need " + std::to_string(need) + " bytes");
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const altgdmin_problem& p = h->prob;
  auto bail = [&](hipError_t e, const char* what) {
    delete h;
    return fail(ALTGDMIN_EHIP, std::string(what) + ": " + hipGetErrorString(e));
  };
  if ((par->flags & ALTGDMIN_FLAG_AUTOTUNE) && !h->hi_phase && !h->auto_rank &&
      (h->fmt == FMT_F32 || h->fmt == FMT_BF16X2)) {
    const int trc = autotune(h, st);
    if (trc) {
      delete h;
      return trc;
    }
  }
  hipError_t e;
  if ((e = launch_reset_ctl(h->ctl, 1, st)) != hipSuccess) return bail(e, "reset");
  if ((e = launch_set_phase(h->ctl, h->hi_phase ? 0 : 1, st)) != hipSuccess) return bail(e, "phase");
  if ((e = launch_fill_int(h->colflags, 0, p.q, st)) != hipSuccess) return bail(e, "flags");
  if (h->fmt == FMT_PFOURIER) {
    // s_k = IHT(y_k, A_k, rho, tau0, 0), L_0 = [A_k^H (y_k - A_k s_k)], U_0 by subspace iteration
    e = (p.n1 == kFN && p.n2 == kFN) ? launch_ftwiddle(F2(h->tw), st) : launch_ftwiddle_gen(F2(h->tw), p.n1, p.n2, st);
    if (e != hipSuccess) return bail(e, "twiddles");
    if ((e = launch_fcol(fcol_args(h, FCOL_INIT), st)) != hipSuccess) return bail(e, "init column kernel");
    if ((e = launch_sum_ctl(h->colrr, p.q, h->ctl, st)) != hipSuccess) return bail(e, "ynorm");
    if (h->auto_rank) {
      // r from the energy of the leading singular values of L_0 (Sec. 2.6), estimated on
      // its real embedding, where each value appears twice: the smallest k' of the
      // doubled sequence is 2r - 1 or 2r.  The only synchronisation of the initialisation.
      const RankShape rsh = rank_shape_complex(p.n, p.q, p.m);
      RankScratch rs = rank_scratch(h->rank_ws, rsh);
      float* block = nullptr;
      if ((e = launch_rank_embed(h->H, p.q, p.n, h->rank_embed, st)) != hipSuccess) return bail(e, "embedding");
      if ((e = enqueue_rank(h->rank_embed, rsh, par->rank_energy, par->rank_iters, rs, &block, st)) != hipSuccess)
        return bail(e, "automatic rank");
      int chosen2 = 0;
      if ((e = hipMemcpyAsync(&chosen2, rs.r, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess)
        return bail(e, "automatic rank copy");
      if ((e = hipStreamSynchronize(st)) != hipSuccess) return bail(e, "automatic rank");
      const int chosen = (chosen2 + 1) / 2;
      if (chosen < 1 || chosen > r_cap) {
        delete h;
        return fail(ALTGDMIN_ENOTBUILT, "automatic rank chose r = " + std::to_string(chosen) + ", above the " +
                                            std::to_string(r_cap) + " this problem is built for");
      }
      h->prob.r = chosen;
    }
    if (p.U_start && !h->auto_rank) e = launch_copy_f(h->Utmp, p.U_start, 2LL * p.n * p.r, st);
    else e = launch_fbasis(F2(h->Utmp), p.n, p.r, st);
    if (e != hipSuccess) return bail(e, "start block");
    if ((e = launch_fqr(fqr_args(h, QR_ORTH), st)) != hipSuccess) return bail(e, "orth");
    for (int it = 0; it < par->power_iters; ++it) {
      if ((e = launch_fltu(CF2(h->H), CF2(h->U), p.n, p.q, p.r, F2(h->Tpow), &h->ctl->conv, st)) != hipSuccess)
        return bail(e, "ltu");
      // L_0 (L_0^H U) with its per-block partial Grams, then CholeskyQR2 and the
      // subspace change over many workgroups
      if ((e = launch_fgrad_gd(CF2(h->H), CF2(h->Tpow), CF2(h->U), p.n, p.q, p.r, F2(h->gpart),
                               reinterpret_cast<double2*>(h->fpart), &h->ctl->conv, st)) != hipSuccess)
        return bail(e, "power grad");
      if ((e = launch_fqr_gd(fqr_args(h, QR_POWER), st)) != hipSuccess) return bail(e, "power qr");
    }
    if ((e = launch_reset_ctl(h->ctl, 0, st)) != hipSuccess) return bail(e, "reset eta");
    *out = h;
    return ALTGDMIN_OK;
  }
  // s_k = IHT(y_k, A_k, rho, tau0, 0) and L_0 columns A_k^T (y_k - A_k s_k); the
  // hi plane alone when a BF16X2 solve starts with a hi-only phase
  ColArgs ca = col_args(h);
  ca.tau = par->tau0; ca.project = 0; ca.has_support = 0; ca.tail = TAIL_BACKPROJ;
  if ((e = col_launch(h, h->hi_phase ? FMT_BF16HI : h->colfmt, ca, st)) != hipSuccess) return bail(e, "init column kernel");
  if ((e = launch_sum_ctl(h->colrr, p.q, h->ctl, st)) != hipSuccess) return bail(e, "ynorm");
  if (h->auto_rank) {
    // r from the energy of the leading singular values of L_0 (Sec. 2.6); the only
    // synchronisation of the initialisation.  U_0 starts from the first r columns of
    // the estimate's block, which span the first r columns' subspace iterate.
    RankScratch rs = rank_scratch(h->rank_ws, rank_shape(p.n, p.q, p.m));
    float* block = nullptr;
    if ((e = enqueue_rank(h->H, rank_shape(p.n, p.q, p.m), par->rank_energy, par->rank_iters, rs, &block, st)) !=
        hipSuccess)
      return bail(e, "automatic rank");
    int chosen = 0;
    if ((e = hipMemcpyAsync(&chosen, rs.r, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess)
      return bail(e, "automatic rank copy");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return bail(e, "automatic rank");
    if (chosen < 1 || chosen > r_cap) {
      delete h;
      return fail(ALTGDMIN_ENOTBUILT, "automatic rank chose r = " + std::to_string(chosen) + ", above the " +
                                          std::to_string(r_cap) + " this problem is built for");
    }
    h->prob.r = chosen;
    e = launch_rank_slice(block, p.n, rank_block(p.n, p.q, p.m), chosen, h->Utmp, st);
  } else if (p.U_start) {
    // U_0: top-r left singular subspace of L_0 by subspace iteration
    e = launch_copy_f(h->Utmp, p.U_start, (long long)p.n * p.r, st);
  } else {
    e = launch_fill_basis(h->Utmp, p.n, p.r, st);
  }
  if (e != hipSuccess) return bail(e, "start block");
  if ((e = launch_qr(qr_args(h, QR_ORTH), st)) != hipSuccess) return bail(e, "orth");
  for (int it = 0; it < par->power_iters; ++it) {
    if ((e = launch_ltu(h->H, h->U, p.n, p.q, p.r, h->Tpow, &h->ctl->conv, st)) != hipSuccess) return bail(e, "ltu");
    if ((e = launch_grad(h->H, h->Tpow, p.n, p.q, p.r, h->KS, h->gpart, &h->ctl->conv, st)) != hipSuccess)
      return bail(e, "power grad");
    if ((e = launch_qr(qr_args(h, QR_POWER), st)) != hipSuccess) return bail(e, "power qr");
  }
  if ((e = launch_reset_ctl(h->ctl, 0, st)) != hipSuccess) return bail(e, "reset eta");
  *out = h;
  return ALTGDMIN_OK;
}

int altgdmin_step(altgdmin_handle* h, int32_t iters, void* stream) {
  if (!h || iters < 0) return fail(ALTGDMIN_EINVAL, "null handle or negative iters");
  NEED_STREAM(stream);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (h->par.flags & ALTGDMIN_FLAG_EAGER) {   // eager launches (no graph)
    for (int i = 0; i < iters; ++i) {
      int rc = enqueue_iteration(h, st);
      if (rc) return rc;
    }
    h->t_host += iters;
    return ALTGDMIN_OK;
  }
  if (!h->have_graph) {
    hipStream_t cs;
    HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_iteration(h, cs);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (rc || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      if (rc) return rc;
      return fail(ALTGDMIN_EHIP, std::string("capture: ") + hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&h->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      h->exec = nullptr;
      return fail(ALTGDMIN_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    h->graph = g;
    h->have_graph = true;
  }
  for (int i = 0; i < iters; ++i) HIPCHK(hipGraphLaunch(h->exec, st));
  h->t_host += iters;
  return ALTGDMIN_OK;
}

int altgdmin_profile_iteration(altgdmin_handle* h, int32_t iters, void* stream, double* ms_out) {
  if (!h || iters < 1 || !ms_out) return fail(ALTGDMIN_EINVAL, "bad profile arguments");
  NEED_STREAM(stream);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const altgdmin_problem& p = h->prob;
  EventPair evp[3];
  for (int i = 0; i < 3; ++i) HIPCHK(evp[i].create());
  const hipEvent_t ev[5] = {evp[0].e[0], evp[0].e[1], evp[1].e[0], evp[1].e[1], evp[2].e[0]};
  double acc[4] = {0, 0, 0, 0};
  int rc = ALTGDMIN_OK;
  for (int it = 0; it < iters && rc == ALTGDMIN_OK && h->fmt == FMT_PFOURIER; ++it) {
    hipError_t e = hipSuccess;
    for (int w = 0; w < 4 && e == hipSuccess; ++w) {
      e = hipEventRecord(ev[w], st);
      if (e == hipSuccess) e = fourier_launch(h, w, st);
    }
    if (e == hipSuccess) e = hipEventRecord(ev[4], st);
    if (e == hipSuccess) e = hipEventSynchronize(ev[4]);
    for (int k = 0; k < 4 && e == hipSuccess; ++k) {
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
      acc[k] += ms;
    }
    if (e != hipSuccess) rc = fail(ALTGDMIN_EHIP, std::string("profile: ") + hipGetErrorString(e));
  }
  for (int it = 0; it < iters && rc == ALTGDMIN_OK && h->fmt != FMT_PFOURIER; ++it) {
    AUArgs au;
    au.n = p.n; au.q = p.q; au.m = p.m; au.r = p.r;
    au.A = p.A; au.Alo = p.A_lo; au.lda = p.lda; au.sA = p.a_stride_k;
    au.U = h->U; au.P = h->P; au.Ginv = h->Ginv; au.flags = h->colflags;
    au.gate = nullptr; au.gate_want = 0;
    au.seed = p.a_seed; au.table = p.normal_table;
    au.waves = au_waves(h->prob);
    ColArgs ca = col_args(h);
    ca.tau = h->par.tau; ca.project = 1; ca.has_support = 1; ca.tail = TAIL_LSGRAD;
    hipError_t e = hipEventRecord(ev[0], st);
    if (e == hipSuccess) e = au_launch(h, h->fmt, au, st);
    if (e == hipSuccess) e = hipEventRecord(ev[1], st);
    if (e == hipSuccess) e = col_launch(h, h->colfmt, ca, st);
    if (e == hipSuccess) e = hipEventRecord(ev[2], st);
    if (e == hipSuccess) e = launch_grad(h->H, h->Bt, p.n, p.q, p.r, h->KS, h->gpart, nullptr, st);
    if (e == hipSuccess) e = hipEventRecord(ev[3], st);
    if (e == hipSuccess) e = launch_qr(qr_args(h, QR_GD), st);
    if (e == hipSuccess) e = hipEventRecord(ev[4], st);
    if (e == hipSuccess) e = hipEventSynchronize(ev[4]);
    for (int k = 0; k < 4 && e == hipSuccess; ++k) {
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
      acc[k] += ms;
    }
    if (e != hipSuccess) rc = fail(ALTGDMIN_EHIP, std::string("profile: ") + hipGetErrorString(e));
  }
  if (rc) return rc;
  for (int k = 0; k < 4; ++k) ms_out[k] = acc[k] / iters;
  h->t_host += iters;
  return ALTGDMIN_OK;
}

int altgdmin_get(altgdmin_handle* h, float* U, float* Bt, int32_t* S_idx, float* S_val, float* U_next,
                 void* stream) {
  if (!h) return fail(ALTGDMIN_EINVAL, "null handle");
  NEED_STREAM(stream);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const altgdmin_problem& p = h->prob;
  const size_t nr = (size_t)p.n * p.r;
  const size_t w = h->fmt == FMT_PFOURIER ? 8 : 4;   // bytes per value: complex64 in the Fourier form
  if (U) HIPCHK(hipMemcpyAsync(U, h->t_host > 0 ? h->Uprev : h->U, nr * w, hipMemcpyDeviceToDevice, st));
  if (U_next) HIPCHK(hipMemcpyAsync(U_next, h->U, nr * w, hipMemcpyDeviceToDevice, st));
  if (Bt) HIPCHK(hipMemcpyAsync(Bt, h->Bt, (size_t)p.q * p.r * w, hipMemcpyDeviceToDevice, st));
  if (S_idx && p.rho > 0) HIPCHK(hipMemcpyAsync(S_idx, h->Tidx, (size_t)p.q * p.rho * 4, hipMemcpyDeviceToDevice, st));
  if (S_val && p.rho > 0) HIPCHK(hipMemcpyAsync(S_val, h->Tval, (size_t)p.q * p.rho * w, hipMemcpyDeviceToDevice, st));
  return ALTGDMIN_OK;
}

int altgdmin_status(altgdmin_handle* h, void* stream, altgdmin_report* rep) {
  if (!h || !rep) return fail(ALTGDMIN_EINVAL, "null handle or report");
  NEED_STREAM(stream);
  hipStream_t st = static_cast<hipStream_t>(stream);
  Ctl c;
  HIPCHK(hipMemcpyAsync(&c, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  rep->iterations = c.t;
  rep->power_iterations = c.power_it;
  rep->error_flags = c.err;
  rep->eta = c.eta;
  rep->resid = c.resid;
  rep->power_sd = c.power_sd;
  rep->converged = (h->par.tol_resid > 0.0 && c.t > 0 && c.err == 0 && c.resid <= h->par.tol_resid) ? 1 : 0;
  rep->refine_iteration = h->hi_phase ? c.refine_t : -1;
  rep->rank = h->prob.r;
  return ALTGDMIN_OK;
}

int altgdmin_status_many(altgdmin_handle* const* hs, int32_t count, void* stream, altgdmin_report* reps) {
  if (!hs || count < 0 || (count > 0 && !reps)) return fail(ALTGDMIN_EINVAL, "bad status_many arguments");
  NEED_STREAM(stream);
  for (int i = 0; i < count; ++i)
    if (!hs[i]) return fail(ALTGDMIN_EINVAL, "null handle");
  if (count == 0) return ALTGDMIN_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  std::vector<Ctl> c(count);
  for (int i = 0; i < count; ++i) HIPCHK(hipMemcpyAsync(&c[i], hs[i]->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int i = 0; i < count; ++i) {
    const altgdmin_handle* h = hs[i];
    altgdmin_report* rep = &reps[i];
    rep->iterations = c[i].t;
    rep->power_iterations = c[i].power_it;
    rep->error_flags = c[i].err;
    rep->eta = c[i].eta;
    rep->resid = c[i].resid;
    rep->power_sd = c[i].power_sd;
    rep->converged = (h->par.tol_resid > 0.0 && c[i].t > 0 && c[i].err == 0 && c[i].resid <= h->par.tol_resid) ? 1 : 0;
    rep->refine_iteration = h->hi_phase ? c[i].refine_t : -1;
    rep->rank = h->prob.r;
  }
  return ALTGDMIN_OK;
}

int altgdmin_residual_log(altgdmin_handle* h, void* stream, double* host_log, int32_t* count) {
  if (!h || !host_log || !count) return fail(ALTGDMIN_EINVAL, "null argument");
  altgdmin_report rep;
  int rc = altgdmin_status(h, stream, &rep);
  if (rc) return rc;
  const int cnt = rep.iterations < h->rlog_len ? rep.iterations : h->rlog_len;
  if (cnt > 0) {
    hipStream_t st = static_cast<hipStream_t>(stream);
    HIPCHK(hipMemcpyAsync(host_log, h->rlog, (size_t)cnt * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  *count = cnt;
  return ALTGDMIN_OK;
}

int altgdmin_destroy(altgdmin_handle* h) {
  if (!h) return ALTGDMIN_OK;
  if (h->exec) (void)hipGraphExecDestroy(h->exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  delete h;
  return ALTGDMIN_OK;
}

int altgdmin_solve(const altgdmin_problem* prob, const altgdmin_params* par, void* workspace, size_t ws_bytes,
                   void* stream, float* U, float* Bt, int32_t* S_idx, float* S_val, altgdmin_report* rep) {
  altgdmin_handle* h = nullptr;
  int rc = altgdmin_init(prob, par, workspace, ws_bytes, stream, &h);
  if (rc) return rc;
  altgdmin_report r;
  std::memset(&r, 0, sizeof(r));
  int done = 0;
  bool conv = false;
  while (done < par->t_max) {
    const int k = (par->t_max - done) < par->poll_every ? (par->t_max - done) : par->poll_every;
    rc = altgdmin_step(h, k, stream);
    if (rc) { altgdmin_destroy(h); return rc; }
    done += k;
    if (par->tol_resid > 0.0) {
      rc = altgdmin_status(h, stream, &r);
      if (rc) { altgdmin_destroy(h); return rc; }
      if (r.error_flags) break;
      if (r.converged) { conv = true; break; }
    }
  }
  rc = altgdmin_get(h, U, Bt, S_idx, S_val, nullptr, stream);
  if (!rc) rc = altgdmin_status(h, stream, &r);
  altgdmin_destroy(h);
  if (rc) return rc;
  if (rep) *rep = r;
  if (r.error_flags) return fail(ALTGDMIN_ENONFINITE, "non-finite value or indefinite Gram matrix during the solve");
  if (par->tol_resid > 0.0 && !conv) return ALTGDMIN_ENOTCONV;
  return ALTGDMIN_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ checkpoint / resume

namespace {

constexpr long long kStateMagic = 0x3130545347544C41LL;   // "ALTGST01"

// A saved state: header words, the control block, U, U_prev (the U that B and S
// were fitted with), B^T, the support indices and values, the column flags and
// the residual log, each block at 256-byte alignment.
struct StateLayout {
  size_t hdr, ctl, U, Uprev, Bt, Tidx, Tval, flags, rlog, total;
};

StateLayout state_layout(const altgdmin_handle* h, int rlog_len) {
  const altgdmin_problem& p = h->prob;
  const size_t w = h->fmt == FMT_PFOURIER ? 8 : 4;   // bytes per value (complex64 in the Fourier form)
  const size_t nr = (size_t)p.n * p.r, qr = (size_t)p.q * p.r, qs = (size_t)p.q * p.rho;
  StateLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    o = (o + kAlign - 1) / kAlign * kAlign;
    const size_t at = o;
    o += bytes;
    return at;
  };
  L.hdr = take(kStateWords * sizeof(long long));
  L.ctl = take(sizeof(Ctl));
  L.U = take(nr * w);
  L.Uprev = take(nr * w);
  L.Bt = take(qr * w);
  L.Tidx = take(qs * sizeof(int));
  L.Tval = take(qs * w);
  L.flags = take((size_t)p.q * sizeof(int));
  L.rlog = take((size_t)rlog_len * sizeof(double));
  L.total = (o + kAlign - 1) / kAlign * kAlign;
  return L;
}

}  // namespace

extern "C" {

int altgdmin_state_bytes(altgdmin_handle* h, size_t* bytes) {
  if (!h || !bytes) return fail(ALTGDMIN_EINVAL, "null handle or bytes");
  *bytes = state_layout(h, h->rlog_len).total;
  return ALTGDMIN_OK;
}

int altgdmin_get_state(altgdmin_handle* h, void* state, size_t bytes, void* stream) {
  if (!h || !state) return fail(ALTGDMIN_EINVAL, "null handle or state");
  NEED_STREAM(stream);
  if (reinterpret_cast<uintptr_t>(state) % kAlign != 0) return fail(ALTGDMIN_EINVAL, "state must be 256-byte aligned");
  const StateLayout L = state_layout(h, h->rlog_len);
  if (bytes < L.total) return fail(ALTGDMIN_ENOWS, "state buffer too small: need " + std::to_string(L.total));
  hipStream_t st = static_cast<hipStream_t>(stream);
  const altgdmin_problem& p = h->prob;
  const size_t w = h->fmt == FMT_PFOURIER ? 8 : 4;
  char* d = static_cast<char*>(state);
  StateWords hw;
  std::memset(&hw, 0, sizeof(hw));
  const long long words[] = {kStateMagic, p.n, p.q, p.m, p.r, p.rho, p.a_format, h->colfmt, h->t_host,
                             h->rlog_len, (long long)L.total};
  std::memcpy(hw.v, words, sizeof(words));
  HIPCHK(launch_put_words(reinterpret_cast<long long*>(d + L.hdr), hw, st));
  auto cp = [&](size_t off, const void* src, size_t n) {
    return n ? hipMemcpyAsync(d + off, src, n, hipMemcpyDeviceToDevice, st) : hipSuccess;
  };
  const size_t nr = (size_t)p.n * p.r;
  HIPCHK(cp(L.ctl, h->ctl, sizeof(Ctl)));
  HIPCHK(cp(L.U, h->U, nr * w));
  HIPCHK(cp(L.Uprev, h->Uprev, nr * w));
  HIPCHK(cp(L.Bt, h->Bt, (size_t)p.q * p.r * w));
  HIPCHK(cp(L.Tidx, h->Tidx, (size_t)p.q * p.rho * sizeof(int)));
  HIPCHK(cp(L.Tval, h->Tval, (size_t)p.q * p.rho * w));
  HIPCHK(cp(L.flags, h->colflags, (size_t)p.q * sizeof(int)));
  HIPCHK(cp(L.rlog, h->rlog, (size_t)h->rlog_len * sizeof(double)));
  return ALTGDMIN_OK;
}

int altgdmin_set_state(altgdmin_handle* h, const void* state, size_t bytes, void* stream) {
  if (!h || !state) return fail(ALTGDMIN_EINVAL, "null handle or state");
  NEED_STREAM(stream);
  if (reinterpret_cast<uintptr_t>(state) % kAlign != 0) return fail(ALTGDMIN_EINVAL, "state must be 256-byte aligned");
  if (bytes < kStateWords * sizeof(long long)) return fail(ALTGDMIN_EINVAL, "state buffer too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const char* d = static_cast<const char*>(state);
  long long hw[kStateWords];
  HIPCHK(hipMemcpyAsync(hw, d, sizeof(hw), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const altgdmin_problem& p = h->prob;
  if (hw[0] != kStateMagic) return fail(ALTGDMIN_EINVAL, "not a saved solver state");
  if (hw[1] != p.n || hw[2] != p.q || hw[3] != p.m || hw[4] != p.r || hw[5] != p.rho || hw[6] != p.a_format ||
      hw[7] != h->colfmt)
    return fail(ALTGDMIN_EINVAL, "saved state is of another problem size or A form");
  const int saved_len = (int)hw[9];
  const StateLayout L = state_layout(h, saved_len);
  if (hw[10] != (long long)L.total || bytes < L.total) return fail(ALTGDMIN_EINVAL, "saved state has an unexpected size");
  const size_t w = h->fmt == FMT_PFOURIER ? 8 : 4;
  auto cp = [&](void* dst, size_t off, size_t n) {
    return n ? hipMemcpyAsync(dst, d + off, n, hipMemcpyDeviceToDevice, st) : hipSuccess;
  };
  const size_t nr = (size_t)p.n * p.r;
  HIPCHK(cp(h->ctl, L.ctl, sizeof(Ctl)));
  HIPCHK(cp(h->U, L.U, nr * w));
  HIPCHK(cp(h->Uprev, L.Uprev, nr * w));
  HIPCHK(cp(h->Bt, L.Bt, (size_t)p.q * p.r * w));
  HIPCHK(cp(h->Tidx, L.Tidx, (size_t)p.q * p.rho * sizeof(int)));
  HIPCHK(cp(h->Tval, L.Tval, (size_t)p.q * p.rho * w));
  HIPCHK(cp(h->colflags, L.flags, (size_t)p.q * sizeof(int)));
  HIPCHK(cp(h->rlog, L.rlog, (size_t)std::min(saved_len, h->rlog_len) * sizeof(double)));
  // the support is the iteration's warm start: a column that is not rho distinct
  // in-range ascending indices is flagged and restarts from s = 0
  HIPCHK(launch_check_support(h->Tidx, h->Tval, h->fmt == FMT_PFOURIER ? 2 : 1, p.q, p.rho, p.n, h->colflags, st));
  h->t_host = (int)hw[8];
  return ALTGDMIN_OK;
}

const char* altgdmin_strerror(int code) {
  switch (code) {
    case ALTGDMIN_OK: return "ok";
    case ALTGDMIN_ENOTCONV: return "t_max reached before tol_resid";
    case ALTGDMIN_EINVAL: return "invalid argument";
    case ALTGDMIN_ENOWS: return "workspace too small";
    case ALTGDMIN_EHIP: return "HIP runtime error";
    case ALTGDMIN_ENONFINITE: return "non-finite value or indefinite Gram matrix";
    case ALTGDMIN_ENOTBUILT: return "no kernel instantiation for these sizes";
    default: return "unknown error";
  }
}

const char* altgdmin_last_error(void) { return g_last_error.c_str(); }

int altgdmin_tuning(altgdmin_handle* h, int32_t* col_unroll, int32_t* au_depth) {
  if (!h) return fail(ALTGDMIN_EINVAL, "null handle");
  if (col_unroll) *col_unroll = h->col_unroll;
  if (au_depth) *au_depth = h->au_depth;
  return ALTGDMIN_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ serving: batched iterations

namespace {

// Launch buckets of a group: problems of one A format whose column kernels share
// an instantiation (NC = ceil(m / 256) for the column kernel, R = r rounded up to
// even for the A_k U kernel), so no problem runs a wider instantiation than its own.
struct Bucket {
  int fmt, inst, waves = kWaves;
  std::vector<int2> map;
  size_t lds = 0, off = 0;
};

struct GroupPlan {
  std::vector<AUArgs> au;
  std::vector<ColArgs> col;
  std::vector<GradArgs> grad;
  std::vector<QRArgs> qr;
  std::map<int, Bucket> au_b, col_b;   // key fmt * 64 + inst
  std::vector<int4> grad_map;
  size_t qr_lds = 0;
  // byte offsets in the group workspace
  size_t o_au, o_col, o_grad, o_qr, o_gm, total;
};

int plan_group(altgdmin_handle* const* hs, int count, GroupPlan& g) {
  if (!hs || count < 1) return fail(ALTGDMIN_EINVAL, "no handles");
  for (int i = 0; i < count; ++i) {
    altgdmin_handle* h = hs[i];
    if (!h) return fail(ALTGDMIN_EINVAL, "null handle");
    if (h->hi_phase) return fail(ALTGDMIN_EINVAL, "a BF16X2 problem with a hi-only phase cannot be batched");
    if (h->fmt == FMT_PFOURIER) return fail(ALTGDMIN_EINVAL, "batched stepping takes the real A formats only");
    const altgdmin_problem& p = h->prob;
    AUArgs au;
    std::memset(&au, 0, sizeof(au));
    au.n = p.n; au.q = p.q; au.m = p.m; au.r = p.r;
    au.A = p.A; au.Alo = p.A_lo; au.lda = p.lda; au.sA = p.a_stride_k;
    au.U = h->U; au.P = h->P; au.Ginv = h->Ginv; au.flags = h->colflags;
    au.seed = p.a_seed; au.table = p.normal_table;
    au.waves = au_waves(h->prob);
    // with tol_resid > 0 a problem whose residual reached it is frozen (every kernel skips it)
    const int* done = h->par.tol_resid > 0.0 ? &h->ctl->done : nullptr;
    au.gate = done; au.gate_want = 0;
    g.au.push_back(au);
    ColArgs ca = col_args(h);
    ca.tau = h->par.tau; ca.project = 1; ca.has_support = 1; ca.tail = TAIL_LSGRAD;
    ca.gate = done; ca.gate_want = 0;
    g.col.push_back(ca);
    GradArgs ga;
    ga.H = h->H; ga.B = h->Bt; ga.n = p.n; ga.q = p.q; ga.r = p.r; ga.KS = h->KS; ga.gpart = h->gpart;
    ga.skip = done;
    g.grad.push_back(ga);
    QRArgs qa = qr_args(h, QR_GD);
    qa.tol = h->par.tol_resid;
    qa.gate_done = done ? 1 : 0;
    qa.lds = (size_t)p.n * p.r * sizeof(float) <= kQRLdsMax ? 1 : 0;
    if (qa.lds) g.qr_lds = std::max(g.qr_lds, (size_t)p.n * p.r * sizeof(float));
    g.qr.push_back(qa);
    const int f = h->fmt, cf = h->colfmt, phx = f == FMT_PHILOX;
    const int nc = (p.m + 255) / 256, rr = (p.r + 1) / 2 * 2, cw = h->col_waves;
    const int aw = au_waves(p);
    Bucket& ab = g.au_b[(f * 64 + rr) * 32 + aw];   // and with others of their A_k U width
    Bucket& cb = g.col_b[(cf * 64 + nc) * 32 + cw];   // problems batch with others of their column width
    ab.fmt = f;
    cb.fmt = cf;
    ab.inst = rr;
    ab.waves = aw;
    cb.inst = nc;
    cb.waves = cw;
    for (int k = 0; k < p.q; ++k) {
      ab.map.push_back(make_int2(i, k));
      cb.map.push_back(make_int2(i, k));
    }
    for (int jb = 0; jb < (p.n + 63) / 64; ++jb)
      for (int ks = 0; ks < h->KS; ++ks) g.grad_map.push_back(make_int4(i, jb, ks, 0));
    ab.lds = std::max(ab.lds, AULayout(p.m, p.r, phx, aw).total);
    cb.lds = std::max(cb.lds, ColLayout(p.n, p.m, p.r, p.rho, 1, phx, cw).total);
  }
  size_t o = 0;
  auto take = [&](size_t bytes) { o = (o + kAlign - 1) / kAlign * kAlign; size_t r = o; o += bytes; return r; };
  g.o_au = take(g.au.size() * sizeof(AUArgs));
  g.o_col = take(g.col.size() * sizeof(ColArgs));
  g.o_grad = take(g.grad.size() * sizeof(GradArgs));
  g.o_qr = take(g.qr.size() * sizeof(QRArgs));
  for (auto& kv : g.au_b) kv.second.off = take(kv.second.map.size() * sizeof(int2));
  for (auto& kv : g.col_b) kv.second.off = take(kv.second.map.size() * sizeof(int2));
  g.o_gm = take(g.grad_map.size() * sizeof(int4));
  g.total = (o + kAlign - 1) / kAlign * kAlign;
  return ALTGDMIN_OK;
}

// Host staging of the launch tables of altgdmin_step_many: a pinned host buffer
// that the library keeps (grown as needed) and an event marking when the last
// upload from it finished, so an upload needs no stream synchronisation (only a
// wait for the previous upload, normally long done, before the buffer is reused).
struct Staging {
  std::mutex mu;
  char* host = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
};
Staging g_stage;

int upload_tables(const std::vector<char>& buf, void* dev, hipStream_t st) {
  std::lock_guard<std::mutex> lk(g_stage.mu);
  if (!g_stage.done) HIPCHK(hipEventCreateWithFlags(&g_stage.done, hipEventDisableTiming));
  if (g_stage.pending) {   // the previous upload still reads the staging buffer
    HIPCHK(hipEventSynchronize(g_stage.done));
    g_stage.pending = false;
  }
  if (g_stage.cap < buf.size()) {
    if (g_stage.host) HIPCHK(hipHostFree(g_stage.host));
    g_stage.host = nullptr;
    g_stage.cap = 0;
    HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&g_stage.host), buf.size(), hipHostMallocDefault));
    g_stage.cap = buf.size();
  }
  std::memcpy(g_stage.host, buf.data(), buf.size());
  HIPCHK(hipMemcpyAsync(dev, g_stage.host, buf.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipEventRecord(g_stage.done, st));
  g_stage.pending = true;
  return ALTGDMIN_OK;
}

}  // namespace

extern "C" {

int altgdmin_group_bytes(altgdmin_handle* const* hs, int32_t count, size_t* bytes) {
  if (!bytes) return fail(ALTGDMIN_EINVAL, "bytes is null");
  GroupPlan g;
  int rc = plan_group(hs, count, g);
  if (rc) return rc;
  *bytes = g.total;
  return ALTGDMIN_OK;
}

int altgdmin_step_many(altgdmin_handle* const* hs, int32_t count, int32_t iters, void* group_ws, size_t group_bytes,
                       void* stream) {
  if (iters < 0 || !group_ws || reinterpret_cast<uintptr_t>(group_ws) % kAlign != 0)
    return fail(ALTGDMIN_EINVAL, "bad step_many arguments");
  NEED_STREAM(stream);
  GroupPlan g;
  int rc = plan_group(hs, count, g);
  if (rc) return rc;
  if (group_bytes < g.total) return fail(ALTGDMIN_ENOWS, "group workspace too small: need " + std::to_string(g.total));
  for (const auto& kv : g.au_b)
    if (kv.second.lds > kMaxLds) return fail(ALTGDMIN_ENOTBUILT, "group needs too much LDS");
  for (const auto& kv : g.col_b)
    if (kv.second.lds > kColLdsMax) return fail(ALTGDMIN_ENOTBUILT, "group needs too much LDS");
  std::vector<char> buf(g.total, 0);
  auto put = [&](size_t off, const void* src, size_t bytes) { if (bytes) std::memcpy(buf.data() + off, src, bytes); };
  put(g.o_au, g.au.data(), g.au.size() * sizeof(AUArgs));
  put(g.o_col, g.col.data(), g.col.size() * sizeof(ColArgs));
  put(g.o_grad, g.grad.data(), g.grad.size() * sizeof(GradArgs));
  put(g.o_qr, g.qr.data(), g.qr.size() * sizeof(QRArgs));
  for (const auto& kv : g.au_b) put(kv.second.off, kv.second.map.data(), kv.second.map.size() * sizeof(int2));
  for (const auto& kv : g.col_b) put(kv.second.off, kv.second.map.data(), kv.second.map.size() * sizeof(int2));
  put(g.o_gm, g.grad_map.data(), g.grad_map.size() * sizeof(int4));
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* dev = static_cast<char*>(group_ws);
  rc = upload_tables(buf, dev, st);
  if (rc) return rc;
  const AUArgs* au_tab = reinterpret_cast<const AUArgs*>(dev + g.o_au);
  const ColArgs* col_tab = reinterpret_cast<const ColArgs*>(dev + g.o_col);
  const GradArgs* grad_tab = reinterpret_cast<const GradArgs*>(dev + g.o_grad);
  const QRArgs* qr_tab = reinterpret_cast<const QRArgs*>(dev + g.o_qr);
  // one load policy for the round: cached loads when the planes streamed by all
  // the problems together fit in the Infinity Cache
  size_t plane_bytes = 0;
  for (int i = 0; i < count; ++i)
    if (hs[i]->fmt != FMT_PFOURIER) plane_bytes += streamed_plane_bytes(hs[i]->prob, hs[i]->colfmt);
  const int pol = load_policy(plane_bytes);
  for (int it = 0; it < iters; ++it) {
    for (const auto& kv : g.au_b) {
      const Bucket& b = kv.second;
      HIPCHK(launch_au_grp(b.fmt, b.inst, b.waves, au_tab, reinterpret_cast<const int2*>(dev + b.off), (int)b.map.size(),
                           b.lds, st, pol));
    }
    for (const auto& kv : g.col_b) {
      const Bucket& b = kv.second;
      HIPCHK(launch_col_grp(b.fmt, b.inst, b.waves, col_tab, reinterpret_cast<const int2*>(dev + b.off),
                            (int)b.map.size(), b.lds, st, pol));
    }
    HIPCHK(launch_grad_grp(grad_tab, reinterpret_cast<const int4*>(dev + g.o_gm), (int)g.grad_map.size(), st));
    HIPCHK(launch_qr_grp(qr_tab, count, g.qr_lds, st));
  }
  for (int i = 0; i < count; ++i) hs[i]->t_host += iters;
  return ALTGDMIN_OK;
}

}  // extern "C"

extern "C" {

// ------------------------------------------------------------------ step-level entry points

int altgdmin_op_select(const float* V, int32_t n, int32_t count, int64_t ldv, int32_t rho, int32_t* idx,
                       float* val, int32_t* flags, void* stream) {
  if (!V || n < 1 || count < 0 || ldv < n || rho < 0 || rho > n) return fail(ALTGDMIN_EINVAL, "bad select arguments");
  if (rho > 0 && (!idx || !val)) return fail(ALTGDMIN_EINVAL, "null idx/val");
  if (select_lds_bytes(n, rho) > kMaxLds) return fail(ALTGDMIN_ENOTBUILT, "n too large for the select kernel");
  NEED_STREAM(stream);
  if (count == 0) return ALTGDMIN_OK;
  HIPCHK(launch_select(V, n, count, ldv, rho, idx, val, flags, static_cast<hipStream_t>(stream)));
  return ALTGDMIN_OK;
}

int altgdmin_op_au(const altgdmin_problem* prob, const float* U, float* P, double* Lc, int32_t* flags,
                   void* stream) {
  altgdmin_params par;
  altgdmin_default_params(&par);
  int rc = validate(prob, &par);
  if (rc) return rc;
  if (!U || !P || !Lc) return fail(ALTGDMIN_EINVAL, "null U/P/Ginv");
  NEED_STREAM(stream);
  AUArgs au;
  au.n = prob->n; au.q = prob->q; au.m = prob->m; au.r = prob->r;
  au.A = prob->A; au.Alo = prob->A_lo; au.lda = prob->lda; au.sA = prob->a_stride_k;
  au.U = U; au.P = P; au.Ginv = Lc; au.flags = flags;
  au.gate = nullptr; au.gate_want = 0;
  au.seed = prob->a_seed; au.table = prob->normal_table;
  au.waves = au_waves(*prob);   // the width the solver takes for this problem
  HIPCHK(launch_au(fmt_of(prob), au, static_cast<hipStream_t>(stream)));
  return ALTGDMIN_OK;
}

static int op_col(const altgdmin_problem* prob, ColArgs& a, void* stream) {
  NEED_STREAM(stream);
  a.waves = choose_col_waves(*prob, false);   // the width the solver takes for this problem
  a.n = prob->n; a.q = prob->q; a.m = prob->m; a.r = prob->r; a.rho = prob->rho;
  a.seed = prob->a_seed; a.table = prob->normal_table;
  a.A = prob->A; a.Alo = prob->A_lo; a.lda = prob->lda; a.sA = prob->a_stride_k;
  a.Y = prob->Y; a.ldy = prob->ldy;
  HIPCHK(launch_col(fmt_of(prob), a, static_cast<hipStream_t>(stream)));
  return ALTGDMIN_OK;
}

int altgdmin_op_iht(const altgdmin_problem* prob, int32_t project, const float* P, const double* Lc, int32_t tau,
                    int32_t has_support, int32_t* S_idx, float* S_val, float* G_out, double* mu_out,
                    int32_t* flags, void* stream) {
  altgdmin_params par;
  altgdmin_default_params(&par);
  int rc = validate(prob, &par);
  if (rc) return rc;
  if (tau < 0 || (project && (!P || !Lc)) || (prob->rho > 0 && (!S_idx || !S_val)))
    return fail(ALTGDMIN_EINVAL, "bad iht arguments");
  ColArgs a;
  std::memset(&a, 0, sizeof(a));
  a.P = P; a.Ginv = Lc; a.Tidx = S_idx; a.Tval = S_val; a.G_out = G_out; a.mu_out = mu_out; a.flags = flags;
  a.tau = tau; a.project = project ? 1 : 0; a.has_support = has_support ? 1 : 0; a.tail = TAIL_NONE;
  return op_col(prob, a, stream);
}

int altgdmin_op_lsgrad(const altgdmin_problem* prob, const float* P, const double* Lc, const int32_t* S_idx,
                       const float* S_val, float* Bt, float* H, double* rr, int32_t* flags, void* stream) {
  altgdmin_params par;
  altgdmin_default_params(&par);
  int rc = validate(prob, &par);
  if (rc) return rc;
  if (!P || !Lc || !Bt || !H || (prob->rho > 0 && (!S_idx || !S_val))) return fail(ALTGDMIN_EINVAL, "bad lsgrad arguments");
  ColArgs a;
  std::memset(&a, 0, sizeof(a));
  // the kernel writes the support back; it is unchanged with tau = 0
  a.P = P; a.Ginv = Lc; a.Tidx = const_cast<int32_t*>(S_idx); a.Tval = const_cast<float*>(S_val);
  a.Bt = Bt; a.H = H; a.rr = rr; a.flags = flags;
  a.tau = 0; a.project = 1; a.has_support = 1; a.tail = TAIL_LSGRAD;
  return op_col(prob, a, stream);
}

int altgdmin_op_backproject(const altgdmin_problem* prob, const int32_t* S_idx, const float* S_val, float* L0t,
                            void* stream) {
  altgdmin_params par;
  altgdmin_default_params(&par);
  int rc = validate(prob, &par);
  if (rc) return rc;
  if (!L0t || (prob->rho > 0 && (!S_idx || !S_val))) return fail(ALTGDMIN_EINVAL, "bad backproject arguments");
  ColArgs a;
  std::memset(&a, 0, sizeof(a));
  a.Tidx = const_cast<int32_t*>(S_idx); a.Tval = const_cast<float*>(S_val); a.H = L0t;
  a.tau = 0; a.project = 0; a.has_support = 1; a.tail = TAIL_BACKPROJ;
  return op_col(prob, a, stream);
}

int altgdmin_op_philox_fill(uint64_t seed, const float* normal_table, int32_t q, int32_t n, int32_t m, int64_t lda,
                            float* A, void* stream) {
  if (!normal_table || !A || q < 1 || n < 1 || m < 1 || lda < m) return fail(ALTGDMIN_EINVAL, "bad philox fill arguments");
  NEED_STREAM(stream);
  HIPCHK(launch_philox_fill(seed, normal_table, q, n, m, lda, A, static_cast<hipStream_t>(stream)));
  return ALTGDMIN_OK;
}

int altgdmin_op_make_a(uint64_t seed, const float* normal_table, int32_t q, int32_t n, int32_t m, int64_t lda,
                       int32_t a_format, void* A, void* A_lo, void* stream) {
  if (!normal_table || !A || q < 1 || n < 1 || m < 1 || lda < m || lda % 4 != 0)
    return fail(ALTGDMIN_EINVAL, "bad make_a arguments");
  NEED_STREAM(stream);
  if (a_format == ALTGDMIN_A_F32) {
    if (reinterpret_cast<uintptr_t>(A) % 16 != 0) return fail(ALTGDMIN_EINVAL, "A not 16-byte aligned");
    HIPCHK(launch_make_a(seed, normal_table, q, n, m, lda, FMT_F32, static_cast<float*>(A), nullptr, nullptr,
                         static_cast<hipStream_t>(stream)));
  } else if (a_format == ALTGDMIN_A_BF16X2) {
    if (!A_lo || reinterpret_cast<uintptr_t>(A) % 8 != 0 || reinterpret_cast<uintptr_t>(A_lo) % 8 != 0)
      return fail(ALTGDMIN_EINVAL, "BF16X2 needs two 8-byte aligned planes");
    HIPCHK(launch_make_a(seed, normal_table, q, n, m, lda, FMT_BF16X2, nullptr, static_cast<uint16_t*>(A),
                         static_cast<uint16_t*>(A_lo), static_cast<hipStream_t>(stream)));
  } else {
    return fail(ALTGDMIN_EINVAL, "make_a writes the F32 or BF16X2 format");
  }
  return ALTGDMIN_OK;
}

int altgdmin_op_measure(const altgdmin_problem* prob, const double* Xt, float* Y, void* stream) {
  if (!prob || !Xt || !Y) return fail(ALTGDMIN_EINVAL, "bad measure arguments");
  NEED_STREAM(stream);
  const altgdmin_problem& p = *prob;
  if (p.n < 1 || p.q < 1 || p.m < 1 || p.ldy < p.m) return fail(ALTGDMIN_EINVAL, "bad measure sizes");
  MeasureArgs a;
  a.n = p.n; a.q = p.q; a.m = p.m;
  a.A = p.A; a.Alo = p.A_lo; a.lda = p.lda; a.sA = p.a_stride_k;
  a.Xt = Xt; a.Y = Y; a.ldy = p.ldy; a.seed = p.a_seed; a.table = p.normal_table;
  int fmt;
  if (p.a_format == ALTGDMIN_A_PHILOX) {
    if (!p.normal_table) return fail(ALTGDMIN_EINVAL, "PHILOX needs the normal table");
    fmt = FMT_PHILOX;
  } else {
    if (!p.A || p.lda < p.m || p.lda % 4 != 0 || p.a_stride_k < p.lda * (int64_t)p.n)
      return fail(ALTGDMIN_EINVAL, "bad A layout");
    if (p.a_format == ALTGDMIN_A_F32) fmt = FMT_F32;
    else if (p.a_format == ALTGDMIN_A_BF16X2 && p.A_lo) fmt = FMT_BF16X2;
    else return fail(ALTGDMIN_EINVAL, "unknown a_format or missing lo plane");
  }
  HIPCHK(launch_measure(fmt, a, static_cast<hipStream_t>(stream)));
  return ALTGDMIN_OK;
}

// scratch layout of the U-side entry points: Ctl | gpart (KS n r) | Utmp (n r) | T (q r)
struct OpScratch {
  Ctl* ctl;
  float* gpart;
  float* Utmp;
  float* T;
  int KS;
  size_t bytes;
};

static OpScratch op_scratch(void* base, int n, int q, int r) {
  OpScratch s;
  Carver c(base);
  s.KS = grad_splits(q);
  s.ctl = c.take<Ctl>(1);
  s.gpart = c.take<float>((size_t)s.KS * n * r);
  s.Utmp = c.take<float>((size_t)n * r);
  s.T = c.take<float>((size_t)q * r);
  s.bytes = c.off;
  return s;
}

int altgdmin_op_scratch_bytes(int32_t n, int32_t q, int32_t r, size_t* bytes) {
  if (n < 1 || q < 1 || r < 1 || r > kRMax || !bytes) return fail(ALTGDMIN_EINVAL, "bad sizes");
  *bytes = op_scratch(nullptr, n, q, r).bytes;
  return ALTGDMIN_OK;
}

int altgdmin_op_grad(const float* H, const float* Bt, int32_t n, int32_t q, int32_t r, float* grad, void* scratch,
                     size_t scratch_bytes, void* stream) {
  if (!H || !Bt || !grad || !scratch || n < 1 || q < 1 || r < 1 || r > kRMax) return fail(ALTGDMIN_EINVAL, "bad grad arguments");
  NEED_STREAM(stream);
  OpScratch s = op_scratch(scratch, n, q, r);
  if (scratch_bytes < s.bytes) return fail(ALTGDMIN_ENOWS, "scratch too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIPCHK(launch_grad(H, Bt, n, q, r, s.KS, s.gpart, nullptr, st));
  HIPCHK(launch_sum_partials(s.gpart, s.KS, (long long)n * r, grad, st));
  return ALTGDMIN_OK;
}

int altgdmin_op_qr_step(const float* U, const float* grad, int32_t n, int32_t r, double eta_c, double* eta_io,
                        float* U_out, void* scratch, size_t scratch_bytes, void* stream) {
  if (!U || !grad || !eta_io || !U_out || !scratch || n < 1 || r < 1 || r > kRMax || r > n)
    return fail(ALTGDMIN_EINVAL, "bad qr arguments");
  NEED_STREAM(stream);
  OpScratch s = op_scratch(scratch, n, 1, r);
  if (scratch_bytes < s.bytes) return fail(ALTGDMIN_ENOWS, "scratch too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIPCHK(launch_copy_f(U_out, U, (long long)n * r, st));
  QRArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = n; a.r = r; a.KS = 1; a.mode = QR_GD; a.gpart = grad; a.U = U_out; a.Utmp = s.Utmp;
  a.eta_c = eta_c; a.eta_io = eta_io;
  HIPCHK(launch_qr(a, st));
  return ALTGDMIN_OK;
}

// The subspace iteration of altgdmin_op_subspace on a given scratch block (the
// caller's buffer, or the library's static one).  Every scratch word it reads is
// written first in the same call: the control block is reset by a kernel, the
// start block is filled, the partial sums and L_0^T U are overwritten.
static int subspace_body(const float* L0t, int32_t n, int32_t q, int32_t r, const float* U_start, int32_t iters,
                         double tol, float* U_out, int32_t* iters_out, void* scratch, size_t scratch_bytes,
                         void* stream) {
  OpScratch s = op_scratch(scratch, n, q, r);
  if (scratch_bytes < s.bytes) return fail(ALTGDMIN_ENOWS, "scratch too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIPCHK(launch_reset_ctl(s.ctl, 1, st));
  if (U_start) HIPCHK(launch_copy_f(s.Utmp, U_start, (long long)n * r, st));
  else HIPCHK(launch_fill_basis(s.Utmp, n, r, st));
  QRArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = n; a.r = r; a.KS = s.KS; a.gpart = s.gpart; a.U = U_out; a.Utmp = s.Utmp; a.ctl = s.ctl;
  a.power_tol = tol;
  a.mode = QR_ORTH;
  HIPCHK(launch_qr(a, st));
  a.mode = QR_POWER;
  for (int it = 0; it < iters; ++it) {
    HIPCHK(launch_ltu(L0t, U_out, n, q, r, s.T, &s.ctl->conv, st));
    HIPCHK(launch_grad(L0t, s.T, n, q, r, s.KS, s.gpart, &s.ctl->conv, st));
    HIPCHK(launch_qr(a, st));
  }
  if (iters_out) HIPCHK(hipMemcpyAsync(iters_out, &s.ctl->power_it, sizeof(int), hipMemcpyDeviceToDevice, st));
  return ALTGDMIN_OK;
}

static int subspace_args_ok(const float* L0t, int32_t n, int32_t q, int32_t r, int32_t iters, const float* U_out) {
  if (!L0t || !U_out || n < 1 || q < 1 || r < 1 || r > kRMax || r > n || iters < 0)
    return fail(ALTGDMIN_EINVAL, "bad subspace arguments");
  return ALTGDMIN_OK;
}

int altgdmin_op_subspace(const float* L0t, int32_t n, int32_t q, int32_t r, const float* U_start, int32_t iters,
                         double tol, float* U_out, int32_t* iters_out, void* scratch, size_t scratch_bytes,
                         void* stream) {
  int rc = subspace_args_ok(L0t, n, q, r, iters, U_out);
  if (rc) return rc;
  if (!scratch) return fail(ALTGDMIN_EINVAL, "null scratch");
  NEED_STREAM(stream);
  return subspace_body(L0t, n, q, r, U_start, iters, tol, U_out, iters_out, scratch, scratch_bytes, stream);
}

}  // extern "C"

extern "C" {

int altgdmin_op_rank_scratch_bytes(int32_t n, int32_t q, int32_t m, size_t* bytes) {
  if (n < 1 || q < 1 || m < 1 || !bytes) return fail(ALTGDMIN_EINVAL, "bad sizes");
  if (rank_budget(n, q, m) > kRankBlockMax)
    return fail(ALTGDMIN_ENOTBUILT, "min(n, q, m) / 10 above the largest block of the estimate");
  *bytes = rank_scratch(nullptr, rank_shape(n, q, m)).bytes;
  return ALTGDMIN_OK;
}

int altgdmin_op_rank(const float* L0t, int32_t n, int32_t q, int32_t m, double energy, int32_t iters,
                     int32_t* r_out, double* sv_out, void* scratch, size_t scratch_bytes, void* stream) {
  if (!L0t || !r_out || !scratch || n < 1 || q < 1 || m < 1 || iters < 1 || !(energy > 0.0 && energy <= 1.0))
    return fail(ALTGDMIN_EINVAL, "bad rank arguments");
  if (rank_budget(n, q, m) > kRankBlockMax)
    return fail(ALTGDMIN_ENOTBUILT, "min(n, q, m) / 10 above the largest block of the estimate");
  NEED_STREAM(stream);
  RankScratch rs = rank_scratch(scratch, rank_shape(n, q, m));
  if (scratch_bytes < rs.bytes) return fail(ALTGDMIN_ENOWS, "scratch too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  float* block = nullptr;
  HIPCHK(enqueue_rank(L0t, rank_shape(n, q, m), energy, iters, rs, &block, st));
  HIPCHK(hipMemcpyAsync(r_out, rs.r, sizeof(int), hipMemcpyDeviceToDevice, st));
  if (sv_out)
    HIPCHK(hipMemcpyAsync(sv_out, rs.sv, (size_t)rank_budget(n, q, m) * sizeof(double), hipMemcpyDeviceToDevice, st));
  return ALTGDMIN_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ allocation-free entry point
//
// For callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops, harnesses that forbid hipMalloc): the scratch of the
// subspace iteration lives in this file-scope device array, one copy per GPU,
// held until the process ends.  In host code `scratch` only names the symbol;
// its device address is taken once per device with hipGetSymbolAddress and only
// that address is handed to kernels and copies.

static __device__ __align__(256) unsigned char scratch[ALTGDMIN_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on its first use there).
int static_scratch(void** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(ALTGDMIN_EINVAL, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(ALTGDMIN_EHIP, "hipGetSymbolAddress returned no address for the static scratch");
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return ALTGDMIN_OK;
}

}  // namespace

extern "C" {

int altgdmin_op_subspace_noalloc(const float* L0t, int32_t n, int32_t q, int32_t r, const float* U_start,
                                 int32_t iters, double tol, float* U_out, int32_t* iters_out, void* stream) {
  int rc = subspace_args_ok(L0t, n, q, r, iters, U_out);
  if (rc) return rc;
  NEED_STREAM(stream);
  const size_t need = op_scratch(nullptr, n, q, r).bytes;
  if (need > ALTGDMIN_STATIC_SCRATCH_BYTES)
    return fail(ALTGDMIN_ENOWS, "sizes need " + std::to_string(need) + " bytes of scratch, more than the " +
                                    std::to_string((size_t)ALTGDMIN_STATIC_SCRATCH_BYTES) + " of the static array");
  void* p = nullptr;
  rc = static_scratch(&p);
  if (rc) return rc;
  return subspace_body(L0t, n, q, r, U_start, iters, tol, U_out, iters_out, p, ALTGDMIN_STATIC_SCRATCH_BYTES, stream);
}

}  // extern "C"
