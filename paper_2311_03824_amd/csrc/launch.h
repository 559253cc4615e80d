// Launchers of the AltGDmin-LR+S kernels (host side, internal to the library).
#pragma once
#include "common.h"

namespace altg {

enum { QR_GD = 0, QR_POWER = 1, QR_ORTH = 2 };

struct QRArgs {
  int n, r, KS, mode;
  const float* gpart;      // KS x n x r partial sums (GD: gradient, POWER: L0 L0^T U)
  float* U;                // n x r, in/out
  float* Uprev;            // n x r, GD: receives the U the step started from
  float* Utmp;             // n x r scratch; ORTH: the block to orthonormalise
  Ctl* ctl;
  double eta_c, power_tol;
  const double* colrr;     // q residual norms^2 of the iteration (GD)
  const int* colflags;     // q column flags (GD)
  int q;
  double* rlog;            // residual log (GD)
  int rlog_len;
  float* grad_out;         // optional copy of the summed partials
  double* eta_io;          // op entry: eta in/out (<= 0: compute), used instead of ctl when ctl == nullptr
  int lds;                 // set by launch_qr: the n x r block is staged in LDS
  int hi_max;              // BF16X2 hi-only budget (iterations)
  double stall;            // BF16X2 stall ratio
  double tol;              // GD with gate_done: set ctl->done once resid <= tol
  int gate_done;           // GD: skip the update when ctl->done is set (batched stepping)
};

// dynamic LDS for the n x r block of k_qr (with its 10 KiB of static LDS, up to the
// CU's 160 KiB; above the default 48 KiB the kernels' limit is raised on first use)
constexpr size_t kQRLdsMax = 144 * 1024;
constexpr size_t kQRLdsDefault = 48 * 1024;
constexpr int kGradWaves = 16;             // waves of a gradient-reduction workgroup

struct GradArgs {
  const float* H;
  const float* B;
  int n, q, r, KS;
  float* gpart;
  const int* skip;   // if non-null and *skip != 0, the workgroup does nothing
};

// pol: POL_STREAM (non-temporal loads of A) or POL_CACHED (ordinary loads; for a
// streamed plane that fits in the Infinity Cache).  The same bits either way;
// a form without a cached instantiation (Philox, 16-wave columns) streams.
hipError_t launch_col(int fmt, const ColArgs& a, hipStream_t st, int pol = 0);
// autotuned variants (FP32 and BF16X2 planes): JU in {1, 2, 3}, AUD in {1, 2, 4}
hipError_t launch_col_tuned(int fmt, int ju, const ColArgs& a, hipStream_t st);
hipError_t launch_au_tuned(int fmt, int aud, const AUArgs& a, hipStream_t st);
hipError_t launch_au(int fmt, const AUArgs& a, hipStream_t st, int pol = 0);
bool au_supported(int m, int r);
hipError_t launch_col_grp(int fmt, int nc, int waves, const ColArgs* tab, const int2* map, int blocks, size_t lds,
                          hipStream_t st, int pol = 0);
// the cached-load instantiations (hipErrorNotSupported where none is built)
hipError_t launch_col_cached(int fmt, const ColArgs& a, hipStream_t st);
hipError_t launch_col_grp_cached(int fmt, int nc, int waves, const ColArgs* tab, const int2* map, int blocks,
                                 size_t lds, hipStream_t st);
hipError_t launch_au_cached(int fmt, const AUArgs& a, hipStream_t st);
hipError_t launch_au_grp_cached(int fmt, int rmax, int waves, const AUArgs* tab, const int2* map, int blocks,
                                size_t lds, hipStream_t st);
// column workgroups of 8 or 16 waves (a.waves); built for 8 waves, and 16 waves at m <= 512
bool col_wide_built(int waves, int nc);
hipError_t launch_col_wide(int fmt, const ColArgs& a, hipStream_t st);
hipError_t launch_col_grp_wide(int fmt, int nc, int waves, const ColArgs* tab, const int2* map, int blocks,
                               size_t lds, hipStream_t st);
// A_k U over several problems; waves: the problems' A_k U width (8 or 4, see AUArgs::waves)
hipError_t launch_au_grp(int fmt, int rmax, int waves, const AUArgs* tab, const int2* map, int blocks, size_t lds,
                         hipStream_t st, int pol = 0);
size_t col_lds_bytes(int n, int m, int r, int rho, int project, int philox, int waves = kWaves);
// A column workgroup takes at most 64 KiB of LDS by default and up to the CU's
// 160 KiB for large n (g, the step and the support bitmap are n-long LDS arrays;
// a CU then holds one column workgroup).  col_allow_big_lds() raises the dynamic
// LDS limit of every column kernel once; call it before the first launch that
// needs more than 64 KiB and before any graph capture.
constexpr size_t kColLdsDefault = 64 * 1024;
constexpr size_t kColLdsMax = 160 * 1024;
hipError_t col_allow_big_lds();
hipError_t col_allow_big_lds_tuned();    // the autotuned and wide variants
hipError_t col_allow_big_lds_cached();   // the cached-load variants
size_t au_lds_bytes(int m, int r, int philox, int waves = kWaves);
hipError_t launch_philox_fill(unsigned long long seed, const float* table, int q, int n, int m, long long lda, float* A,
                              hipStream_t st);
size_t select_lds_bytes(int n, int rho);
hipError_t launch_select(const float* V, int n, int count, long long ldv, int rho, int* idx, float* val,
                         int* flags, hipStream_t st);
hipError_t launch_sum_partials(const float* gpart, int KS, long long nr, float* out, hipStream_t st);
hipError_t launch_grad(const float* H, const float* B, int n, int q, int r, int KS, float* gpart,
                       const int* skip, hipStream_t st);
hipError_t launch_ltu(const float* L0t, const float* U, int n, int q, int r, float* T, const int* skip,
                      hipStream_t st);
hipError_t launch_qr(const QRArgs& a, hipStream_t st);
hipError_t launch_grad_grp(const GradArgs* tab, const int4* map, int blocks, hipStream_t st);
hipError_t launch_qr_grp(const QRArgs* tab, int count, size_t lds, hipStream_t st);
hipError_t launch_sum_ctl(const double* colrr, int q, Ctl* ctl, hipStream_t st);
hipError_t launch_reset_ctl(Ctl* ctl, int full, hipStream_t st);
hipError_t launch_set_phase(Ctl* ctl, int phase, hipStream_t st);
hipError_t launch_fill_int(int* p, int v, long long count, hipStream_t st);
hipError_t launch_fill_basis(float* U, int n, int r, hipStream_t st);
hipError_t launch_copy_f(float* dst, const float* src, long long count, hipStream_t st);
hipError_t launch_copy_i(int* dst, const int* src, long long count, hipStream_t st);
// header words of a saved solver state, written on the stream by a kernel (so the
// host values are captured at launch, with no host buffer to keep alive)
constexpr int kStateWords = 16;
struct StateWords {
  long long v[kStateWords];
};
hipError_t launch_put_words(long long* dst, const StateWords& w, hipStream_t st);
hipError_t launch_check_support(int* idx, float* val, int vpe, int q, int rho, int n, int* flags, hipStream_t st);

// partial Fourier form (96 x 96 complex frames by FFT; other frame sizes by direct line DFTs)
constexpr int kFN = 96;                // 1D transform size
constexpr int kFP = 97;                // LDS row stride of a frame (complex elements)
constexpr int kFGrid = kFN * kFP;      // complex elements of a padded frame
constexpr int kFThreads = 1024;        // workgroup of the Fourier kernels
constexpr int kFWaves = kFThreads / 64;
constexpr int kFRMax = 8;              // largest rank of the Fourier kernels
constexpr int kFRhoMax = 256;          // largest rho of the Fourier column kernel
constexpr int kFGenPer = 4;            // generic frames: n <= kFGenPer * kFThreads elements
constexpr int kFGenLineMax = 1024;     // generic frames: n1, n2 <= 1024 (twiddle tables in LDS)
constexpr size_t kFLdsMax = 160 * 1024;   // LDS of one CU, the most a Fourier column workgroup takes
enum { FCOL_INIT = 0, FCOL_GD = 1 };

struct FColArgs {
  int n, q, m, r, rho, tau, mode;
  const int* mask;       // q x m frequency indices, ascending per frame
  const float2* Y;       // y_k at Y[k * ldy]
  long long ldy;
  const float2* FU;      // n x r, the 2D DFT of U's columns (GD)
  const float2* tw;      // 96 x 96 frames: 96 twiddles exp(-2 pi i t / 96); other frames: W_n1^t, then W_n2^t
  int n1, n2;            // frame size (n = n1 n2)
  int* Sidx;             // q x rho, in (GD) / out
  float2* Sval;          // q x rho
  float2* Bt;            // q x r (GD)
  float2* H;             // q x n: L_0 columns (init) or A_k^H r_k (GD)
  double* colrr;         // q: ||y_k||^2 (init) or ||r_k||^2 (GD)
  int* flags;            // q
};

struct FQRArgs {
  int n, r, q, mode;
  const float2* G;       // n x r: grad_U f (GD) or L_0 L_0^H U (POWER)
  float2* U;
  float2* Uprev;
  float2* Utmp;
  Ctl* ctl;
  double eta_c, power_tol;
  const double* colrr;
  const int* colflags;
  double* rlog;
  int rlog_len;
  double2* part;         // over many workgroups: per-block partial Grams (nb x 3 r^2); POWER also
                         // the per-block change sums after nb r^2
  double2* rinv;         // R1^{-1}, R2^{-1} (2 r^2)
  int nb;                // 256-row blocks of n
};

size_t fcol_lds_bytes(int rho, int r, int n, int m, int n1, int n2);
hipError_t launch_fu_gen(const float2* U, int n, int r, int n1, int n2, const float2* tw, float2* FU,
                         hipStream_t st);
hipError_t launch_ftwiddle_gen(float2* tw, int n1, int n2, hipStream_t st);
hipError_t launch_fgrad_gd(const float2* H, const float2* B, const float2* U, int n, int q, int r, float2* Gsum,
                           double2* part, const int* skip, hipStream_t st);
hipError_t launch_fqr_gd(const FQRArgs& a, hipStream_t st);
hipError_t launch_fcol(const FColArgs& a, hipStream_t st);
hipError_t launch_fu(const float2* U, int r, const float2* tw, float2* FU, hipStream_t st);
hipError_t launch_fltu(const float2* H, const float2* U, int n, int q, int r, float2* Tc, const int* skip,
                       hipStream_t st);
hipError_t launch_fqr(const FQRArgs& a, hipStream_t st);
hipError_t launch_ftwiddle(float2* tw, hipStream_t st);
hipError_t launch_fbasis(float2* U, int n, int r, hipStream_t st);

// automatic rank (Sec. 2.6): block subspace iteration, CholeskyQR2, Rayleigh-Ritz by Jacobi
constexpr int kRankBlockMax = 88;   // block columns b: the b x b FP64 matrices stay under 64 KiB of LDS
size_t rank_lds_bytes(int b);
hipError_t launch_rank_mm(bool trans, const float* A, long long lda, const float* B, long long ldb, float* C,
                          long long ldc, int M, int N, int K, hipStream_t st);
hipError_t launch_rank_gram(const float* X, int rows, int b, double* W, hipStream_t st);
hipError_t launch_rank_chol(const double* W, int b, double* Xinv, float* Xf, int* flag, hipStream_t st);
hipError_t launch_rank_jacobi(const double* M, int b, int K, double energy, double* sv, int* r_out,
                              hipStream_t st);
hipError_t launch_rank_slice(const float* Ub, int n, int b, int r, float* U, hipStream_t st);
// Et (2q x 2n real) = the transpose of the real embedding [[X, -Y], [Y, X]] of the
// complex L_0 = X + iY given as L0t (q x n complex64)
hipError_t launch_rank_embed(const float* L0t, int q, int n, float* Et, hipStream_t st);

// synthetic instances on the device
struct MeasureArgs {
  int n, q, m;
  const void* A;
  const void* Alo;
  long long lda, sA;
  const double* Xt;   // q x n, x_k at Xt[k * n]
  float* Y;
  long long ldy;
  unsigned long long seed;
  const float* table;
};
hipError_t launch_make_a(unsigned long long seed, const float* table, int q, int n, int m, long long lda, int fmt,
                         float* A32, uint16_t* hi, uint16_t* lo, hipStream_t st);
hipError_t launch_measure(int fmt, const MeasureArgs& a, hipStream_t st);

}  // namespace altg
