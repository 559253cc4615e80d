/*
 * altgdmin.h -- C ABI of the MI355X (gfx950) hot path of AltGDmin-LR+S.
 *
 * Method: S. Babu, N. Vaswani, "A Fast Algorithm for Low Rank + Sparse
 * column-wise Compressive Sensing", arXiv 2311.03824.  Problem statement of
 * Sec. 1.1: recover X = L + S (n x q), L = U B of rank r and every column of S
 * holding rho nonzeros, from y_k = A_k x_k, k = 0..q-1, A_k an m x n matrix.
 * The solver is Alg. 1 (altGDmin-L+S) with Alg. 2 (IHT) inside.
 *
 * Conventions shared by every entry point
 *  - All array pointers are DEVICE pointers unless the argument says "host".
 *    The library never allocates or frees device memory: the caller owns the
 *    inputs, the outputs and the workspace, which must outlive every call
 *    that uses them (and the handle).
 *  - Work is enqueued on the caller's HIP stream (`stream`, a hipStream_t
 *    passed as void*).  The library never enqueues on the null (legacy default)
 *    stream: a NULL stream is rejected with ALTGDMIN_EINVAL.  Calls return as
 *    soon as the work is enqueued unless they say they synchronise.
 *  - Layout of A (format ALTGDMIN_A_F32): A_k is column-major with the row
 *    index fastest: element (i, j) of A_k is A[k*a_stride_k + j*lda + i].
 *    lda >= m and lda, a_stride_k and the base address must be multiples of 4
 *    floats (16 bytes).  Rows m..lda-1 do not change any result but are read, so
 *    they must hold finite values (zeros, as altgdmin_op_make_a writes them).
 *    Format ALTGDMIN_A_BF16X2: A_k = hi + lo with hi and lo bfloat16 planes of
 *    the same layout (uint16 elements; lda, a_stride_k multiples of 8).
 *  - Y: y_k at Y[k*ldy + i], ldy >= m.
 *  - U: n x r row-major (U[j*r + c]); B is returned transposed, Bt q x r
 *    row-major (Bt[k*r + c] = b_k[c]); S as q x rho arrays of row indices
 *    (int32, strictly ascending within a column) and values (float).  A start
 *    support handed in by the caller (altgdmin_op_iht, altgdmin_op_lsgrad,
 *    altgdmin_op_backproject) whose indices are out of range, or not strictly
 *    ascending (unsorted or repeated), is flagged (error bit 2) and that column
 *    is treated as having no start (s = 0).
 *  - Partial Fourier form (a_format ALTGDMIN_A_PFOURIER): A_k x = (F x)[mask_k]
 *    with F the unitary 2D DFT, (F x)[u1, u2] = (n1 n2)^(-1/2) sum x[j1, j2]
 *    exp(-2 pi i (u1 j1 / n1 + u2 j2 / n2)); A is never stored (A, A_lo, lda
 *    and a_stride_k are ignored).  Y, U, Bt and S_val hold complex64 values
 *    (interleaved re, im float pairs; ldy counts complex elements), so every
 *    float* output of such a problem receives twice the float count of the
 *    real form.  Frames of 96 x 96 run 2D FFTs; other frame sizes with
 *    n = n1 n2 <= 4096 and n1, n2 <= 1024 (n1 = 1 gives a 1D DFT of length n2)
 *    run direct line DFTs, as long as the frame and the rows of P_k fit the
 *    LDS of one CU.  Limits: m <= min(n, 2048), r <= 8, rho <= 256.  Every
 *    transpose of Alg. 1 and Alg. 2 becomes a conjugate transpose and
 *    HardThreshold ranks by the modulus, computed as the FP32 key
 *    fl(fl(re*re) + fl(im*im)) (lower index first on equal keys).
 *  - Threads: a handle keeps host state (iteration count, the captured graph),
 *    so calls on one handle must not overlap; different handles may be used
 *    from different host threads at once (the process-wide autotuning cache is
 *    locked).  Work enqueued on one handle from different streams must be
 *    ordered by the caller.
 *  - Return codes: ALTGDMIN_OK (0); negative values are errors; the positive
 *    ALTGDMIN_ENOTCONV is a warning.  altgdmin_last_error() gives the text of
 *    the last error of the calling thread.  Faults inside kernels surface at
 *    the next call that synchronises.
 */
#ifndef ALTGDMIN_H
#define ALTGDMIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ALTGDMIN_OK = 0,
  ALTGDMIN_ENOTCONV = 1,     /* t_max reached before tol_resid (warning) */
  ALTGDMIN_EINVAL = -1,      /* invalid argument or unsupported size */
  ALTGDMIN_ENOWS = -2,       /* workspace too small */
  ALTGDMIN_EHIP = -3,        /* HIP runtime error */
  ALTGDMIN_ENONFINITE = -4,  /* a NaN/Inf reached the selection, or a Gram matrix was not positive definite */
  ALTGDMIN_ENOTBUILT = -5    /* no kernel instantiation for these sizes */
};

enum {
  ALTGDMIN_A_F32 = 0,        /* FP32 plane */
  ALTGDMIN_A_BF16X2 = 1,     /* BF16 hi plane + BF16 lo plane, A = hi + lo */
  ALTGDMIN_A_PHILOX = 2,     /* regenerated in the kernels from a counter; never stored (see altgdmin_op_philox_fill) */
  ALTGDMIN_A_PFOURIER = 3    /* partial Fourier: rows fourier_mask[k] of the unitary 2D DFT of n1 x n2 complex frames */
};

/* altgdmin_params.flags bits */
#define ALTGDMIN_FLAG_EAGER 1      /* launch each iteration's kernels directly instead of replaying a HIP graph */
#define ALTGDMIN_FLAG_AUTOTUNE 2   /* FP32 / BF16X2 planes: altgdmin_init times the loads-in-flight variants of the
                                      streaming kernels on the problem and keeps the fastest (see altgdmin_tuning) */
#define ALTGDMIN_FLAG_BF16_MIXED 4 /* BF16X2 planes, mixed form: every product that forms a residual (A_k U and the
                                      support gathers A_k s_k) reads hi + lo, i.e. A exactly; the streaming
                                      transposed products A_k^T v (IHT gradients, h_k of grad_U f, the
                                      back-projection L_0) and the IHT step-length product read the hi plane
                                      alone, at half the bytes.  The exact iterate X* stays a fixed point; the
                                      search directions carry the 2^-9 relative error of the hi plane.  Needs
                                      bf16_hi_max = 0. */

/* Entries of the normal table of the Philox form: |z| = -Phi^{-1}(v) at
 * v = 2^(e-33) (1 + s/64), e = 0..31, s = 0..63 (index e*64 + s), then two zeros. */
#define ALTGDMIN_NORMAL_TABLE_SIZE (32 * 64 + 2)

/* Problem of Sec. 1.1: sizes, measurement matrices and measurements. */
typedef struct altgdmin_problem {
  int32_t n, q, m, r, rho;   /* 1 <= r <= min(m, n), 0 <= rho <= n; rho is the threshold budget (Sec. 2.6).
                                r = 0: the automatic rank of Sec. 2.6, chosen by altgdmin_init from L_0 (see
                                altgdmin_params.rank_energy); the workspace is then laid out for r_cap =
                                min(K, 16, m, n) (min(K, 8, m, n) in the Fourier form) with K = max(1,
                                floor(min(n, q, m) / 10)), U_start is not used, and altgdmin_report.rank gives
                                the r chosen (outputs have r columns).  The Fourier form estimates the values
                                on the real embedding [[X, -Y], [Y, X]] of L_0 = X + iY (each value twice);
                                K <= 88 (44 in the Fourier form), else ALTGDMIN_ENOTBUILT */
  int32_t a_format;          /* ALTGDMIN_A_* */
  const void* A;             /* F32: const float*; BF16X2: hi plane, const uint16_t* */
  const void* A_lo;          /* BF16X2: lo plane; NULL otherwise */
  int64_t lda;               /* column stride of A_k in elements */
  int64_t a_stride_k;        /* stride between A_k and A_{k+1} in elements, >= lda*n */
  const float* Y;            /* q x ldy */
  int64_t ldy;
  const float* U_start;      /* optional n x r start block of the subspace iteration (NULL: a fixed disjoint-support
                                basis); complex64 pairs for PFOURIER */
  uint64_t a_seed;           /* PHILOX: 64-bit key of A */
  const float* normal_table; /* PHILOX: device array of ALTGDMIN_NORMAL_TABLE_SIZE FP32 */
  int32_t n1, n2;            /* PFOURIER: frame size, n = n1 * n2 (x_k flattened row-major): 96 x 96 (FFT), or
                                n <= 4096 with n1, n2 <= 1024 (direct line DFTs) */
  const int32_t* fourier_mask; /* PFOURIER: q x m frequency indices u = u1 * n2 + u2, ascending per frame */
} altgdmin_problem;

/* Parameters of Alg. 1 / Sec. 2.6. */
typedef struct altgdmin_params {
  int32_t tau0;              /* IHT iterations of the initialisation (paper: 10) */
  int32_t tau;               /* IHT iterations per GDmin iteration (paper: 3) */
  int32_t t_max;             /* GDmin iterations (paper: 200) */
  int32_t power_iters;       /* max subspace iterations for U_0 (top-r left singular vectors of L_0); the
                                change shrinks by (sigma_{r+1} / sigma_r)^2 of L_0 per step, so a small gap
                                (ratio near 1) needs more than the default 100 */
  int32_t poll_every;        /* altgdmin_solve reads the residual every poll_every iterations */
  int32_t flags;             /* ALTGDMIN_FLAG_* bits, 0 by default */
  double eta_c;              /* eta = eta_c / ||grad_U f(U_0, B_1, S_1)||_2 (paper: 0.14) */
  double power_tol;          /* stop the subspace iteration when ||(I - U_p U_p^T) U_{p+1}||_F <= power_tol,
                                or when that change, below 1e-3, shrank by less than 1 % in a step (the
                                FP32 rounding floor of the iterate) */
  double tol_resid;          /* altgdmin_solve stops when ||Y - A(UB+S)||_F / ||Y||_F <= tol_resid (0: never) */
  int32_t bf16_hi_max;       /* BF16X2 only: the initialisation and up to this many GDmin iterations read
                                the hi plane alone (2 bytes per element); 0 disables the hi-only phase */
  int32_t pad0;
  double bf16_stall;         /* BF16X2 hi-only phase ends early once resid_t >= bf16_stall * resid_{t-1} */
  double rank_energy;        /* r = 0: the energy fraction of the automatic rank (paper: 0.65) */
  int32_t rank_iters;        /* r = 0: steps of the block subspace iteration that estimates the leading
                                singular values of L_0 (default 30) */
  int32_t pad1;
} altgdmin_params;

/* Fills *p with the paper's defaults (tau0 = 10, tau = 3, t_max = 200, eta_c = 0.14). Host call. */
void altgdmin_default_params(altgdmin_params* p);

typedef struct altgdmin_handle altgdmin_handle;

/* Host-side status, filled by altgdmin_status (synchronises the stream). */
typedef struct altgdmin_report {
  int32_t iterations;        /* GDmin iterations done */
  int32_t power_iterations;  /* subspace iterations used for U_0 */
  int32_t error_flags;       /* bit 0: NaN at a selection; bit 1: Gram not positive definite; bit 2: invalid start
                                support (index out of range, unsorted or repeated) or frequency index out of range */
  int32_t converged;         /* 1 when the last residual <= tol_resid and no error flag is set */
  int32_t refine_iteration;  /* BF16X2: first GDmin iteration that read hi + lo (-1: still hi-only or no hi-only phase) */
  int32_t rank;              /* the rank r in use (with r = 0 in the problem: the one altgdmin_init chose) */
  double eta;                /* step size (0 before iteration 1) */
  double resid;              /* ||Y - A(U B + S)||_F / ||Y||_F of the last iteration's consistent pair (NaN once a
                                non-finite value reached a residual); an iteration whose QR step failed (error bit
                                1) is still counted and leaves U unchanged */
  double power_sd;           /* last subspace-iteration change */
} altgdmin_report;

/* Exact device workspace size for a problem (host call, no GPU work). */
int altgdmin_workspace_bytes(const altgdmin_problem* prob, const altgdmin_params* par, size_t* bytes);

/* Validates, carves the workspace and enqueues the initialisation of Alg. 1
 * (Sec. 2.3): s_k = IHT(y_k, A_k, rho, tau0, 0), L_0 = [A_k^T (y_k - A_k s_k)],
 * U_0 = top-r left singular subspace of L_0 by subspace iteration.  *out gets a
 * small host object; the problem arrays and workspace must outlive it. */
int altgdmin_init(const altgdmin_problem* prob, const altgdmin_params* par, void* workspace,
                  size_t ws_bytes, void* stream, altgdmin_handle** out);

/* Enqueues `iters` GDmin iterations of Alg. 1 (z_k/M_k from U, warm-started IHT
 * for s_k, LS for b_k (eq. (bk_LS)), grad_U f, eta at t = 1, U+ = QR(U - eta grad)).
 * The iteration is captured once as a HIP graph and replayed.  Asynchronous. */
int altgdmin_step(altgdmin_handle* h, int32_t iters, void* stream);

/* Copies the consistent state (U that B and S were fitted with, Bt, S) into
 * caller buffers (device pointers, torch shapes (n,r), (q,r), (q,rho), (q,rho)).
 * Any pointer may be NULL.  U_next (optional) receives the already-updated U. */
int altgdmin_get(altgdmin_handle* h, float* U, float* Bt, int32_t* S_idx, float* S_val,
                 float* U_next, void* stream);

/* Synchronises `stream` and reads the device status into *rep (host). */
int altgdmin_status(altgdmin_handle* h, void* stream, altgdmin_report* rep);

/* Status of several handles with one synchronisation of `stream` (serving
 * polls): reps (host, count entries) as altgdmin_status fills them. */
int altgdmin_status_many(altgdmin_handle* const* hs, int32_t count, void* stream, altgdmin_report* reps);

/* Per-iteration relative residual log, host array of length >= t_max; returns count in *count. Synchronises. */
int altgdmin_residual_log(altgdmin_handle* h, void* stream, double* host_log, int32_t* count);

/* init + step until tol_resid or t_max, polling every poll_every iterations,
 * then copies the consistent state out (device pointers, any may be NULL).
 * Synchronises.  Returns ALTGDMIN_ENOTCONV when t_max is reached first and
 * tol_resid > 0. */
int altgdmin_solve(const altgdmin_problem* prob, const altgdmin_params* par, void* workspace,
                   size_t ws_bytes, void* stream, float* U, float* Bt, int32_t* S_idx,
                   float* S_val, altgdmin_report* rep);

/* Measurement hook: runs `iters` GDmin iterations with eager launches and a
 * HIP event pair around each of the four kernels of an iteration (A_k U,
 * column kernel, gradient reduction, U update), on `stream`.  ms_out (host,
 * 4 doubles) receives the average duration of each kernel in milliseconds.
 * Advances the solve like altgdmin_step.  Synchronises. */
int altgdmin_profile_iteration(altgdmin_handle* h, int32_t iters, void* stream, double* ms_out);

/* Autotuner (with ALTGDMIN_FLAG_AUTOTUNE): the column-kernel unroll JU (columns
 * per load group, 1, 2, 4 or 8) and the A_k U pipeline depth AUD (1, 2, 3, 4 or 8) chosen for
 * this handle; 0 means the default instantiation, -1 the default instantiation
 * with cached loads of A.  Without the autotuner every handle reports 0, or -1
 * when the plane of A that the column passes stream (4 bytes per element, 2 in
 * the mixed BF16 form) takes at most 200 MiB, so that the Infinity Cache keeps
 * it between passes; otherwise A is read with non-temporal loads.  With the
 * autotuner that default (0 or -1) is the baseline the variants are timed
 * against.  The default A_k U kernels keep deeper load pipelines for launches of
 * at most 256 columns (one workgroup per CU), and problems of at most 512 columns
 * run A_k U in 8-wave workgroups, whose partial sums, and so bits, differ from
 * the 4-wave ones (ALTGDMIN_AU_WAVES=4|8 forces the width; the depth variants are
 * built for 4 waves).  The environment
 * variable ALTGDMIN_LOAD_POLICY=stream|cached forces the load policy of the
 * default instantiations (for tests; the batched altgdmin_step_many applies the
 * same 200 MiB rule to all its problems together).  The choice is made once per
 * (GPU architecture, A format, n, q, m, r, rho) in a process by timing the
 * default and each variant five times on the problem's own data (A_k U from a
 * fixed orthonormal U; the column kernel as in a GDmin iteration, from an empty
 * support) before the initialisation; a variant replaces the default only when
 * it is at least 2 % faster than the best so far.  With the environment variable
 * ALTGDMIN_TUNE_CACHE naming a file, choices are read from and appended to it as
 * JSON lines keyed by the architecture.  ALTGDMIN_TUNE_FORCE="JU,AUD" takes the given variants without
 * timing (JU = 8 falls back to 4 above 512 rows; -1 selects the cached
 * default).  Every variant and both load policies compute the same bits.  Host
 * call. */
int altgdmin_tuning(altgdmin_handle* h, int32_t* col_unroll, int32_t* au_depth);

/* Device bytes of the launch tables altgdmin_step_many needs for these handles (host call). */
int altgdmin_group_bytes(altgdmin_handle* const* hs, int32_t count, size_t* bytes);

/* Serving: `iters` GDmin iterations of every handle in hs[0..count), with the
 * column work of all problems batched into shared launches (per A format and
 * kernel instantiation -- ceil(m / 256) for the column kernel, r rounded up to
 * even for A_k U -- one A_k U launch and one column-kernel launch over the
 * columns of those problems; then one gradient-reduction launch and one
 * U-update launch with a workgroup per problem).  Each problem keeps its own
 * U/B/S state in its workspace and follows exactly the arithmetic of
 * altgdmin_step (problems are also bucketed by their column-workgroup width, 8
 * waves for q <= 320 and 4 above: the width sets the order of the kernels'
 * cross-wave sums).  A problem whose params have tol_resid > 0 is frozen from the
 * iteration after its residual first reaches tol_resid: its kernels skip it, so
 * its state, report.iterations and report.resid stay those of the first
 * iteration that met the tolerance.  group_ws (device, 256-byte aligned,
 * >= altgdmin_group_bytes) holds the launch tables; each call uploads them on
 * `stream` from a pinned host buffer the library keeps, without synchronising
 * the stream (the call returns once the work is enqueued).  The batched launches use the
 * default loads-in-flight instantiations (an autotuned choice applies to
 * altgdmin_step / altgdmin_solve; every variant gives the same bits).  Handles
 * of a BF16X2 problem with a hi-only phase are rejected (EINVAL). */
int altgdmin_step_many(altgdmin_handle* const* hs, int32_t count, int32_t iters, void* group_ws,
                       size_t group_bytes, void* stream);

/* Checkpoint and resume.  Sec. 2.5 lists what the method keeps between
 * iterations: U (n x r), B (r x q) and the 2 rho q numbers of S; with them a
 * saved state holds the step size eta (fixed at t = 1), the iteration count
 * and the rest of the device control block (residual, BF16 phase, error
 * flags), U_prev (the U that B and S were fitted with) and the residual log.
 * altgdmin_state_bytes: bytes of a saved state of this handle (host call).
 * altgdmin_get_state: enqueues device-to-device copies of the state into
 *   `state` (device, 256-byte aligned, >= altgdmin_state_bytes); asynchronous.
 * altgdmin_set_state: loads a state saved from a handle of the same problem
 *   (n, q, m, r, rho, A format and column form) into h, e.g. a fresh handle
 *   after altgdmin_init; the next altgdmin_step continues from it, giving the
 *   same bits as iterating on without the save.  Synchronises `stream` once to
 *   read the saved header; EINVAL if it is not a state of such a problem.  The
 *   problem arrays (A, Y) must be those of the saved solve. */
int altgdmin_state_bytes(altgdmin_handle* h, size_t* bytes);
int altgdmin_get_state(altgdmin_handle* h, void* state, size_t bytes, void* stream);
int altgdmin_set_state(altgdmin_handle* h, const void* state, size_t bytes, void* stream);

/* Frees the host handle only. */
int altgdmin_destroy(altgdmin_handle* h);

const char* altgdmin_strerror(int code);
const char* altgdmin_last_error(void);

/* ------------------------------------------------------------------------
 * Step-level entry points.  Each runs one step of the path on caller buffers,
 * with the same kernels the solver uses, so that every step can be checked on
 * its own.  Stateless; asynchronous on `stream`.
 * ---------------------------------------------------------------------- */

/* HardThreshold(v, rho) of Alg. 2 on `count` vectors v_c = V[c*ldv + 0..n-1]:
 * keeps the rho entries of largest |v| (lower index first on ties), writes
 * their indices ascending to idx[c*rho + t] and values to val[c*rho + t].
 * flags[c] (optional) gets bit 0 if v_c holds a NaN. */
int altgdmin_op_select(const float* V, int32_t n, int32_t count, int64_t ldv, int32_t rho,
                       int32_t* idx, float* val, int32_t* flags, void* stream);

/* The Philox form of A written out in the FP32 layout (A[k*n*lda + j*lda + i],
 * rows i < m): element (i, j) of A_k is output word i % 4 of Philox4x32-10
 * (Salmon et al., SC'11) at counter (i / 4, j, k, 0) with key (seed low word,
 * seed high word), made a normal deviate by the table transform: with
 * v = (2 (x & 0x7fffffff) + 1) * 2^-33 (FP32), idx = 64 * (exponent(v) + 33) +
 * top 6 mantissa bits of v, t = low 17 mantissa bits * 2^-17,
 * |z| = T[idx] + (T[idx+1] - T[idx]) * t (each operation rounded to FP32), sign
 * from the top bit of x.  The kernels of the PHILOX format compute exactly these
 * values in registers.  For tests and for callers that want the matrix. */
int altgdmin_op_philox_fill(uint64_t seed, const float* normal_table, int32_t q, int32_t n, int32_t m,
                            int64_t lda, float* A, void* stream);

/* Synthetic measurement matrices (input generation, not a step of Alg. 1): the
 * draw a of element (i, j) of A_k is the value altgdmin_op_philox_fill writes; the
 * stored matrix is the canonical A = hi + lo, hi = bf16_RN(a), lo = bf16_RN(a - hi)
 * (round to nearest even), exact in FP32.  a_format ALTGDMIN_A_F32 writes hi + lo
 * as FP32 into A; ALTGDMIN_A_BF16X2 writes the hi plane into A and the lo plane
 * into A_lo (uint16).  Layout A[k*n*lda + j*lda + i]; rows m..lda-1 are written
 * as zeros; lda a multiple of 4.  Asynchronous on `stream`. */
int altgdmin_op_make_a(uint64_t seed, const float* normal_table, int32_t q, int32_t n, int32_t m,
                       int64_t lda, int32_t a_format, void* A, void* A_lo, void* stream);

/* Measurements of the model of Sec. 1.1, y_k = A_k x_k (noise-free), for the A
 * of `prob` in any format (prob->Y is ignored).  Xt: q x n FP64 row-major
 * (x_k at Xt[k*n]); Y: y_k at Y[k*ldy + i] in FP32.  Each y_k[i] is accumulated
 * in FP64 over j = 0..n-1 in order and rounded once.  Asynchronous. */
int altgdmin_op_measure(const altgdmin_problem* prob, const double* Xt, float* Y, void* stream);

/* P_k = A_k U (m x r, row-major per k at P[k*m*r]) and the inverse Gram
 * G_k^{-1} = (P_k^T P_k)^{-1} (r x r row-major FP64 at Lc[k*r*r]), the pieces of
 * (A_k U)^dagger in eq. (bk_LS).  flags[k] gets bit 1 (value 2) if G_k is not
 * positive definite; Lc then holds the identity for that k.  Asynchronous. */
int altgdmin_op_au(const altgdmin_problem* prob, const float* U, float* P, double* Lc,
                   int32_t* flags, void* stream);

/* tau IHT iterations of Alg. 2 per column on caller state.  project = 1:
 * z_k, M_k of the GDmin loop (needs P, Lc from altgdmin_op_au); project = 0:
 * M = A_k, z = y_k as in the initialisation.  has_support = 0 starts from
 * s = 0 (S_idx/S_val ignored on entry); so does a start whose rho values are
 * all zero (the step size then takes its support from HardThreshold(g), as
 * for s = 0).  S_idx/S_val are updated in place; with tau = 0 and no start
 * they become indices 0 .. rho - 1 with zero values.
 * G_out (optional, q x n) gets the gradient of the last iteration, mu_out
 * (optional, q) its step size. */
int altgdmin_op_iht(const altgdmin_problem* prob, int32_t project, const float* P, const double* Lc,
                    int32_t tau, int32_t has_support, int32_t* S_idx, float* S_val,
                    float* G_out, double* mu_out, int32_t* flags, void* stream);

/* LS and gradient pieces of one GDmin iteration for the given U (through P,
 * Lc) and S: b_k = (A_k U)^dagger (y_k - A_k s_k) -> Bt (q x r),
 * h_k = A_k^T (A_k (U b_k + s_k) - y_k) -> H (q x n), ||r_k||^2 -> rr (q, FP64). */
int altgdmin_op_lsgrad(const altgdmin_problem* prob, const float* P, const double* Lc,
                       const int32_t* S_idx, const float* S_val, float* Bt, float* H,
                       double* rr, int32_t* flags, void* stream);

/* Back-projection of the initialisation: L0t[k*n + j] = (A_k^T (y_k - A_k s_k))_j. */
int altgdmin_op_backproject(const altgdmin_problem* prob, const int32_t* S_idx, const float* S_val,
                            float* L0t, void* stream);

/* Device scratch (bytes) that altgdmin_op_grad, altgdmin_op_qr_step and
 * altgdmin_op_subspace need for sizes (n, q, r).  Host call. */
int altgdmin_op_scratch_bytes(int32_t n, int32_t q, int32_t r, size_t* bytes);

/* grad_U f = sum_k h_k b_k^T (n x r row-major), summed in a fixed order (Sec. 2.1). */
int altgdmin_op_grad(const float* H, const float* Bt, int32_t n, int32_t q, int32_t r,
                     float* grad, void* scratch, size_t scratch_bytes, void* stream);

/* Projected GD step: U_out = Q of the thin QR (positive diagonal R) of
 * U - eta*grad, by CholeskyQR2 with FP64 Gram and Cholesky.  If *eta_io <= 0
 * on entry (device double) it is first set to eta_c / ||grad||_2. */
int altgdmin_op_qr_step(const float* U, const float* grad, int32_t n, int32_t r, double eta_c,
                        double* eta_io, float* U_out, void* scratch, size_t scratch_bytes,
                        void* stream);

/* Automatic rank (Sec. 2.6, "b% energy threshold"): with sigma_1 >= sigma_2 >= ...
 * the singular values of L_0 (n x q, given as L0t q x n row-major) and
 * K = max(1, floor(min(n, q, m) / 10)), r is the smallest k with
 * sum_{i<=k} sigma_i^2 >= energy * sum_{i<=K} sigma_i^2.  The K values are Ritz
 * values of `iters` steps of a block subspace iteration with b = min(K + 8, 88,
 * n, q) columns (CholeskyQR2 with FP64 Grams), from a fixed orthonormal start;
 * ENOTBUILT when K > 88.  r_out: device int32; sv_out (optional): device
 * double[K], descending.  Scratch: altgdmin_op_rank_scratch_bytes.  Asynchronous. */
int altgdmin_op_rank_scratch_bytes(int32_t n, int32_t q, int32_t m, size_t* bytes);
int altgdmin_op_rank(const float* L0t, int32_t n, int32_t q, int32_t m, double energy, int32_t iters,
                     int32_t* r_out, double* sv_out, void* scratch, size_t scratch_bytes, void* stream);

/* Top-r left singular subspace of L0 (n x q, given as L0t q x n) by subspace
 * iteration from U_start (n x r), at most `iters` iterations or until the
 * change drops to tol.  U_out: n x r orthonormal.  iters_out (optional, device
 * int32) gets the count used. */
int altgdmin_op_subspace(const float* L0t, int32_t n, int32_t q, int32_t r, const float* U_start,
                         int32_t iters, double tol, float* U_out, int32_t* iters_out,
                         void* scratch, size_t scratch_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Allocation-free entry point, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).
 * ---------------------------------------------------------------------- */

/* Bytes of the library's static device scratch array (one per GPU, held until the process ends). */
#define ALTGDMIN_STATIC_SCRATCH_BYTES (16u << 20)

/* altgdmin_op_subspace without the scratch argument: its scratch (the
 * altgdmin_op_scratch_bytes(n, q, r) bytes) is the library's static device
 * array of ALTGDMIN_STATIC_SCRATCH_BYTES on the current GPU, so the call
 * allocates nothing; results are those of altgdmin_op_subspace bit for bit.
 * Sizes whose scratch exceeds the array are rejected (ALTGDMIN_ENOWS).  The
 * array is shared by every call on that GPU and keeps the last call's contents
 * (each call rewrites what it reads): calls that overlap on one GPU -- on
 * different streams, or from host threads without ordering -- race and must
 * be serialised by the caller.  Asynchronous on `stream`. */
int altgdmin_op_subspace_noalloc(const float* L0t, int32_t n, int32_t q, int32_t r, const float* U_start,
                                 int32_t iters, double tol, float* U_out, int32_t* iters_out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* ALTGDMIN_H */
