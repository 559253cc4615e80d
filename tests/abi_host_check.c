/* Host-only exercise of the C ABI for the sanitizer build (no GPU calls):
 * argument validation, workspace and scratch sizes, error strings, and the
 * entry points that must refuse null handles or streams before touching a
 * device.  Prints "ok" and exits 0 when every check holds. */
#include <stdio.h>
#include <string.h>
#include "altgdmin.h"

#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      printf("failed: %s (line %d): %s\n", #c, __LINE__, altgdmin_last_error()); \
      return 1;                                                    \
    }                                                              \
  } while (0)

static altgdmin_problem problem(void) {
  altgdmin_problem p;
  memset(&p, 0, sizeof(p));
  p.n = 1000; p.q = 1000; p.m = 400; p.r = 10; p.rho = 50;
  p.a_format = ALTGDMIN_A_F32;
  p.A = (const void*)(1ull << 20); p.Y = (const float*)(1ull << 24);
  p.lda = 400; p.a_stride_k = 400 * 1000; p.ldy = 400;
  return p;
}

int main(void) {
  altgdmin_params par;
  altgdmin_default_params(&par);
  size_t b = 0, b0 = 0;
  altgdmin_problem p = problem();
  CHECK(altgdmin_workspace_bytes(&p, &par, &b) == ALTGDMIN_OK && b > 0);
  p.r = 0;   /* automatic rank */
  CHECK(altgdmin_workspace_bytes(&p, &par, &b0) == ALTGDMIN_OK && b0 > 0);
  p = problem(); p.r = 17;
  CHECK(altgdmin_workspace_bytes(&p, &par, &b) == ALTGDMIN_ENOTBUILT);
  p = problem(); p.lda = 402;
  CHECK(altgdmin_workspace_bytes(&p, &par, &b) == ALTGDMIN_EINVAL);
  p = problem(); p.Y = NULL;
  CHECK(altgdmin_workspace_bytes(&p, &par, &b) == ALTGDMIN_EINVAL);
  CHECK(altgdmin_workspace_bytes(NULL, &par, &b) == ALTGDMIN_EINVAL);
  CHECK(strlen(altgdmin_last_error()) > 0);
  p = problem(); p.rho = 1001;
  CHECK(altgdmin_workspace_bytes(&p, &par, &b) == ALTGDMIN_EINVAL);
  p = problem(); p.r = -1;
  CHECK(altgdmin_workspace_bytes(&p, &par, &b) == ALTGDMIN_EINVAL);
  p = problem(); p.a_stride_k = 100;
  CHECK(altgdmin_workspace_bytes(&p, &par, &b) == ALTGDMIN_EINVAL);
  p = problem(); p.a_format = 7;
  CHECK(altgdmin_workspace_bytes(&p, &par, &b) == ALTGDMIN_EINVAL);
  p = problem(); p.a_format = ALTGDMIN_A_BF16X2;   /* lo plane missing */
  CHECK(altgdmin_workspace_bytes(&p, &par, &b) == ALTGDMIN_EINVAL);
  p = problem(); p.a_format = ALTGDMIN_A_PHILOX; p.A = NULL;   /* normal table missing */
  CHECK(altgdmin_workspace_bytes(&p, &par, &b) == ALTGDMIN_EINVAL);
  p = problem(); par.tau = -1;
  CHECK(altgdmin_workspace_bytes(&p, &par, &b) == ALTGDMIN_EINVAL);
  altgdmin_default_params(&par);
  p = problem();
  /* partial Fourier: the 96 x 96 frames, a generic frame, and sizes beyond the limits */
  altgdmin_problem f;
  memset(&f, 0, sizeof(f));
  f.n = 96 * 96; f.q = 64; f.m = 1536; f.r = 6; f.rho = 184; f.n1 = 96; f.n2 = 96;
  f.a_format = ALTGDMIN_A_PFOURIER; f.fourier_mask = (const int32_t*)(1ull << 20);
  f.Y = (const float*)(1ull << 24); f.ldy = 1536;
  CHECK(altgdmin_workspace_bytes(&f, &par, &b) == ALTGDMIN_OK);
  f.n = 400; f.n1 = 20; f.n2 = 20; f.m = 100; f.ldy = 100; f.rho = 5; f.r = 4;
  CHECK(altgdmin_workspace_bytes(&f, &par, &b) == ALTGDMIN_OK);
  f.n = 2 * 4096; f.n1 = 2; f.n2 = 4096;
  CHECK(altgdmin_workspace_bytes(&f, &par, &b) == ALTGDMIN_ENOTBUILT);
  f.n = 401; f.n1 = 20; f.n2 = 20;   /* n != n1 * n2 */
  CHECK(altgdmin_workspace_bytes(&f, &par, &b) == ALTGDMIN_EINVAL);
  f.n = 400; f.fourier_mask = NULL;
  CHECK(altgdmin_workspace_bytes(&f, &par, &b) == ALTGDMIN_EINVAL);
  /* scratch sizes */
  CHECK(altgdmin_op_scratch_bytes(1000, 1000, 10, &b) == ALTGDMIN_OK && b > 0);
  CHECK(altgdmin_op_scratch_bytes(0, 1000, 10, &b) == ALTGDMIN_EINVAL);
  CHECK(altgdmin_op_rank_scratch_bytes(1000, 1000, 400, &b) == ALTGDMIN_OK && b > 0);
  CHECK(altgdmin_op_rank_scratch_bytes(2000, 2000, 1000, &b) == ALTGDMIN_ENOTBUILT);
  /* null handles, null streams: refused before any device call */
  CHECK(altgdmin_step(NULL, 1, (void*)1) == ALTGDMIN_EINVAL);
  CHECK(altgdmin_state_bytes(NULL, &b) == ALTGDMIN_EINVAL);
  CHECK(altgdmin_get_state(NULL, (void*)256, 256, (void*)1) == ALTGDMIN_EINVAL);
  CHECK(altgdmin_set_state(NULL, (void*)256, 256, (void*)1) == ALTGDMIN_EINVAL);
  CHECK(altgdmin_tuning(NULL, NULL, NULL) == ALTGDMIN_EINVAL);
  CHECK(altgdmin_status_many(NULL, 1, (void*)1, NULL) == ALTGDMIN_EINVAL);
  CHECK(altgdmin_destroy(NULL) == ALTGDMIN_OK);
  altgdmin_handle* h = NULL;
  CHECK(altgdmin_init(&p, &par, (void*)(1ull << 30), b, NULL, &h) == ALTGDMIN_EINVAL && h == NULL);
  CHECK(altgdmin_op_subspace_noalloc((const float*)256, 300000, 1000, 16, NULL, 5, 1e-7, (float*)256, NULL,
                                     (void*)4096) == ALTGDMIN_ENOWS);
  for (int c = -6; c <= 2; ++c) CHECK(altgdmin_strerror(c) != NULL && strlen(altgdmin_strerror(c)) > 0);
  printf("ok\n");
  return 0;
}
