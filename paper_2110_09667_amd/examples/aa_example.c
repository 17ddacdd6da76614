/* aa_example.c -- the C ABI on its own, from C: Anderson acceleration of the
 * 1D Poisson fixed-point map G(x) = x - omega (A x - b), A = tridiag(-1, 2,
 * -1) / h^2 on n points, b ~ U[-1, 1] from the library's seeded generator.
 * The caller owns every device buffer (hipMalloc here); the library only
 * carves the workspace it is given.
 *
 * usage: aa_example OUT N M VARIANT ITERS OMEGA H
 *   writes the final iterate (N doubles, native byte order) to OUT and prints
 *   one line per 10 iterations with ||f_i|| / ||f_0||.  Exit status 0 on
 *   success. */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "aa.h"

#define CHECK_HIP(x)                                                       \
  do {                                                                     \
    hipError_t e_ = (x);                                                   \
    if (e_ != hipSuccess) {                                                \
      fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));              \
      return 2;                                                            \
    }                                                                      \
  } while (0)
#define CHECK_AA(x)                                                        \
  do {                                                                     \
    aa_status s_ = (x);                                                    \
    if (s_ != AA_OK) {                                                     \
      fprintf(stderr, "%s: status %d\n", #x, (int)s_);                     \
      return 3;                                                            \
    }                                                                      \
  } while (0)

int main(int argc, char **argv) {
  if (argc != 8) {
    fprintf(stderr, "usage: %s OUT N M VARIANT ITERS OMEGA H\n", argv[0]);
    return 1;
  }
  const char *out = argv[1];
  const int64_t n = atoll(argv[2]);
  const int m = atoi(argv[3]), variant = atoi(argv[4]), iters = atoi(argv[5]);
  const double omega = atof(argv[6]), h = atof(argv[7]);
  hipStream_t st;
  CHECK_HIP(hipStreamCreate(&st));
  size_t bytes = 0;
  CHECK_AA(aa_workspace_size(n, m, variant, 0, &bytes));
  void *ws = NULL;
  double *b = NULL, *x = NULL, *g = NULL;
  CHECK_HIP(hipMalloc(&ws, bytes));
  CHECK_HIP(hipMalloc((void **)&b, n * sizeof(double)));
  CHECK_HIP(hipMalloc((void **)&x, n * sizeof(double)));
  CHECK_HIP(hipMalloc((void **)&g, n * sizeof(double)));
  CHECK_HIP(hipMemsetAsync(x, 0, n * sizeof(double), st));
  CHECK_AA(aa_fill_uniform(b, n, 1, 0, 0, -1.0, 1.0, st));
  aa_ctx *ctx = NULL;
  CHECK_AA(aa_init(&ctx, n, m, variant, 0, ws, bytes, st));
  for (int i = 0; i <= iters; ++i) {
    CHECK_AA(aa_problem_apply(1, n, h, omega, 0.0, b, x, g, st));
    CHECK_AA(aa_step(ctx, x, g, x));
    if (i > 0 && i % 10 == 0) {
      aa_info info;
      CHECK_AA(aa_get_info(ctx, &info));
      printf("iteration %d: ||f|| / ||f_0|| = %.6e (k = %d)\n", i,
             info.res_norm / info.res0_norm, info.k);
    }
  }
  double *hx = (double *)malloc(n * sizeof(double));
  if (!hx) return 4;
  CHECK_HIP(hipStreamSynchronize(st));
  CHECK_HIP(hipMemcpy(hx, x, n * sizeof(double), hipMemcpyDeviceToHost));
  FILE *fh = fopen(out, "wb");
  if (!fh || fwrite(hx, sizeof(double), (size_t)n, fh) != (size_t)n) return 5;
  fclose(fh);
  free(hx);
  CHECK_AA(aa_destroy(ctx));
  CHECK_HIP(hipFree(ws));
  CHECK_HIP(hipFree(b));
  CHECK_HIP(hipFree(x));
  CHECK_HIP(hipFree(g));
  CHECK_HIP(hipStreamDestroy(st));
  printf("%s\n", aa_version());
  return 0;
}
