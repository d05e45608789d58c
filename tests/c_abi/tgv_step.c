/* A plain C11 user of liblbm (include/lbm.h), no Python: D3Q27, FP64
 * storage, a 32^3 periodic grid over [0, 2 pi)^3, initialised at rest density
 * with the Taylor-Green velocity u0 (sin x cos y cos z, -cos x sin y cos z, 0)
 * (Sec. 4.2), `steps` time steps (default 20), then the diagnostics and the
 * enstrophy; then a checkpoint to host memory (lbm_get_state), five more
 * steps, a restore (lbm_set_state) and the same five steps again, which must
 * give the same bits.  Buffers come from hipMalloc; every call's status is
 * checked.  Prints one line: mass, kinetic energy before and after,
 * enstrophy, whether the resumed run matched bit for bit and whether the
 * five steps changed the state.
 * Test infrastructure: tests/test_gpu_c_abi.py runs it and compares with the
 * same run through the Python binding. */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbm.h"

#define LBM_TRY(x)                                                                             \
  do {                                                                                         \
    int rc_ = (x);                                                                             \
    if (rc_ != LBM_OK) {                                                                       \
      fprintf(stderr, "%s: %s (%s)\n", #x, lbm_strerror(rc_), lbm_last_error());              \
      return 1;                                                                                \
    }                                                                                          \
  } while (0)
#define HIP_TRY(x)                                                                             \
  do {                                                                                         \
    hipError_t e_ = (x);                                                                       \
    if (e_ != hipSuccess) {                                                                    \
      fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                                  \
      return 1;                                                                                \
    }                                                                                          \
  } while (0)

int main(int argc, char **argv) {
  const int64_t n = 32, grid[3] = {n, n, n}, ncell = n * n * n;
  const int steps = argc > 1 ? atoi(argv[1]) : 20;
  const double pi = 3.14159265358979323846;
  const double u0 = 0.05, cs = 1.0, tau = 0.6;
  lbm_options opt;
  lbm_default_options(&opt);
  opt.storage = LBM_F64;
  opt.stencil = 4;
  opt.dx = 2.0 * pi / (double)n;
  opt.cs = cs;
  opt.dt = 0.4 * opt.dx / (sqrt(3.0) * cs); /* fastest component moves 0.4 cells */
  lbm_ctx *ctx = NULL;
  LBM_TRY(lbm_create(&ctx, LBM_D3Q27, grid, tau, 2, &opt));
  const size_t bytes = lbm_state_bytes(ctx);
  void *b0 = NULL, *b1 = NULL, *drho = NULL, *du = NULL, *dv = NULL;
  HIP_TRY(hipMalloc(&b0, bytes));
  HIP_TRY(hipMalloc(&b1, bytes));
  HIP_TRY(hipMalloc(&drho, sizeof(double) * (size_t)ncell));
  HIP_TRY(hipMalloc(&du, sizeof(double) * 3 * (size_t)ncell));
  HIP_TRY(hipMalloc(&dv, sizeof(double) * 3 * (size_t)ncell));
  LBM_TRY(lbm_bind(ctx, b0, b1));
  double *rho = malloc(sizeof(double) * (size_t)ncell), *u = malloc(sizeof(double) * 3 * (size_t)ncell);
  if (!rho || !u) return 1;
  for (int64_t z = 0; z < n; ++z)
    for (int64_t y = 0; y < n; ++y)
      for (int64_t x = 0; x < n; ++x) {
        const int64_t e = (z * n + y) * n + x;
        const double X = x * opt.dx, Y = y * opt.dx, Z = z * opt.dx;
        rho[e] = 1.0;
        u[e] = u0 * sin(X) * cos(Y) * cos(Z);
        u[ncell + e] = -u0 * cos(X) * sin(Y) * cos(Z);
        u[2 * ncell + e] = 0.0;
      }
  HIP_TRY(hipMemcpy(drho, rho, sizeof(double) * (size_t)ncell, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(du, u, sizeof(double) * 3 * (size_t)ncell, hipMemcpyHostToDevice));
  LBM_TRY(lbm_init_equilibrium(ctx, drho, du, NULL));
  lbm_diag d0, d1;
  LBM_TRY(lbm_moments(ctx, NULL, NULL, NULL, NULL, &d0));
  LBM_TRY(lbm_step(ctx, steps));
  LBM_TRY(lbm_moments(ctx, NULL, NULL, dv, NULL, &d1));
  double ens = 0.0;
  LBM_TRY(lbm_enstrophy(ctx, dv, 8, &ens));
  unsigned char *ck = malloc(bytes), *s1 = malloc(bytes), *s2 = malloc(bytes);
  if (!ck || !s1 || !s2) return 1;
  LBM_TRY(lbm_get_state(ctx, ck));
  LBM_TRY(lbm_step(ctx, 5));
  LBM_TRY(lbm_get_state(ctx, s1));
  LBM_TRY(lbm_set_state(ctx, ck));
  LBM_TRY(lbm_step(ctx, 5));
  LBM_TRY(lbm_get_state(ctx, s2));
  const int same = memcmp(s1, s2, bytes) == 0, moved = memcmp(ck, s1, bytes) != 0;
  printf("mass %.17g ke0 %.17g ke %.17g enstrophy %.17g resumed_identical %d stepped %d\n", d1.mass, d0.ke,
         d1.ke, ens, same, moved);
  free(ck);
  free(s1);
  free(s2);
  LBM_TRY(lbm_destroy(ctx));
  HIP_TRY(hipFree(b0));
  HIP_TRY(hipFree(b1));
  HIP_TRY(hipFree(drho));
  HIP_TRY(hipFree(du));
  HIP_TRY(hipFree(dv));
  free(rho);
  free(u);
  return 0;
}
