/* Sanitizer driver for the FP64 oracle: a small 2D and 3D scene stepped
 * forward and backward, a checkpoint-free rollout with its reverse pass, and
 * the argument and domain errors.  Built with -fsanitize=address,undefined
 * by tests/test_sanitizers.py; any report fails the run. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/mpm_oracle.h"

static double frand(unsigned *s) {
  *s = *s * 1664525u + 1013904223u;
  return (double)(*s >> 8) / 16777216.0;
}

static int run(int dim, int n, int N, int T) {
  const int d2 = dim * dim;
  orc_scene sc;
  memset(&sc, 0, sizeof sc);
  sc.dim = dim;
  sc.n_grid = n;
  sc.n_particles = N;
  sc.n_act = 2;
  sc.wall = 3;
  sc.dt = 1e-4;
  sc.E = 10.0;
  sc.nu = 0.3;
  sc.rho = 1.0;
  sc.V0 = pow(0.5 / n, dim);
  sc.gravity[1] = -9.8;
  sc.act_axis[1] = 1.0;
  double *x = calloc((size_t)dim * N, sizeof(double));
  double *v = calloc((size_t)dim * N, sizeof(double));
  double *C = calloc((size_t)d2 * N, sizeof(double));
  double *F = calloc((size_t)d2 * N, sizeof(double));
  double *x1 = calloc((size_t)dim * N, sizeof(double));
  double *v1 = calloc((size_t)dim * N, sizeof(double));
  double *C1 = calloc((size_t)d2 * N, sizeof(double));
  double *F1 = calloc((size_t)d2 * N, sizeof(double));
  double *gx = calloc((size_t)dim * N, sizeof(double));
  double *gv = calloc((size_t)dim * N, sizeof(double));
  double *gC = calloc((size_t)d2 * N, sizeof(double));
  double *gF = calloc((size_t)d2 * N, sizeof(double));
  double *act = calloc((size_t)T * 2, sizeof(double));
  double *gact = calloc((size_t)T * 2, sizeof(double));
  int32_t *ids = calloc((size_t)N, sizeof(int32_t));
  unsigned seed = 12345u + (unsigned)dim;
  for (int p = 0; p < N; ++p) {
    for (int a = 0; a < dim; ++a) {
      x[a * N + p] = 0.35 + 0.3 * frand(&seed);
      v[a * N + p] = 0.2 * (frand(&seed) - 0.5);
      gx[a * N + p] = frand(&seed) / N;
    }
    for (int k = 0; k < d2; ++k) {
      C[k * N + p] = 0.5 * (frand(&seed) - 0.5);
      F[k * N + p] = (k % (dim + 1) == 0 ? 1.0 : 0.0) + 0.02 * (frand(&seed) - 0.5);
    }
    ids[p] = (p % 3) - 1;
  }
  for (int k = 0; k < 2 * T; ++k) act[k] = frand(&seed) - 0.5;
  int rc = orc_step_fwd(&sc, ids, act, x, v, C, F, x1, v1, C1, F1);
  if (rc) return 10 + rc;
  rc = orc_step_bwd(&sc, ids, act, x, v, C, F, gx, gv, gC, gF, gx, gv, gC, gF, gact);
  if (rc) return 20 + rc;
  memset(gv, 0, sizeof(double) * dim * N);
  memset(gC, 0, sizeof(double) * d2 * N);
  memset(gF, 0, sizeof(double) * d2 * N);
  memset(gact, 0, sizeof(double) * 2 * T);
  rc = orc_rollout(&sc, ids, T, act, x, v, C, F, x1, v1, C1, F1, gx, gv, gC, gF, gx, gv, gC,
                   gF, gact);
  if (rc) return 30 + rc;
  /* errors: a bad argument, a particle whose stencil leaves the grid */
  sc.dim = 4;
  if (orc_step_fwd(&sc, ids, act, x, v, C, F, x1, v1, C1, F1) != ORC_ERR_ARG) return 40;
  sc.dim = dim;
  x[0] = 0.1 / n;
  if (orc_step_fwd(&sc, ids, act, x, v, C, F, x1, v1, C1, F1) != ORC_ERR_DOMAIN) return 41;
  free(x); free(v); free(C); free(F); free(x1); free(v1); free(C1); free(F1);
  free(gx); free(gv); free(gC); free(gF); free(act); free(gact); free(ids);
  return 0;
}

int main(void) {
  int rc = run(2, 16, 40, 6);
  if (!rc) rc = run(3, 12, 24, 4);
  printf("oracle sanitizer run: %d\n", rc);
  return rc;
}
