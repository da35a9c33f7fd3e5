/* Drives every entry point of the CPU oracle on small grids so that a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer checks its memory
 * accesses and arithmetic: guard fill, predictor-corrector step (also per
 * block with face fluxes), SSP Runge-Kutta steps of order 2 and 3, the
 * corner-transport-upwind step and both CFL rules, on 8^3 blocks with mixed
 * boundaries and a one-block grid.  Exits non-zero on a non-finite result. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "hydro_oracle.h"

static unsigned long long rng_state = 88172645463325252ull;
static double urand(void) { /* xorshift64 */
  rng_state ^= rng_state << 13;
  rng_state ^= rng_state >> 7;
  rng_state ^= rng_state << 17;
  return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static void random_state(const oracle_grid *g, double *U) {
  const int P = g->n + 2 * g->ng;
  const long nblk = (long)g->nb[0] * g->nb[1] * g->nb[2];
  const long vs = (long)P * P * P;
  for (long b = 0; b < nblk; ++b)
    for (long c = 0; c < vs; ++c) {
      double *u = U + b * 5 * vs + c;
      const double rho = 0.5 + urand(), p = 0.5 + urand();
      const double vx = urand() - 0.5, vy = urand() - 0.5, vz = urand() - 0.5;
      u[0] = rho;
      u[vs] = rho * vx;
      u[2 * vs] = rho * vy;
      u[3 * vs] = rho * vz;
      u[4 * vs] = p / (g->gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz);
    }
}

static int check(const char *what, const oracle_grid *g, const double *U) {
  const size_t n = oracle_block_doubles(g) * (size_t)g->nb[0] * g->nb[1] * g->nb[2];
  for (size_t i = 0; i < n; ++i)
    if (!isfinite(U[i])) {
      fprintf(stderr, "%s: non-finite value at %zu\n", what, i);
      return 1;
    }
  return 0;
}

static int run(const oracle_grid *g) {
  const long nblk = (long)g->nb[0] * g->nb[1] * g->nb[2];
  const size_t nd = oracle_block_doubles(g) * (size_t)nblk;
  double *U = malloc(nd * sizeof *U), *V = malloc(nd * sizeof *V);
  long cnt[ORACLE_NCNT] = {0, 0, 0};
  int bad = 0;
  if (!U || !V) return 1;
  random_state(g, U);
  oracle_fill_guards(g, U);
  const double dt = oracle_dt(g, U, 0.4);
  memcpy(V, U, nd * sizeof *U);
  oracle_step(g, U, V, dt, cnt);
  bad |= check("step", g, V);
  const int n = g->n;
  const size_t nf = (size_t)5 * (n + 1) * n * n;
  double *F0 = malloc(nf * sizeof *F0), *F1 = malloc(nf * sizeof *F1), *F2 = malloc(nf * sizeof *F2);
  double *Ob = malloc(oracle_block_doubles(g) * sizeof *Ob);
  oracle_step_block_fluxes(g, U, nblk - 1, Ob, dt, F0, F1, F2, cnt);
  for (size_t i = 0; i < nf; ++i) bad |= !isfinite(F0[i]) || !isfinite(F1[i]) || !isfinite(F2[i]);
  for (int order = 2; order <= 3; ++order) {
    memcpy(V, U, nd * sizeof *U);
    bad |= oracle_step_rk(g, U, V, dt, order, cnt) != 0;
    bad |= check(order == 2 ? "rk2" : "rk3", g, V);
  }
  const double dtc = oracle_dt_ctu(g, U, 0.4);
  memcpy(V, U, nd * sizeof *U);
  oracle_step_ctu(g, U, V, dtc, cnt);
  bad |= check("ctu", g, V);
  printf("grid %dx%dx%d of %d^3: dt %.6g, ctu dt %.6g, events %ld %ld %ld\n", g->nb[0], g->nb[1], g->nb[2], n,
         dt, dtc, cnt[0], cnt[1], cnt[2]);
  free(F0);
  free(F1);
  free(F2);
  free(Ob);
  free(U);
  free(V);
  return bad;
}

int main(void) {
  oracle_set_threads(2);
  oracle_grid a = {8, 4, {2, 1, 3}, {0.1, 0.12, 0.08}, {ORACLE_BC_OUTFLOW, ORACLE_BC_PERIODIC, ORACLE_BC_OUTFLOW},
                   1.4, 1e-10};
  oracle_grid b = {8, 4, {1, 1, 1}, {0.1, 0.1, 0.1}, {ORACLE_BC_PERIODIC, ORACLE_BC_PERIODIC, ORACLE_BC_PERIODIC},
                   5.0 / 3.0, 1e-10};
  int bad = run(&a) | run(&b);
  if (oracle_cons_to_prim((const double[5]){1.0, 0.1, 0.2, 0.3, 2.0}, 1.4, 1e-10, (double[5]){0}) < 0) bad = 1;
  printf(bad ? "FAILED\n" : "ok\n");
  return bad;
}
