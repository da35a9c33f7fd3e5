/*
 * Plain FP64 CPU oracle of the unsplit second-order Godunov hydro step.
 * TEST INFRASTRUCTURE ONLY: see hydro_oracle.h for scope, layout and the
 * readings of the method.  Compiled with -O2 -fno-fast-math -ffp-contract=off
 * so that every operation below is one IEEE-754 double operation in the
 * written order.  Loops are the definition written out; the only parallelism
 * is an OpenMP loop over independent blocks, which changes no arithmetic.
 */
#include "hydro_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* Host threads of the OpenMP loops over blocks (timing of the baseline). */
void oracle_set_threads(int n) {
  if (n > 0) omp_set_num_threads(n);
}

int oracle_max_threads(void) { return omp_get_max_threads(); }

/* ---- layout ------------------------------------------------------------ */

static int edge(const oracle_grid *g) { return g->n + 2 * g->ng; }

size_t oracle_block_doubles(const oracle_grid *g) {
  size_t P = (size_t)edge(g);
  return 5 * P * P * P;
}

/* Offset of (var, i, j, k) inside a block; i, j, k are interior-relative
 * (interior cells are 0..n-1, guards are -ng..-1 and n..n+ng-1). */
static size_t at(const oracle_grid *g, int var, int i, int j, int k) {
  size_t P = (size_t)edge(g);
  return (((size_t)var * P + (size_t)(k + g->ng)) * P + (size_t)(j + g->ng)) * P + (size_t)(i + g->ng);
}

/* ---- a1: same-level guard fill (§2: block-by-block update with boundary
 *      data supplied by the Grid unit; reading: periodic = mod, outflow =
 *      clamp, composed per axis) ----------------------------------------- */

static long map_index(long I, long N, int bc) {
  if (bc == ORACLE_BC_PERIODIC) {
    long r = I % N;
    return r < 0 ? r + N : r;
  }
  if (I < 0) return 0;
  if (I > N - 1) return N - 1;
  return I;
}

void oracle_fill_guards_block(const oracle_grid *g, double *U, long b) {
  const int n = g->n, ng = g->ng;
  const long nbx = g->nb[0], nby = g->nb[1];
  const long bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
  const long N[3] = {(long)g->nb[0] * n, (long)g->nb[1] * n, (long)g->nb[2] * n};
  const size_t bd = oracle_block_doubles(g);
  double *dst = U + (size_t)b * bd;
  for (int k = -ng; k < n + ng; ++k)
    for (int j = -ng; j < n + ng; ++j)
      for (int i = -ng; i < n + ng; ++i) {
        int interior = i >= 0 && i < n && j >= 0 && j < n && k >= 0 && k < n;
        if (interior) continue;
        long I = map_index(bx * n + i, N[0], g->bc[0]);
        long J = map_index(by * n + j, N[1], g->bc[1]);
        long K = map_index(bz * n + k, N[2], g->bc[2]);
        long sb = (I / n) + nbx * ((J / n) + nby * (K / n));
        const double *src = U + (size_t)sb * bd;
        for (int v = 0; v < 5; ++v)
          dst[at(g, v, i, j, k)] = src[at(g, v, (int)(I % n), (int)(J % n), (int)(K % n))];
      }
}

void oracle_fill_guards(const oracle_grid *g, double *U) {
  long nblk = (long)g->nb[0] * g->nb[1] * g->nb[2];
  /* Guards are written only from interiors, so blocks are independent. */
#pragma omp parallel for schedule(dynamic, 4)
  for (long b = 0; b < nblk; ++b) oracle_fill_guards_block(g, U, b);
}

/* ---- a2: conservative -> primitive, gamma-law EOS (§2.2, Equations of
 *      State: the perfect-gas EOS) --------------------------------------- */

int oracle_cons_to_prim(const double U[5], double gamma, double small_p, double W[5]) {
  double rho = U[0];
  double u = U[1] / rho;
  double v = U[2] / rho;
  double w = U[3] / rho;
  double kinetic = 0.5 * rho * ((u * u + v * v) + w * w);
  double p = (gamma - 1.0) * (U[4] - kinetic);
  int floored = 0;
  if (p < small_p) {
    p = small_p;
    floored = 1;
  }
  W[0] = rho;
  W[1] = u;
  W[2] = v;
  W[3] = w;
  W[4] = p;
  return floored;
}

/* ---- a3: van Leer harmonic slope ---------------------------------------- */

double oracle_van_leer(double dl, double dr) {
  double prod = dl * dr;
  if (prod > 0.0) return (2.0 * prod) / (dl + dr);
  return 0.0;
}

/* ---- a4: Euler flux and HLLC (§2: explicit methods for compressible flow
 *      with strong shocks; HLLC with Davis speeds and Batten's S*) ------- */

static double total_energy(const double W[5], double gamma) {
  return W[4] / (gamma - 1.0) + 0.5 * W[0] * ((W[1] * W[1] + W[2] * W[2]) + W[3] * W[3]);
}

void oracle_euler_flux(const double W[5], int d, double gamma, double F[5]) {
  double un = W[1 + d];
  double E = total_energy(W, gamma);
  double mass = W[0] * un;
  F[0] = mass;
  F[1] = mass * W[1];
  F[2] = mass * W[2];
  F[3] = mass * W[3];
  F[1 + d] += W[4];
  F[4] = un * (E + W[4]);
}

/* Conserved star state of side K (Toro's HLLC star state with the normal
 * velocity replaced by S*, tangential velocities kept). */
static void star_state(const double W[5], int d, double gamma, double S, double Sstar, double Us[5]) {
  double rho = W[0], un = W[1 + d], p = W[4];
  double E = total_energy(W, gamma);
  double factor = rho * (S - un) / (S - Sstar);
  Us[0] = factor;
  Us[1] = factor * W[1];
  Us[2] = factor * W[2];
  Us[3] = factor * W[3];
  Us[1 + d] = factor * Sstar;
  Us[4] = factor * (E / rho + (Sstar - un) * (Sstar + p / (rho * (S - un))));
}

static void prim_to_cons(const double W[5], double gamma, double U[5]) {
  U[0] = W[0];
  U[1] = W[0] * W[1];
  U[2] = W[0] * W[2];
  U[3] = W[0] * W[3];
  U[4] = total_energy(W, gamma);
}

void oracle_hllc(const double WL[5], const double WR[5], int d, double gamma, double F[5]) {
  double rL = WL[0], uL = WL[1 + d], pL = WL[4];
  double rR = WR[0], uR = WR[1 + d], pR = WR[4];
  double cL = sqrt(gamma * pL / rL);
  double cR = sqrt(gamma * pR / rR);
  double SL = (uL - cL < uR - cR) ? uL - cL : uR - cR;
  double SR = (uL + cL > uR + cR) ? uL + cL : uR + cR;
  double Sstar = (pR - pL + rL * uL * (SL - uL) - rR * uR * (SR - uR)) /
                 (rL * (SL - uL) - rR * (SR - uR));
  if (SL >= 0.0) {
    oracle_euler_flux(WL, d, gamma, F);
  } else if (Sstar >= 0.0) {
    double FK[5], UK[5], Us[5];
    oracle_euler_flux(WL, d, gamma, FK);
    prim_to_cons(WL, gamma, UK);
    star_state(WL, d, gamma, SL, Sstar, Us);
    for (int v = 0; v < 5; ++v) F[v] = FK[v] + SL * (Us[v] - UK[v]);
  } else if (SR > 0.0) {
    double FK[5], UK[5], Us[5];
    oracle_euler_flux(WR, d, gamma, FK);
    prim_to_cons(WR, gamma, UK);
    star_state(WR, d, gamma, SR, Sstar, Us);
    for (int v = 0; v < 5; ++v) F[v] = FK[v] + SR * (Us[v] - UK[v]);
  } else {
    oracle_euler_flux(WR, d, gamma, F);
  }
}

/* ---- a3 predictor: A_d(W) * dW, the primitive-form Euler Jacobian along d - */

static void jacobian_times(const double W[5], int d, double gamma, const double dW[5], double out[5]) {
  double rho = W[0], un = W[1 + d], p = W[4];
  out[0] = un * dW[0] + rho * dW[1 + d];
  out[1] = un * dW[1];
  out[2] = un * dW[2];
  out[3] = un * dW[3];
  out[1 + d] += dW[4] / rho;
  out[4] = gamma * p * dW[1 + d] + un * dW[4];
}

/* ---- one block: a2..a5 -------------------------------------------------
 * hancock = 1: the predictor-corrector step (§2.2 Hydrodynamics: predictor,
 * then corrector), face states extrapolated from the half-step predicted
 * centre.  hancock = 0: one method-of-lines stage of the SSP Runge-Kutta
 * solver (§2.2 Hydrodynamics), face states extrapolated from the cell centre
 * itself, and the result combined with a base state U0b when U0b != NULL:
 * Uo = a0*U0 + a1*(U - div F). */

static void update_block(const oracle_grid *g, const double *U, long b, double *Uo, double dt, int hancock,
                         const double *U0b, double a0, double a1, long cnt[ORACLE_NCNT], double *Fout[3]) {
  const int n = g->n, ng = g->ng, P = edge(g);
  const double gamma = g->gamma;
  const double lam[3] = {dt / g->dx[0], dt / g->dx[1], dt / g->dx[2]};
  const size_t bd = oracle_block_doubles(g);
  const double *Ub = U + (size_t)b * bd;
  /* Cells that need face states: interior plus one layer, i.e. -1..n per axis. */
  const int M = n + 2;
  size_t ncell = (size_t)P * P * P;
  size_t nm = (size_t)M * M * M;
  double *W = (double *)malloc(sizeof(double) * 5 * ncell);    /* primitives, all cells */
  double *S = (double *)malloc(sizeof(double) * 15 * nm);      /* slopes [d][var] */
  double *Wp = (double *)malloc(sizeof(double) * 5 * nm);      /* predicted centre */
  char *fb = (char *)malloc(nm);                               /* fallback flag */
  size_t nf = (size_t)(n + 1) * n * n;
  double *F[3];
  for (int d = 0; d < 3; ++d) F[d] = (double *)malloc(sizeof(double) * 5 * nf);

#define WI(i, j, k) (W + 5 * (((size_t)((k) + ng) * P + (size_t)((j) + ng)) * P + (size_t)((i) + ng)))
#define MI(i, j, k) ((((size_t)((k) + 1) * M + (size_t)((j) + 1)) * M + (size_t)((i) + 1)))

  /* a2: primitives of every stored cell; floor hits counted on the interior. */
  for (int k = -ng; k < n + ng; ++k)
    for (int j = -ng; j < n + ng; ++j)
      for (int i = -ng; i < n + ng; ++i) {
        double Uc[5];
        for (int v = 0; v < 5; ++v) Uc[v] = Ub[at(g, v, i, j, k)];
        int fl = oracle_cons_to_prim(Uc, gamma, g->small_p, WI(i, j, k));
        if (fl && i >= 0 && i < n && j >= 0 && j < n && k >= 0 && k < n) cnt[ORACLE_CNT_FLOOR]++;
      }

  /* a3: slopes, Hancock predictor, positivity check of the six face states. */
  for (int k = -1; k <= n; ++k)
    for (int j = -1; j <= n; ++j)
      for (int i = -1; i <= n; ++i) {
        const double *Wc = WI(i, j, k);
        double *Sc = S + 15 * MI(i, j, k);
        const int off[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        for (int d = 0; d < 3; ++d) {
          const double *Wm = WI(i - off[d][0], j - off[d][1], k - off[d][2]);
          const double *Wq = WI(i + off[d][0], j + off[d][1], k + off[d][2]);
          for (int v = 0; v < 5; ++v) Sc[5 * d + v] = oracle_van_leer(Wc[v] - Wm[v], Wq[v] - Wc[v]);
        }
        double *Wt = Wp + 5 * MI(i, j, k);
        if (hancock) {
          double A[3][5];
          for (int d = 0; d < 3; ++d) jacobian_times(Wc, d, gamma, Sc + 5 * d, A[d]);
          for (int v = 0; v < 5; ++v)
            Wt[v] = Wc[v] - 0.5 * ((lam[0] * A[0][v] + lam[1] * A[1][v]) + lam[2] * A[2][v]);
        } else {
          for (int v = 0; v < 5; ++v) Wt[v] = Wc[v];
        }
        int bad = 0;
        for (int d = 0; d < 3; ++d)
          for (int s = -1; s <= 1; s += 2) {
            double r = Wt[0] + 0.5 * s * Sc[5 * d + 0];
            double p = Wt[4] + 0.5 * s * Sc[5 * d + 4];
            if (!(r > 0.0) || !(p > 0.0)) bad = 1;
          }
        fb[MI(i, j, k)] = (char)bad;
        if (bad && i >= 0 && i < n && j >= 0 && j < n && k >= 0 && k < n) cnt[ORACLE_CNT_FALLBACK]++;
      }

  /* a4: HLLC on every face of the interior; face (d, i, j, k) lies on the low
   * side of cell (i, j, k) along d, with i (or j, k) running 0..n. */
  for (int d = 0; d < 3; ++d) {
    const int ex = d == 0, ey = d == 1, ez = d == 2;
    const int ni = n + ex, nj = n + ey, nk = n + ez;
    for (int k = 0; k < nk; ++k)
      for (int j = 0; j < nj; ++j)
        for (int i = 0; i < ni; ++i) {
          int li = i - ex, lj = j - ey, lk = k - ez;
          double WL[5], WR[5];
          size_t mL = MI(li, lj, lk), mR = MI(i, j, k);
          for (int v = 0; v < 5; ++v) {
            WL[v] = fb[mL] ? WI(li, lj, lk)[v] : Wp[5 * mL + v] + 0.5 * S[15 * mL + 5 * d + v];
            WR[v] = fb[mR] ? WI(i, j, k)[v] : Wp[5 * mR + v] - 0.5 * S[15 * mR + 5 * d + v];
          }
          size_t f = ((size_t)k * nj + (size_t)j) * ni + (size_t)i;
          oracle_hllc(WL, WR, d, gamma, F[d] + 5 * f);
        }
  }

  /* a5: conservative update of the interior. */
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        size_t fx0 = ((size_t)k * n + j) * (n + 1) + i, fx1 = fx0 + 1;
        size_t fy0 = ((size_t)k * (n + 1) + j) * n + i, fy1 = fy0 + n;
        size_t fz0 = ((size_t)k * n + j) * n + i, fz1 = fz0 + (size_t)n * n;
        double Un[5];
        for (int v = 0; v < 5; ++v) {
          double div = (lam[0] * (F[0][5 * fx1 + v] - F[0][5 * fx0 + v]) +
                        lam[1] * (F[1][5 * fy1 + v] - F[1][5 * fy0 + v])) +
                       lam[2] * (F[2][5 * fz1 + v] - F[2][5 * fz0 + v]);
          Un[v] = Ub[at(g, v, i, j, k)] - div;
          if (U0b) Un[v] = a0 * U0b[at(g, v, i, j, k)] + a1 * Un[v];
          Uo[at(g, v, i, j, k)] = Un[v];
        }
        int ok = Un[0] > 0.0 && Un[4] > 0.0;
        for (int v = 0; v < 5; ++v) ok = ok && isfinite(Un[v]);
        if (!ok) cnt[ORACLE_CNT_NONPHYS]++;
      }
  if (Fout)
    for (int d = 0; d < 3; ++d)
      if (Fout[d]) memcpy(Fout[d], F[d], sizeof(double) * 5 * nf);
#undef WI
#undef MI
  free(W);
  free(S);
  free(Wp);
  free(fb);
  for (int d = 0; d < 3; ++d) free(F[d]);
}

void oracle_step_block(const oracle_grid *g, const double *U, long b, double *Uo, double dt,
                       long cnt[ORACLE_NCNT]) {
  update_block(g, U, b, Uo, dt, 1, NULL, 0.0, 0.0, cnt, NULL);
}

void oracle_step_block_fluxes(const oracle_grid *g, const double *U, long b, double *Uo, double dt,
                              double *Fx, double *Fy, double *Fz, long cnt[ORACLE_NCNT]) {
  double *Fout[3] = {Fx, Fy, Fz};
  update_block(g, U, b, Uo, dt, 1, NULL, 0.0, 0.0, cnt, Fout);
}

void oracle_stage_block(const oracle_grid *g, const double *U, long b, double *Uo, double dt,
                        const double *U0b, double a0, double a1, long cnt[ORACLE_NCNT]) {
  update_block(g, U, b, Uo, dt, 0, U0b, a0, a1, cnt, NULL);
}

void oracle_step(const oracle_grid *g, double *U, double *Unew, double dt, long cnt[ORACLE_NCNT]) {
  long nblk = (long)g->nb[0] * g->nb[1] * g->nb[2];
  oracle_fill_guards(g, U);
  long c0 = 0, c1 = 0, c2 = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : c0, c1, c2)
  for (long b = 0; b < nblk; ++b) {
    long c[ORACLE_NCNT] = {0, 0, 0};
    oracle_step_block(g, U, b, Unew + (size_t)b * oracle_block_doubles(g), dt, c);
    c0 += c[0];
    c1 += c[1];
    c2 += c[2];
  }
  cnt[ORACLE_CNT_FLOOR] += c0;
  cnt[ORACLE_CNT_FALLBACK] += c1;
  cnt[ORACLE_CNT_NONPHYS] += c2;
}

/* The listed blocks only (their guards filled first); block t's new interior
 * goes to out + t * oracle_block_doubles(g).  Blocks are independent, so an
 * OpenMP loop spreads them over the host cores. */
void oracle_step_block_list(const oracle_grid *g, double *U, const long *blocks, long nlist,
                            double *out, double dt, long cnt[ORACLE_NCNT]) {
  const size_t bd = oracle_block_doubles(g);
  long c0 = 0, c1 = 0, c2 = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : c0, c1, c2)
  for (long t = 0; t < nlist; ++t) {
    long c[ORACLE_NCNT] = {0, 0, 0};
    oracle_fill_guards_block(g, U, blocks[t]);
    oracle_step_block(g, U, blocks[t], out + (size_t)t * bd, dt, c);
    c0 += c[0];
    c1 += c[1];
    c2 += c[2];
  }
  cnt[ORACLE_CNT_FLOOR] += c0;
  cnt[ORACLE_CNT_FALLBACK] += c1;
  cnt[ORACLE_CNT_NONPHYS] += c2;
}

/* ---- f1: SSP Runge-Kutta method-of-lines step (§2.2 Hydrodynamics: the
 *      compressible solver with second- or third-order strong-stability-
 *      preserving Runge-Kutta time integration).  Shu-Osher form with
 *      L(U) = -div F(U) from the stage operator above:
 *        order 2: U1 = U + dt L(U);  U' = 1/2 U + 1/2 (U1 + dt L(U1))
 *        order 3: U1 = U + dt L(U);  U2 = 3/4 U + 1/4 (U1 + dt L(U1));
 *                 U' = 1/3 U + 2/3 (U2 + dt L(U2))
 *      Each stage fills the guards of its input first. ------------------- */

static void stage_all(const oracle_grid *g, double *Us, const double *U0, double a0, double a1, double *Uo,
                      double dt, long cnt[ORACLE_NCNT]) {
  long nblk = (long)g->nb[0] * g->nb[1] * g->nb[2];
  const size_t bd = oracle_block_doubles(g);
  oracle_fill_guards(g, Us);
  long c0 = 0, c1 = 0, c2 = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : c0, c1, c2)
  for (long b = 0; b < nblk; ++b) {
    long c[ORACLE_NCNT] = {0, 0, 0};
    update_block(g, Us, b, Uo + (size_t)b * bd, dt, 0, U0 ? U0 + (size_t)b * bd : NULL, a0, a1, c, NULL);
    c0 += c[0];
    c1 += c[1];
    c2 += c[2];
  }
  cnt[ORACLE_CNT_FLOOR] += c0;
  cnt[ORACLE_CNT_FALLBACK] += c1;
  cnt[ORACLE_CNT_NONPHYS] += c2;
}

int oracle_step_rk(const oracle_grid *g, double *U, double *Unew, double dt, int order, long cnt[ORACLE_NCNT]) {
  if (order != 2 && order != 3) return -1;
  long nblk = (long)g->nb[0] * g->nb[1] * g->nb[2];
  size_t total = (size_t)nblk * oracle_block_doubles(g);
  double *U1 = (double *)calloc(total, sizeof(double));
  double *U2 = order == 3 ? (double *)calloc(total, sizeof(double)) : NULL;
  if (!U1 || (order == 3 && !U2)) {
    free(U1);
    free(U2);
    return -2;
  }
  stage_all(g, U, NULL, 0.0, 0.0, U1, dt, cnt);
  if (order == 2) {
    stage_all(g, U1, U, 0.5, 0.5, Unew, dt, cnt);
  } else {
    stage_all(g, U1, U, 0.75, 0.25, U2, dt, cnt);
    stage_all(g, U2, U, 1.0 / 3.0, 2.0 / 3.0, Unew, dt, cnt);
  }
  free(U1);
  free(U2);
  return 0;
}

/* ---- f2: corner-transport-upwind (CTU) unsplit step ----------------------
 * §2.2 Hydrodynamics names the unsplit predictor-corrector solver; its
 * corner-coupled form is taken here: the three-dimensional corner transport
 * upwind scheme with twelve Riemann solves per cell (Colella 1990; Saltzman
 * 1994; the hydrodynamic part of Gardiner & Stone 2008), on the same
 * ingredients (EOS, van Leer slopes on primitives, HLLC):
 *   1. normal predictor, each direction d alone: W_d = W - (lam_d/2) A_d D_d,
 *      face states W_d -+ D_d/2 (low / high face of the cell); first-order
 *      fallback when any of the six has rho <= 0 or p <= 0;
 *   2. 1-D fluxes F1_d at every d-face from the normal face states;
 *   3. corner states: the conserved normal face state of direction d minus
 *      lam_t/3 times the difference of F1_t over the cell, for each
 *      transverse t; corner fluxes F_{d|t} from them;
 *   4. final states: the conserved normal face state minus lam_t/2 times the
 *      difference of F_{t|u} and lam_u/2 times that of F_{u|t} over the cell
 *      ({t, u} the transverse pair); final fluxes;
 *   5. the conservative update.
 * A corrected state with rho <= 0 or p <= 0 falls back to the normal face
 * state it came from (counted as a fallback).  dt uses the per-direction
 * CFL rule (oracle_dt_ctu). */

/* Primitive of a corrected conserved state; 0 when it is not physical. */
static int corrected_prim(const double U[5], double gamma, double W[5]) {
  double rho = U[0];
  if (!(rho > 0.0)) return 0;
  double u = U[1] / rho, v = U[2] / rho, w = U[3] / rho;
  double p = (gamma - 1.0) * (U[4] - 0.5 * rho * ((u * u + v * v) + w * w));
  if (!(p > 0.0)) return 0;
  W[0] = rho;
  W[1] = u;
  W[2] = v;
  W[3] = w;
  W[4] = p;
  return 1;
}

/* Characteristic tracing of the normal predictor (Colella 1990; the
 * upwind-projection form of Stone et al. 2008, §4.2): the primitive slope S
 * along d is split over the right eigenvectors of the primitive Jacobian
 * A_d(W), S = sum_k beta_k R_k with beta_k = L_k . S, and each face keeps
 * only the waves that move toward it during the step:
 *   high face: W + sum_{lambda_k > 0} (1 - lam lambda_k)/2 beta_k R_k
 *   low face:  W - sum_{lambda_k < 0} (1 + lam lambda_k)/2 beta_k R_k
 * (lam = dt/dx_d).  With c = sqrt(gamma p / rho) and u the normal velocity
 * the waves of A_d in (rho, u_n, u_t1, u_t2, p) are
 *   lambda = u - c:  beta = (dp/c^2 - rho du_n/c)/2,  R = (1, -c/rho, 0, 0, c^2)
 *   lambda = u:      the entropy and shear waves, beta R =
 *                    (drho - dp/c^2, 0, du_t1, du_t2, 0)
 *   lambda = u + c:  beta = (dp/c^2 + rho du_n/c)/2,  R = (1, c/rho, 0, 0, c^2)
 * (vector slots in the solver's order: normal velocity in slot 1 + d). */
void oracle_trace_faces(const double W[5], const double S[5], int d, double lam, double gamma, double lo[5],
                        double hi[5]) {
  const double rho = W[0], un = W[1 + d], p = W[4];
  const double c = sqrt(gamma * p / rho);
  double wave[3][5], speed[3];
  for (int k = 0; k < 3; ++k)
    for (int v = 0; v < 5; ++v) wave[k][v] = 0.0;
  /* the acoustic waves, beta_k R_k */
  const double bm = 0.5 * (S[4] / (c * c) - rho * S[1 + d] / c);
  const double bp = 0.5 * (S[4] / (c * c) + rho * S[1 + d] / c);
  wave[0][0] = bm;
  wave[0][1 + d] = -bm * c / rho;
  wave[0][4] = bm * c * c;
  wave[2][0] = bp;
  wave[2][1 + d] = bp * c / rho;
  wave[2][4] = bp * c * c;
  /* entropy and shear waves together */
  for (int v = 1; v < 4; ++v)
    if (v != 1 + d) wave[1][v] = S[v];
  wave[1][0] = S[0] - S[4] / (c * c);
  speed[0] = un - c;
  speed[1] = un;
  speed[2] = un + c;
  for (int v = 0; v < 5; ++v) {
    hi[v] = W[v];
    lo[v] = W[v];
  }
  for (int k = 0; k < 3; ++k) {
    if (speed[k] > 0.0)
      for (int v = 0; v < 5; ++v) hi[v] += 0.5 * (1.0 - lam * speed[k]) * wave[k][v];
    if (speed[k] < 0.0)
      for (int v = 0; v < 5; ++v) lo[v] -= 0.5 * (1.0 + lam * speed[k]) * wave[k][v];
  }
}

/* trace = 1: the normal predictor traces characteristics
 * (oracle_trace_faces); 0: primitive-form half step W_d = W - lam_d/2 A_d S_d
 * with face states W_d -+ S_d/2. */
static void ctu_block(const oracle_grid *g, const double *U, long b, double *Uo, double dt, int trace,
                      long cnt[ORACLE_NCNT]) {
  const int n = g->n;
  const double gamma = g->gamma;
  const double lam[3] = {dt / g->dx[0], dt / g->dx[1], dt / g->dx[2]};
  const size_t bd = oracle_block_doubles(g);
  const double *Ub = U + (size_t)b * bd;
  const int m = n + 2;                 /* cells -1..n per axis */
  const size_t nm = (size_t)m * m * m;
  /* transverse pairs: for direction d, t = tr[d][0], u = tr[d][1] */
  const int tr[3][2] = {{1, 2}, {0, 2}, {0, 1}};
  double *Wf = (double *)malloc(sizeof(double) * 30 * nm);   /* normal face states [d][side][v], side 0 low 1 high */
  double *Uf = (double *)malloc(sizeof(double) * 30 * nm);   /* the same, conserved */
  double *F1 = (double *)malloc(sizeof(double) * 15 * nm);   /* 1-D flux at the low d-face of a cell [d][v] */
  double *Fc = (double *)malloc(sizeof(double) * 30 * nm);   /* corner flux F_{d|t} at the low d-face [d][k][v], t = tr[d][k] */

#define CI(i, j, k) ((((size_t)((k) + 1) * m + (size_t)((j) + 1)) * m + (size_t)((i) + 1)))
  /* 1. normal predictor on cells -1..n */
  for (int k = -1; k <= n; ++k)
    for (int j = -1; j <= n; ++j)
      for (int i = -1; i <= n; ++i) {
        const int off[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        double W[5], Wm[5], Wq[5], Sl[3][5];
        double Uc[5];
        for (int v = 0; v < 5; ++v) Uc[v] = Ub[at(g, v, i, j, k)];
        int fl = oracle_cons_to_prim(Uc, gamma, g->small_p, W);
        int interior = i >= 0 && i < n && j >= 0 && j < n && k >= 0 && k < n;
        if (fl && interior) cnt[ORACLE_CNT_FLOOR]++;
        for (int d = 0; d < 3; ++d) {
          double Um_[5], Uq_[5];
          for (int v = 0; v < 5; ++v) {
            Um_[v] = Ub[at(g, v, i - off[d][0], j - off[d][1], k - off[d][2])];
            Uq_[v] = Ub[at(g, v, i + off[d][0], j + off[d][1], k + off[d][2])];
          }
          oracle_cons_to_prim(Um_, gamma, g->small_p, Wm);
          oracle_cons_to_prim(Uq_, gamma, g->small_p, Wq);
          for (int v = 0; v < 5; ++v) Sl[d][v] = oracle_van_leer(W[v] - Wm[v], Wq[v] - W[v]);
        }
        double *wf = Wf + 30 * CI(i, j, k);
        int bad = 0;
        for (int d = 0; d < 3; ++d) {
          if (trace) {
            oracle_trace_faces(W, Sl[d], d, lam[d], gamma, wf + (2 * d + 0) * 5, wf + (2 * d + 1) * 5);
          } else {
            double A[5], Wt[5];
            jacobian_times(W, d, gamma, Sl[d], A);
            for (int v = 0; v < 5; ++v) Wt[v] = W[v] - 0.5 * lam[d] * A[v];
            for (int v = 0; v < 5; ++v) {
              wf[(2 * d + 0) * 5 + v] = Wt[v] - 0.5 * Sl[d][v];
              wf[(2 * d + 1) * 5 + v] = Wt[v] + 0.5 * Sl[d][v];
            }
          }
          for (int sd = 0; sd < 2; ++sd)
            if (!(wf[(2 * d + sd) * 5 + 0] > 0.0) || !(wf[(2 * d + sd) * 5 + 4] > 0.0)) bad = 1;
        }
        if (bad) {
          for (int q = 0; q < 6; ++q)
            for (int v = 0; v < 5; ++v) wf[q * 5 + v] = W[v];
          if (interior) cnt[ORACLE_CNT_FALLBACK]++;
        }
        for (int q = 0; q < 6; ++q) prim_to_cons(wf + q * 5, gamma, Uf + 30 * CI(i, j, k) + q * 5);
      }

  /* 2. 1-D fluxes at d-faces between cells c - e_d and c, c_d in 0..n */
  for (int d = 0; d < 3; ++d)
    for (int k = -1; k <= n; ++k)
      for (int j = -1; j <= n; ++j)
        for (int i = -1; i <= n; ++i) {
          const int c[3] = {i, j, k};
          if (c[d] < 0) continue;
          const int li = i - (d == 0), lj = j - (d == 1), lk = k - (d == 2);
          oracle_hllc(Wf + 30 * CI(li, lj, lk) + (2 * d + 1) * 5, Wf + 30 * CI(i, j, k) + (2 * d + 0) * 5, d, gamma,
                      F1 + 15 * CI(i, j, k) + 5 * d);
        }

  /* 3. corner states and corner fluxes F_{d|t} at d-faces with c_t in 0..n-1 */
  for (int d = 0; d < 3; ++d)
    for (int q = 0; q < 2; ++q) {
      const int t = tr[d][q];
      for (int k = -1; k <= n; ++k)
        for (int j = -1; j <= n; ++j)
          for (int i = -1; i <= n; ++i) {
            const int c[3] = {i, j, k};
            if (c[d] < 0 || c[t] < 0 || c[t] > n - 1) continue;
            double Wside[2][5];
            for (int sd = 0; sd < 2; ++sd) {   /* sd 0: the low cell's high face, 1: this cell's low face */
              const int ci = i - (sd == 0 && d == 0), cj = j - (sd == 0 && d == 1), ck = k - (sd == 0 && d == 2);
              const int face = sd == 0 ? 1 : 0;
              const size_t cc = CI(ci, cj, ck);
              const size_t ch = CI(ci + (t == 0), cj + (t == 1), ck + (t == 2)); /* cell above in t */
              double Ucor[5];
              for (int v = 0; v < 5; ++v)
                Ucor[v] = Uf[30 * cc + (2 * d + face) * 5 + v] -
                          (lam[t] / 3.0) * (F1[15 * ch + 5 * t + v] - F1[15 * cc + 5 * t + v]);
              if (!corrected_prim(Ucor, gamma, Wside[sd])) {
                for (int v = 0; v < 5; ++v) Wside[sd][v] = Wf[30 * cc + (2 * d + face) * 5 + v];
                cnt[ORACLE_CNT_FALLBACK]++;
              }
            }
            oracle_hllc(Wside[0], Wside[1], d, gamma, Fc + 30 * CI(i, j, k) + (2 * d + q) * 5);
          }
    }

  /* 4. final states and fluxes at the interior faces; 5. update */
  double *Ff = (double *)malloc(sizeof(double) * 15 * nm);
  for (int d = 0; d < 3; ++d) {
    const int t = tr[d][0], u = tr[d][1];
    for (int k = 0; k <= n; ++k)
      for (int j = 0; j <= n; ++j)
        for (int i = 0; i <= n; ++i) {
          const int c[3] = {i, j, k};
          if (c[t] > n - 1 || c[u] > n - 1) continue;
          double Wside[2][5];
          for (int sd = 0; sd < 2; ++sd) {
            const int ci = i - (sd == 0 && d == 0), cj = j - (sd == 0 && d == 1), ck = k - (sd == 0 && d == 2);
            const int face = sd == 0 ? 1 : 0;
            const size_t cc = CI(ci, cj, ck);
            const size_t ct = CI(ci + (t == 0), cj + (t == 1), ck + (t == 2));
            const size_t cu = CI(ci + (u == 0), cj + (u == 1), ck + (u == 2));
            /* index of u among t's transverse pair, and of t among u's */
            const int kt = tr[t][0] == u ? 0 : 1;
            const int ku = tr[u][0] == t ? 0 : 1;
            double Ufin[5];
            for (int v = 0; v < 5; ++v)
              Ufin[v] = Uf[30 * cc + (2 * d + face) * 5 + v] -
                        0.5 * (lam[t] * (Fc[30 * ct + (2 * t + kt) * 5 + v] - Fc[30 * cc + (2 * t + kt) * 5 + v]) +
                               lam[u] * (Fc[30 * cu + (2 * u + ku) * 5 + v] - Fc[30 * cc + (2 * u + ku) * 5 + v]));
            if (!corrected_prim(Ufin, gamma, Wside[sd])) {
              for (int v = 0; v < 5; ++v) Wside[sd][v] = Wf[30 * cc + (2 * d + face) * 5 + v];
              cnt[ORACLE_CNT_FALLBACK]++;
            }
          }
          oracle_hllc(Wside[0], Wside[1], d, gamma, Ff + 15 * CI(i, j, k) + 5 * d);
        }
  }
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        const size_t c0 = CI(i, j, k);
        const size_t cx = CI(i + 1, j, k), cy = CI(i, j + 1, k), cz = CI(i, j, k + 1);
        double Un[5];
        for (int v = 0; v < 5; ++v) {
          double div = (lam[0] * (Ff[15 * cx + v] - Ff[15 * c0 + v]) +
                        lam[1] * (Ff[15 * cy + 5 + v] - Ff[15 * c0 + 5 + v])) +
                       lam[2] * (Ff[15 * cz + 10 + v] - Ff[15 * c0 + 10 + v]);
          Un[v] = Ub[at(g, v, i, j, k)] - div;
          Uo[at(g, v, i, j, k)] = Un[v];
        }
        int ok = Un[0] > 0.0 && Un[4] > 0.0;
        for (int v = 0; v < 5; ++v) ok = ok && isfinite(Un[v]);
        if (!ok) cnt[ORACLE_CNT_NONPHYS]++;
      }
#undef CI
  free(Wf);
  free(Uf);
  free(F1);
  free(Fc);
  free(Ff);
}

void oracle_ctu_block(const oracle_grid *g, const double *U, long b, double *Uo, double dt,
                      long cnt[ORACLE_NCNT]) {
  ctu_block(g, U, b, Uo, dt, 0, cnt);
}

void oracle_ctu_char_block(const oracle_grid *g, const double *U, long b, double *Uo, double dt,
                           long cnt[ORACLE_NCNT]) {
  ctu_block(g, U, b, Uo, dt, 1, cnt);
}

static void step_ctu_all(const oracle_grid *g, double *U, double *Unew, double dt, int trace,
                         long cnt[ORACLE_NCNT]) {
  long nblk = (long)g->nb[0] * g->nb[1] * g->nb[2];
  oracle_fill_guards(g, U);
  long c0 = 0, c1 = 0, c2 = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : c0, c1, c2)
  for (long b = 0; b < nblk; ++b) {
    long c[ORACLE_NCNT] = {0, 0, 0};
    ctu_block(g, U, b, Unew + (size_t)b * oracle_block_doubles(g), dt, trace, c);
    c0 += c[0];
    c1 += c[1];
    c2 += c[2];
  }
  cnt[ORACLE_CNT_FLOOR] += c0;
  cnt[ORACLE_CNT_FALLBACK] += c1;
  cnt[ORACLE_CNT_NONPHYS] += c2;
}

void oracle_step_ctu(const oracle_grid *g, double *U, double *Unew, double dt, long cnt[ORACLE_NCNT]) {
  step_ctu_all(g, U, Unew, dt, 0, cnt);
}

void oracle_step_ctu_char(const oracle_grid *g, double *U, double *Unew, double dt, long cnt[ORACLE_NCNT]) {
  step_ctu_all(g, U, Unew, dt, 1, cnt);
}

/* ---- a6: CFL signal speed and dt ---------------------------------------- */

double oracle_max_signal(const oracle_grid *g, const double *U, long b0, long b1) {
  const int n = g->n;
  const size_t bd = oracle_block_doubles(g);
  double smax = 0.0;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(max : smax) reduction(| : bad)
  for (long b = b0; b < b1; ++b) {
    const double *Ub = U + (size_t)b * bd;
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          double Uc[5], W[5];
          for (int v = 0; v < 5; ++v) Uc[v] = Ub[at(g, v, i, j, k)];
          oracle_cons_to_prim(Uc, g->gamma, g->small_p, W);
          double c = sqrt(g->gamma * W[4] / W[0]);
          double s = ((fabs(W[1]) + c) / g->dx[0] + (fabs(W[2]) + c) / g->dx[1]) + (fabs(W[3]) + c) / g->dx[2];
          if (!isfinite(s)) bad = 1;
          else if (s > smax) smax = s;
        }
  }
  return bad ? NAN : smax;
}

/* max over interior cells and directions of (|u_d| + c)/dx_d: the
 * per-direction CFL rule of the CTU step. */
double oracle_max_signal_dir(const oracle_grid *g, const double *U, long b0, long b1) {
  const int n = g->n;
  const size_t bd = oracle_block_doubles(g);
  double smax = 0.0;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(max : smax) reduction(| : bad)
  for (long b = b0; b < b1; ++b) {
    const double *Ub = U + (size_t)b * bd;
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          double Uc[5], W[5];
          for (int v = 0; v < 5; ++v) Uc[v] = Ub[at(g, v, i, j, k)];
          oracle_cons_to_prim(Uc, g->gamma, g->small_p, W);
          double c = sqrt(g->gamma * W[4] / W[0]);
          for (int d = 0; d < 3; ++d) {
            double s = (fabs(W[1 + d]) + c) / g->dx[d];
            if (!isfinite(s)) bad = 1;
            else if (s > smax) smax = s;
          }
        }
  }
  return bad ? NAN : smax;
}

double oracle_dt_ctu(const oracle_grid *g, const double *U, double cfl) {
  long nblk = (long)g->nb[0] * g->nb[1] * g->nb[2];
  double s = oracle_max_signal_dir(g, U, 0, nblk);
  if (!(s > 0.0) || !isfinite(s)) return -1.0;
  return cfl / s;
}

double oracle_dt(const oracle_grid *g, const double *U, double cfl) {
  long nblk = (long)g->nb[0] * g->nb[1] * g->nb[2];
  double s = oracle_max_signal(g, U, 0, nblk);
  if (!(s > 0.0) || !isfinite(s)) return -1.0;
  return cfl / s;
}
