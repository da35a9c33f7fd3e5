/*
 * Plain FP64 CPU oracle of the unsplit second-order Godunov hydro step.
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the HIP path; it is
 * called from the test suite, from the package's smoke check and from the
 * CPU-baseline leg of the benchmark, never from the product path.  It shares
 * no code, header, table or helper with the HIP library.
 *
 * What it computes (the method behind the paper's compressible solver, §2
 * "Software Description": explicit shock-capturing methods, block-by-block
 * update on a uniform grid; §2.2 "Software Functionalities", Hydrodynamics:
 * the predictor-corrector unsplit compressible solver; §2.2, Equations of
 * State: the perfect-gas EOS).  The paper states the method by name only, so
 * the formulas follow the textbook statement of each ingredient:
 *   - same-level guard fill: periodic (index mod N) or zero-gradient outflow
 *     (index clamped into the domain), composed per axis;
 *   - conservative -> primitive with a gamma-law EOS and a pressure floor;
 *   - van Leer harmonic slope 2ab/(a+b) for ab>0 (else 0) on primitives;
 *   - MUSCL-Hancock half-step predictor in primitive form, all three
 *     directions at once (fully unsplit, no transverse corner coupling);
 *   - HLLC fluxes with Davis wave speeds and the Batten contact speed;
 *   - the conservative flux-difference update;
 *   - dt = CFL / max over cells of sum_d (|u_d| + c) / dx_d;
 *   - the SSP Runge-Kutta variant (§2.2 Hydrodynamics, the other compressible
 *     solver): method-of-lines stages with face states from the cell centre,
 *     combined in Shu-Osher form (second and third order).
 *
 * Layout: a grid of nb[0]*nb[1]*nb[2] cubic blocks, block id
 * b = bx + nb0*(by + nb1*bz).  Each block stores 5 conserved variables
 * (rho, rho*u, rho*v, rho*w, E), each as a P^3 array (P = n + 2*ng), x
 * fastest:  U[((b*5 + var)*P + k)*P*P + j*P + i], guard layers included.
 *
 * Every function is pinned by CPU tests against facts independent of this
 * code: closed forms, special cases that reduce to textbook schemes, the
 * exact Sod Riemann solution, conservation, symmetry and convergence order.
 */
#ifndef HYDRO_ORACLE_H
#define HYDRO_ORACLE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_BC_PERIODIC 0
#define ORACLE_BC_OUTFLOW 1

typedef struct {
  int n;          /* interior cells per block edge */
  int ng;         /* guard layers per side (>= 2 needed by the stencil) */
  int nb[3];      /* blocks per axis */
  double dx[3];   /* cell widths */
  int bc[3];      /* ORACLE_BC_* per axis (both sides) */
  double gamma;   /* ratio of specific heats */
  double small_p; /* pressure floor */
} oracle_grid;

/* Event counters of one step: [0] pressure-floor hits on interior cells,
 * [1] interior cells whose face states fell back to first order,
 * [2] interior cells left nonphysical (rho<=0, E<=0 or non-finite). */
enum { ORACLE_CNT_FLOOR = 0, ORACLE_CNT_FALLBACK = 1, ORACLE_CNT_NONPHYS = 2, ORACLE_NCNT = 3 };

size_t oracle_block_doubles(const oracle_grid *g);

/* Host threads used by the loops over blocks (timing only; no effect on results). */
void oracle_set_threads(int n);
int oracle_max_threads(void);

/* Primitive recovery of one cell; returns 1 when the pressure floor was hit. */
int oracle_cons_to_prim(const double U[5], double gamma, double small_p, double W[5]);
/* van Leer harmonic slope. */
double oracle_van_leer(double dl, double dr);
/* HLLC flux across a face normal to axis d (0,1,2) between primitive states. */
void oracle_hllc(const double WL[5], const double WR[5], int d, double gamma, double F[5]);
/* Exact Euler flux along axis d of a primitive state. */
void oracle_euler_flux(const double W[5], int d, double gamma, double F[5]);

/* Fill the guard layers of block b (or of every block) from block interiors. */
void oracle_fill_guards_block(const oracle_grid *g, double *U, long b);
void oracle_fill_guards(const oracle_grid *g, double *U);

/* New interior of block b after one step of size dt.  U must hold block b's
 * guards filled.  Uo is one block's storage (oracle_block_doubles values);
 * its interior receives the result, its guards are left untouched. */
void oracle_step_block(const oracle_grid *g, const double *U, long b, double *Uo,
                       double dt, long cnt[ORACLE_NCNT]);

/* The same step of block b, also returning every face flux of the block:
 * Fx[(k*n + j)*(n+1) + i][v] at the low x face of cell (i, j, k), i = 0..n
 * (i = n: the high face of cell n-1); Fy[(k*(n+1) + j)*n + i][v], j = 0..n;
 * Fz[(k*n + j)*n + i][v], k = 0..n.  Each array holds 5*(n+1)*n*n values.
 * (For refluxing at refinement jumps.) */
void oracle_step_block_fluxes(const oracle_grid *g, const double *U, long b, double *Uo, double dt,
                              double *Fx, double *Fy, double *Fz, long cnt[ORACLE_NCNT]);

/* Step a list of blocks (guards of each filled first, then updated); block
 * t's result goes to out + t*oracle_block_doubles(g).  Guards are written
 * only from interiors, so the blocks are independent. */
void oracle_step_block_list(const oracle_grid *g, double *U, const long *blocks, long nlist,
                            double *out, double dt, long cnt[ORACLE_NCNT]);

/* One full step: fills U's guards, then updates every block into Unew. */
void oracle_step(const oracle_grid *g, double *U, double *Unew, double dt, long cnt[ORACLE_NCNT]);

/* One method-of-lines stage of block b (the SSP Runge-Kutta solver of §2.2):
 * face states are the cell-centred primitives plus or minus half the van Leer
 * slope (no predictor half step; the same first-order fallback), fluxes by
 * HLLC, and Uo's interior = U - div F when U0b is NULL, else
 * a0*U0b + a1*(U - div F) (U0b: block b's storage of the base state). */
void oracle_stage_block(const oracle_grid *g, const double *U, long b, double *Uo, double dt,
                        const double *U0b, double a0, double a1, long cnt[ORACLE_NCNT]);

/* One SSP Runge-Kutta step of order 2 or 3 (Shu-Osher form) from U into
 * Unew; U's guards are refilled in place.  Returns 0, -1 for another order,
 * -2 when the stage buffers cannot be allocated. */
int oracle_step_rk(const oracle_grid *g, double *U, double *Unew, double dt, int order, long cnt[ORACLE_NCNT]);

/* One corner-transport-upwind step of block b (U's guards filled; Uo is
 * block b's storage): normal predictor, 1-D fluxes, corner states with
 * lam/3 transverse corrections and their fluxes, final states with lam/2
 * cross corrections, final fluxes, update (twelve HLLC solves per cell).
 * Counters: floors and normal-state fallbacks on interior cells, plus every
 * corrected state that fell back to its normal state. */
void oracle_ctu_block(const oracle_grid *g, const double *U, long b, double *Uo, double dt,
                      long cnt[ORACLE_NCNT]);
/* One CTU step of the whole grid (fills U's guards first). */
void oracle_step_ctu(const oracle_grid *g, double *U, double *Unew, double dt, long cnt[ORACLE_NCNT]);

/* The same CTU step with characteristic tracing in its normal predictor
 * (the unsplit solver of §2.2 as Lee's papers describe it: the slopes are
 * projected onto the characteristic waves of A_d and each face keeps the
 * waves moving toward it; see oracle_trace_faces). */
void oracle_ctu_char_block(const oracle_grid *g, const double *U, long b, double *Uo, double dt,
                           long cnt[ORACLE_NCNT]);
void oracle_step_ctu_char(const oracle_grid *g, double *U, double *Unew, double dt, long cnt[ORACLE_NCNT]);

/* Traced face states of one cell along d (primitive W, van Leer primitive
 * slope S, lam = dt/dx_d): lo / hi receive the low / high face states. */
void oracle_trace_faces(const double W[5], const double S[5], int d, double lam, double gamma, double lo[5],
                        double hi[5]);

/* max over interior cells of sum_d (|u_d| + c)/dx_d; the block range [b0,b1). */
double oracle_max_signal(const oracle_grid *g, const double *U, long b0, long b1);
/* dt = cfl / max signal over all blocks; returns -1 when the maximum is not positive and finite. */
double oracle_dt(const oracle_grid *g, const double *U, double cfl);
/* Per-direction rule of the CTU step: max over cells and d of (|u_d| + c)/dx_d, and cfl / that. */
double oracle_max_signal_dir(const oracle_grid *g, const double *U, long b0, long b1);
double oracle_dt_ctu(const oracle_grid *g, const double *U, double cfl);

#ifdef __cplusplus
}
#endif
#endif
