/*
 * libhydro: FP64 unsplit second-order Godunov hydro step on a uniform grid of
 * cubic blocks, for AMD Instinct MI355X (gfx950).  C ABI; plain pointers and
 * sizes only.
 *
 * The operation is the explicit finite-volume update of the compressible
 * Euler equations that the paper's software description names (§2: explicit
 * methods for compressible flow with strong shocks, advanced block by block
 * on a uniform grid with guard cells supplied by the Grid unit; §2.2
 * Hydrodynamics: the predictor-corrector unsplit compressible solver; §2.2
 * Equations of State: the perfect-gas EOS).  One step is
 *   (1) same-level guard fill: periodic (index mod N) or zero-gradient
 *       outflow (index clamped into the domain), per axis;
 *   (2) conservative -> primitive recovery, p = (gamma-1)(E - rho|v|^2/2),
 *       floored at small_p;
 *   (3) van Leer slopes 2ab/(a+b) (ab > 0, else 0) of the primitives along
 *       x, y, z and a MUSCL-Hancock half-step predictor using all three
 *       directions; a cell whose six face states are not all positive in
 *       density and pressure falls back to its cell-centred state;
 *   (4) HLLC fluxes (Davis wave speeds, Batten contact speed) on every face;
 *   (5) U' = U - ((dt/dx (Fx+ - Fx-) + dt/dy (Fy+ - Fy-)) + dt/dz (Fz+ - Fz-));
 *   (6) CFL: dt = cfl / max over cells of sum_d (|u_d| + c) / dx_d.
 * All arithmetic is IEEE FP64 (round to nearest, denormals kept).
 *
 * Grid: nblk[0] x nblk[1] x nblk[2] cubic blocks of nxb^3 interior cells,
 * each with nguard = 4 guard layers per side.  Blocks are numbered
 * b = bx + nblk[0]*(by + nblk[1]*bz).
 *
 * State layout (device memory, owned by the caller): interior cells only.
 * Block b holds 5 conserved variables (rho, rho*u, rho*v, rho*w, E) in that
 * order, each an nxb^3 array of doubles, x fastest:
 *     U[((b*5 + var)*nxb + k)*nxb*nxb + j*nxb + i],   0 <= i, j, k < nxb.
 * The guard layers are not stored with the state: hydro_step gathers each
 * block's guard cells from its neighbours' interiors on chip (the same-level
 * fill), and hydro_fill_guards writes the guarded view of every block,
 *     G[((b*5 + var)*P + (k + nguard))*P*P + (j + nguard)*P + (i + nguard)],
 * P = nxb + 2*nguard, -nguard <= i, j, k < nxb + nguard, into a caller
 * buffer.  (Streaming a state stored with its guard layers in place measured
 * about 40% below the compact layout on MI355X HBM3E.)
 *
 * Ownership: every buffer named in a descriptor (state buffers, workspace,
 * stream) belongs to the caller and must outlive the handle.  The library
 * never allocates or frees device memory; a handle holds host metadata only.
 *
 * Asynchrony: every call is ordered on the descriptor's stream and returns
 * without waiting, except hydro_dt, hydro_last_dt and hydro_counters, which
 * wait for the stream.  A handle is not thread-safe;
 * different handles may be used from different threads and streams.
 *
 * Errors: 0 on success, a negative HYDRO_E* code otherwise; the message of
 * the last failure on the calling thread is returned by hydro_last_error().
 */
#ifndef HYDRO_H
#define HYDRO_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HYDRO_OK 0
#define HYDRO_EINVAL (-1)   /* invalid argument or descriptor */
#define HYDRO_ESIZE (-2)    /* workspace too small */
#define HYDRO_EDEVICE (-3)  /* HIP runtime error (message has the HIP text) */
#define HYDRO_ENONPHYS (-4) /* a step left a cell with rho<=0, E<=0 or a non-finite value */

#define HYDRO_BC_PERIODIC 0
#define HYDRO_BC_OUTFLOW 1

#define HYDRO_NGUARD 4

/* Time integration (hydro_set_scheme). */
#define HYDRO_SCHEME_MH 0  /* predictor-corrector (MUSCL-Hancock) step, the default */
#define HYDRO_SCHEME_RK2 2 /* second-order SSP Runge-Kutta, method-of-lines stages */
#define HYDRO_SCHEME_RK3 3 /* third-order SSP Runge-Kutta, method-of-lines stages */
#define HYDRO_SCHEME_CTU 4 /* corner-transport-upwind unsplit step, per-direction CFL rule */
#define HYDRO_SCHEME_CTU_CHAR 5 /* the same with characteristic tracing in the normal predictor */

typedef struct hydro_grid hydro_grid;

typedef struct {
  int nxb;          /* interior cells per block edge: 8, 16 or 32 */
  int nguard;       /* guard layers per side: must be HYDRO_NGUARD */
  int nblk[3];      /* blocks along x, y, z (each >= 1) */
  double lo[3];     /* domain lower corner */
  double hi[3];     /* domain upper corner; dx_d = (hi-lo)/(nblk_d*nxb) > 0 */
  int bc[3];        /* HYDRO_BC_* per axis, applied on both sides */
  double gamma;     /* ratio of specific heats, > 1 */
  double small_p;   /* pressure floor, >= 0 */
  double *U;        /* device: state buffer, hydro_state_doubles() values, 256-aligned */
  double *U_alt;    /* device: second state buffer of the same size */
  void *work;       /* device: workspace, hydro_work_bytes() bytes, 256-aligned */
  size_t work_bytes;
  void *stream;     /* hipStream_t the calls are ordered on (NULL: null stream) */
} hydro_grid_desc;

/* Doubles in one state buffer: nblk * 5 * nxb^3.  0 if invalid. */
size_t hydro_state_doubles(const hydro_grid_desc *d);

/* Doubles in the guarded view: nblk * 5 * (nxb + 2*nguard)^3.  0 if invalid. */
size_t hydro_guarded_doubles(const hydro_grid_desc *d);

/* Workspace bytes the grid needs (signal-speed slots, event counters). */
size_t hydro_work_bytes(const hydro_grid_desc *d);

/* Validate the descriptor and create a handle.  The current state starts in
 * U.  Clears the workspace (stream-ordered).  Errors: HYDRO_EINVAL for any
 * invalid field (including nguard != 4, nxb not in {8,16,32}, NULL or
 * misaligned buffers, U == U_alt, a z layer of blocks -- nblk[0]*nblk[1]
 * blocks, 40*nxb^3 bytes each -- of 4 GiB or more: kernels address a layer
 * with 32-bit byte offsets), HYDRO_ESIZE for a short workspace,
 * HYDRO_EDEVICE when the device is not gfx950 or a HIP call fails. */
int hydro_init_grid(const hydro_grid_desc *d, hydro_grid **out);

/* Same-level guard fill (§2: the Grid unit supplies each block's boundary
 * data): writes the guarded view of the current state into `guarded`
 * (device, hydro_guarded_doubles() values, 8-byte aligned, disjoint from
 * both state buffers): every block's interior plus all nguard layers (faces,
 * edges, corners), each guard cell holding the interior value at its mapped
 * global index (periodic: mod N, outflow: clamped).  Async. */
int hydro_fill_guards(hydro_grid *g, double *guarded);

/* One step of size dt (finite, > 0) from the current state into the other
 * buffer, which then becomes current.  Steps (1)-(5), with the guard fill
 * done on chip from neighbouring interiors; also reduces the signal speed
 * (6) of the new state for the next hydro_dt.  Async. */
int hydro_step(hydro_grid *g, double dt);

/* One step whose dt = cfl / max signal speed of the current state is formed
 * on the device (no host round trip); the dt used is kept for
 * hydro_last_dt.  Async. */
int hydro_step_cfl(hydro_grid *g, double cfl);

/* dt = cfl / max over interior cells of sum_d (|u_d| + c)/dx_d of the current
 * state.  Waits for the stream.  Returns HYDRO_ENONPHYS (and still writes
 * dt_out when it is finite) if any step since init left a nonphysical cell,
 * else HYDRO_EINVAL if the maximum is not positive and finite.  If the state was
 * modified outside the library after the last hydro_step, call
 * hydro_state_changed first. */
int hydro_dt(hydro_grid *g, double cfl, double *dt_out);

/* The dt used by the most recent hydro_step_cfl (or hydro_step).  Waits. */
int hydro_last_dt(hydro_grid *g, double *dt_out);

/* Declare that the current state was written outside the library, so the
 * signal speed kept from the last step is stale. */
int hydro_state_changed(hydro_grid *g);

/* Which buffer (U or U_alt of the descriptor) holds the current state. */
int hydro_current(hydro_grid *g, double **U_cur);

/* Event counters summed over all steps since init: [0] pressure-floor hits,
 * [1] cells whose face states fell back to first order, [2] nonphysical
 * cells after an update.  Waits for the stream. */
int hydro_counters(hydro_grid *g, long long out[3]);

/* Destroy the handle (host metadata only; no device memory is freed).
 * Refused (HYDRO_EINVAL) while the grid belongs to a batch. */
int hydro_free_grid(hydro_grid *g);

/* Rebind the grid's two state buffers (same size and alignment rules as in
 * the descriptor): U must hold the current state, U_alt becomes the output
 * of the next step.  The kept signal speed and counters are unchanged, so U
 * must hold exactly the state the handle last produced or was given (or
 * call hydro_state_changed).  Lets a caller keep one state buffer per grid
 * and lend output buffers only to grids with a step in flight. */
int hydro_set_buffers(hydro_grid *g, double *U, double *U_alt);

/* Tuning: split each block column into nseg z pencils (1, 2 or 4), one
 * workgroup each; more workgroups for small grids at the cost of two extra
 * halo planes per pencil.  Results are bitwise independent of it. */
int hydro_set_pencils(hydro_grid *g, int nseg);

/* Tuning: z pencils of `planes` consecutive planes of the whole grid (a
 * pencil may span several blocks along z: fewer re-read halo planes per
 * updated plane on tall grids; or part of a block).  planes >= 2 and must
 * divide nblk[2]*nxb; the default is nxb (one block).  Results are bitwise
 * independent of it.  Errors: HYDRO_EINVAL. */
int hydro_set_pencil_planes(hydro_grid *g, int planes);

/* Tuning: edge of the column tiles a workgroup marches along z (8 or 16;
 * 8 for nxb = 8; default 16 for nxb 16 and 32).  Smaller tiles give four
 * times the workgroups (small grids fill the GPU) at the cost of a
 * relatively larger ring of re-predicted cells.  Results are bitwise
 * independent of it.  Errors: HYDRO_EINVAL (other value, 16 with nxb 8,
 * grid in a batch). */
int hydro_set_tile(hydro_grid *g, int tile);

/* Time integration of the grid's steps (§2.2 Hydrodynamics names two
 * compressible solvers: the predictor-corrector one and one with second- or
 * third-order strong-stability-preserving Runge-Kutta time integration).
 *   HYDRO_SCHEME_MH  (default): the predictor-corrector step above.
 *   HYDRO_SCHEME_RK2 / _RK3: Shu-Osher SSP Runge-Kutta of order 2 / 3 over
 *     method-of-lines stages.  A stage uses the same guard fill, EOS,
 *     van Leer slopes, positivity fallback, HLLC and flux difference, with
 *     face states W +- Delta/2 from the cell centre (no predictor half step):
 *       order 2: U1 = U + dt L(U);  U' = U/2 + (U1 + dt L(U1))/2
 *       order 3: U1 = U + dt L(U);  U2 = 3U/4 + (U1 + dt L(U1))/4;
 *                U' = U/3 + 2(U2 + dt L(U2))/3
 *     dt is the step's (host value, or cfl / the maximum signal speed of
 *     U); the signal speed of U' is reduced for the next dt.  The state
 *     stays in the current buffer (the other one holds U1; the last stage
 *     overwrites U cell by cell), so hydro_current does not change.
 * U_stage: caller-owned device buffer of hydro_state_doubles values,
 * 256-byte aligned, not overlapping U or U_alt; required by RK3 (holds U2),
 * ignored otherwise (may be NULL).  Counters sum over stages.
 *   HYDRO_SCHEME_CTU: the corner-coupled form of the unsplit predictor-
 *     corrector step (corner transport upwind, twelve HLLC solves per
 *     cell): normal predictor per direction (W_d = W - (dt/2dx_d) A_d D_d,
 *     face states W_d -+ D_d/2, first-order fallback); 1-D fluxes F1_d;
 *     corner states U_d - (dt/3dx_t) dF1_t over the cell for each
 *     transverse t and their fluxes F_{d|t}; final states
 *     U_d - (dt/2dx_t) dF_{t|u} - (dt/2dx_u) dF_{u|t} and their fluxes;
 *     update.  A corrected state with rho <= 0 or p <= 0 falls back to the
 *     normal face state (counted).  Its CFL rule is per direction:
 *     dt = cfl / max over cells and d of (|u_d|+c)/dx_d (hydro_dt and
 *     hydro_step_cfl follow it for a CTU grid).  U_stage is ignored (the
 *     step keeps its intermediate states on chip: 8 x 8 column tiles
 *     marching along z through each block).
 *   HYDRO_SCHEME_CTU_CHAR: the CTU step whose normal predictor traces
 *     characteristics, as the unsplit solver §2.2 names does (Lee's papers,
 *     after Colella 1990): the van Leer primitive slope D_d is projected on
 *     the waves of A_d -- speeds u-c, u (entropy and shear), u+c, with
 *     amplitudes D_p/(2c^2) -+ rho D_u/(2c) on the right eigenvectors
 *     (1, -+c/rho, 0, 0, c^2) and (D_rho - D_p/c^2, 0, D_t1, D_t2, 0) --
 *     and the high face state is W + sum over waves of speed s > 0 of
 *     (1 - (dt/dx_d) s)/2 times the wave, the low one W - sum over s < 0 of
 *     (1 + (dt/dx_d) s)/2 times the wave; everything else as for
 *     HYDRO_SCHEME_CTU (same fallbacks and CFL rule).
 * Errors: HYDRO_EINVAL (unknown scheme, RK3 without a valid buffer, grid in
 * a batch).  Batches take HYDRO_SCHEME_MH grids only. */
int hydro_set_scheme(hydro_grid *g, int scheme, double *U_stage);

/* ---- batches: many independent grids, one persistent launch per step ----
 * (§2: physics is updated block by block, independently of how blocks are
 * distributed; here blocks of many simulations share one launch.)  A batch
 * groups grid handles (mixed nxb allowed).  Each step, a persistent grid
 * of G workgroups walks a device work list of (grid, pencil) items, the
 * heaviest first, workgroup w taking items w, w+G, w+2G, ...; each grid
 * takes its own dt = cfl / its own maximum signal speed, formed on the
 * device.  A grid's results are bitwise the same alone or in any batch.
 * While a grid belongs to a batch its own step calls are refused; hydro_dt,
 * hydro_current, hydro_counters and hydro_fill_guards keep working (the
 * handles follow the batch's steps).  The caller orders work on the member
 * grids' streams before the batch's stream. */
typedef struct hydro_batch hydro_batch;

/* Device workspace bytes a batch of these grids needs (0 if invalid). */
size_t hydro_batch_work_bytes(hydro_grid *const *grids, int n);

/* Create a batch over n distinct grids not in another batch; work is device
 * memory (256-byte aligned, hydro_batch_work_bytes bytes) owned by the
 * caller; stream is the hipStream_t batch steps are ordered on. */
int hydro_batch_create(hydro_grid *const *grids, int n, void *work, size_t work_bytes, void *stream,
                       hydro_batch **out);

/* nsteps steps of every active member with dt = cfl / its own max signal
 * speed.  Async.  With graphs enabled, runs of 6 steps replay one captured
 * HIP graph (kernel nodes only). */
int hydro_batch_step(hydro_batch *b, double cfl, int nsteps);

/* mask[i] != 0: member i takes part in the following steps. */
int hydro_batch_set_active(hydro_batch *b, const unsigned char *mask);

/* Tuning (results are bitwise independent of them): z pencils per column for
 * nxb = 8, 16, 32 (each 1, 2 or 4); persistent workgroups per CU (1..8);
 * whether to replay steps through a captured HIP graph. */
int hydro_batch_set_pencils(hydro_batch *b, const int nseg[3]);
int hydro_batch_set_workgroups(hydro_batch *b, int per_cu);
/* Column tile edge per block size (nxb 8, 16, 32): 8 for nxb 8, 8 or 16
 * otherwise (default 8, 16, 16).  Bitwise independent of it. */
int hydro_batch_set_tiles(hydro_batch *b, const int tile[3]);
int hydro_batch_use_graph(hydro_batch *b, int enable);

/* dt_out[i] = dt of member i's most recent step.  Waits for the stream. */
int hydro_batch_dts(hydro_batch *b, double *dt_out);

/* Destroy the batch (host metadata only); members become free grids. */
int hydro_batch_free(hydro_batch *b);

/* Allocation-free batch steps, for callers that cannot allocate device
 * memory (tight serving loops, harnesses that forbid hipMalloc): the same
 * steps as hydro_batch_create + hydro_batch_step(cfl, nsteps) +
 * hydro_batch_free over the n grids (distinct, not in a batch, predictor-
 * corrector scheme), with the member table and work list in the library's
 * own static device scratch instead of a caller workspace.  The scratch is
 * one file-scope array per device, held until the process ends, sized for
 * HYDRO_STATIC_MAX_GRIDS grids and HYDRO_STATIC_MAX_ITEMS work items (one
 * item per z pencil of a column tile: nblk * (nxb/16)^2 * nseg per grid, or
 * nblk * nseg for nxb = 8).  nseg: z pencils per column for nxb 8, 16, 32
 * (1, 2 or 4 each; NULL for 1, 1, 1).  Plain launches, 2 persistent
 * workgroups per CU; results bitwise equal to the handle-based batch.  The
 * grids' handles advance as after hydro_batch_step.  Every call on a device
 * shares that device's scratch and overwrites it (the tables are uploaded
 * on `stream` before the launches that read them): calls on one stream are
 * ordered, calls that overlap on different streams of one device race.
 * Calls no hipMalloc / hipFree.  Async.  Errors: HYDRO_ESIZE (more grids or
 * items than the limits), HYDRO_EINVAL (as hydro_batch_create / _step),
 * HYDRO_EDEVICE. */
#define HYDRO_STATIC_MAX_GRIDS 4096
#define HYDRO_STATIC_MAX_ITEMS 524288
int hydro_batch_step_static(hydro_grid *const *grids, int n, const int nseg[3], double cfl, int nsteps,
                            void *stream);

/* Bandwidth probe (not part of the method): copies n doubles from src to dst
 * (device, 16-byte aligned, disjoint) with a plain streaming kernel on
 * `stream`.  Its runtime and HBM counters calibrate the roofline and
 * traffic figures of the step kernel.  Async. */
int hydro_copy_probe(const double *src, double *dst, size_t n, void *stream);

/* Message of the last failed call on this thread ("" if none). */
const char *hydro_last_error(void);

/* ---- block-structured AMR -------------------------------------------------
 * (§2: the Grid unit's block-structured mesh with adaptive refinement:
 * blocks of nxb^3 cells, guard cells across refinement jumps, conservative
 * fluxes at fine-coarse faces.)  An octree of blocks: level 0 is the root
 * grid of nblk blocks; each refined block of level l is covered by eight
 * children of level l+1 at half its cell width.  The blocks of level l+1
 * are the children of level l's refined blocks in increasing block index,
 * child cx + 2*cy + 4*cz covering cells (cx*nxb/2.., cy*nxb/2.., cz*nxb/2..)
 * of its parent.  Nesting (checked at creation): every refined block of a
 * level >= 1 has its 26 neighbours (boundary map applied; positions beyond
 * an outflow boundary excluded) at its own level, so leaf levels differ by
 * at most one across faces, edges and corners.  Refinement is fixed for a
 * handle; hydro_amr_estimate / hydro_amr_transfer regrid two-level meshes.
 * Every leaf takes the predictor-corrector step with the same dt:
 *   1. guard fill: level 0 by the same-level map over its state (refined
 *      blocks hold the restriction of their children); a guard position of
 *      level l >= 1 (mapped at that level) copies the cell of the level-l
 *      block there, or is prolonged from level l-1: U_c + sum_d S_d (+-1/4),
 *      S_d the van Leer slope of the conserved variable over level-(l-1)
 *      cells d-1, d, d+1, keeping U_c if the result has rho <= 0 or p <= 0;
 *   2. the step of each leaf from its guarded view (lam = dt/dx of its level);
 *   3. refluxing: a leaf next to a refined block of its level replaces the
 *      flux of each cell on that face by the mean of the four finer fluxes;
 *   4. restriction, finest level first: refined blocks take the mean of
 *      their children (a cell: the two 2 x 2 sums of its eight child cells'
 *      planes, added, times 1/8; the children that refluxing leaves alone
 *      write it from their own step).
 * Layouts (device, caller-owned, 256-byte aligned): Ur [nroot][5][nxb^3]
 * (block id bx + nb0*(by + nb1*bz)); Uf: the blocks of levels 1, 2, ...
 * concatenated, [5][nxb^3] each.  The step updates Ur and Uf in place: a
 * leaf's own cells are read by the workgroup that then writes them, every
 * other read of the old state goes through the leaves' guard views formed in
 * the workspace first (two guard layers; for nxb 8 and 16 only those
 * layers, for nxb 32 with the interior), and the refluxing fluxes are
 * formed before the leaf steps.  refine: host flags of level 0, one per root block;
 * refine_deep: host flags of levels 1, 2, ... (one per block of each level,
 * concatenated; NULL with nrefine_deep 0 for two levels); both copied at
 * creation. */
typedef struct hydro_amr hydro_amr;
typedef struct {
  int nxb;                     /* 8, 16 or 32 */
  int nguard;                  /* must be HYDRO_NGUARD */
  int nblk[3];                 /* root blocks per axis */
  double lo[3], hi[3];         /* domain; root dx_d = (hi - lo)/(nblk_d*nxb) */
  int bc[3];                   /* HYDRO_BC_* per axis */
  double gamma, small_p;
  const unsigned char *refine; /* host, nblk[0]*nblk[1]*nblk[2] flags of level 0 */
  double *Ur;                  /* device root state */
  double *Uf;                  /* device state of levels >= 1 (may be NULL without refinement) */
  void *work;                  /* device workspace, hydro_amr_work_bytes */
  size_t work_bytes;
  void *stream;                /* hipStream_t */
  const unsigned char *refine_deep;  /* host flags of levels 1, 2, ... (may be NULL) */
  size_t nrefine_deep;               /* their count: whole levels */
} hydro_amr_desc;

/* Number of blocks of levels >= 1 (the length of Uf in blocks); 0 for an
 * invalid descriptor. */
size_t hydro_amr_fine_blocks(const hydro_amr_desc *d);
/* Number of levels (>= 1) and the blocks of each (nblocks[l], 0 beyond);
 * a negative error code for an invalid descriptor (bad nesting included). */
int hydro_amr_levels(const hydro_amr_desc *d, long nblocks[8]);
/* Workspace bytes: header, mesh tables, guard views of every block of every
 * level (nxb 8, 16: the two guard layers, 5*(nxb*((nxb+4)^2 - nxb^2) +
 * 4*(nxb+4)^2) doubles per block; nxb 32: 5*(nxb+4)^3), fluxes on block
 * faces (used at fine-coarse faces), one refinement indicator per block. */
size_t hydro_amr_work_bytes(const hydro_amr_desc *d);
/* Validate and build the mesh tables (uploaded to the workspace; waits for
 * the upload).  Errors: HYDRO_EINVAL, HYDRO_ESIZE, HYDRO_EDEVICE. */
int hydro_amr_create(const hydro_amr_desc *d, hydro_amr **out);
/* One step of size dt (stream-ordered).  Every step also reduces the new
 * state's signal speed (fused into the leaf steps and refluxing), so the
 * next hydro_amr_step_cfl needs no extra pass. */
int hydro_amr_step(hydro_amr *a, double dt);
/* One step with dt = cfl / max over leaves of sum_d (|u_d|+c)/dx_d of the
 * current state formed on the device (no host round trip); the dt used is
 * kept for hydro_amr_last_dt.  Async. */
int hydro_amr_step_cfl(hydro_amr *a, double cfl);
/* dt of the most recent step (waits).  HYDRO_EINVAL before the first step. */
int hydro_amr_last_dt(hydro_amr *a, double *dt_out);
/* Call after writing Ur / Uf outside the library: the signal speed the
 * last step reduced no longer describes the state. */
int hydro_amr_state_changed(hydro_amr *a);
/* dt = cfl / max over leaves of sum_d (|u_d|+c)/dx_d of their level (waits;
 * reduces the current state first unless a step already did).
 * Returns HYDRO_ENONPHYS (dt_out written when finite) if a step since
 * creation left a nonphysical cell, else HYDRO_EINVAL if the maximum is not
 * positive and finite. */
int hydro_amr_dt(hydro_amr *a, double cfl, double *dt_out);
/* Adaptivity (the Grid unit's refinement is adaptive; the paper names no
 * criterion): per root block, the largest squared Loehner second-derivative
 * ratio of density and of pressure over its cells (root state; refined
 * blocks hold their children's restriction),
 *   E^2 = sum_d num_d^2 / sum_d den_d^2,  num_d = (fR - f0) - (f0 - fL),
 *   den_d = (|fR - f0| + |f0 - fL|) + eps ((|fR| + 2|f0|) + |fL|),
 * neighbours along d by the root map, 0 where the denominator is 0, every
 * operation rounded as written.  New level-0 flags: 1 where
 * E^2 > refine_cutoff^2, 0 for a refined block where E^2 < derefine_cutoff^2,
 * else the current flag.  flags_out: host, nroot; E2_out: host, nroot, may be NULL.  Waits.
 * Errors: HYDRO_EINVAL (NULL, eps < 0, cutoffs not 0 <= derefine <= refine). */
int hydro_amr_estimate(hydro_amr *a, double eps, double refine_cutoff, double derefine_cutoff, double *E2_out,
                       unsigned char *flags_out);
/* Adaptivity of a mesh of any depth: the indicator of every leaf at its own
 * level (the per-cell quantity above, its neighbours read at the leaf's
 * level; a position with no block of that level takes the cell's own
 * state), then the rule: a leaf with E^2 > refine_cutoff^2 below level
 * max_levels-1 is refined; a refined block whose eight children are leaves
 * with E^2 < derefine_cutoff^2 loses them; nesting is then restored by
 * refining, coarsest level first and positions in increasing (x, y, z)
 * order, every block whose absence leaves a refined block of level >= 1
 * without a same-level neighbour, until nothing changes.  flags_out (host,
 * capacity cap) receives the new flags in descriptor order (level 0, then
 * each deeper level); *nflags_out their count (HYDRO_ESIZE when cap is
 * short).  E2_out (host, may be NULL): one value per block of every level
 * (refined blocks 0).  Waits.  Errors: HYDRO_EINVAL (NULL handle or
 * nflags_out, eps < 0, cutoffs not 0 <= derefine <= refine, max_levels not
 * in 1..8), HYDRO_ESIZE (cap short; *nflags_out still set, so a first call
 * with cap 0 sizes the buffer), HYDRO_EDEVICE. */
int hydro_amr_estimate_tree(hydro_amr *a, double eps, double refine_cutoff, double derefine_cutoff, int max_levels,
                            double *E2_out, unsigned char *flags_out, size_t cap, size_t *nflags_out);
/* Regridding: fill the state of mesh `to` (created with the new flags over
 * the same root grid, its own fine buffer) from mesh `from`: the root state
 * is copied (unless both use one buffer), children of blocks refined in both
 * are copied, children of newly refined blocks are prolonged from the root
 * state (the guard-fill prolongation, conservative), and every refined root
 * block of `to` takes its children's restriction; derefined blocks keep
 * their root values (the restriction of the children they lose).  Waits for
 * `from`'s stream, then runs on `to`'s.  `from` may be freed afterwards.
 * Any depth: level by level, a block of `to` at a position `from` has at
 * that level is copied, a new one is prolonged from `to`'s level above. */
int hydro_amr_transfer(hydro_amr *from, hydro_amr *to);
/* Event counters summed since creation: floors, fallbacks, nonphysical cells (waits). */
int hydro_amr_counters(hydro_amr *a, long long out[3]);
/* Tuning (no effect on results): the leaf steps advance columns of up to
 * `cap` leaves of one level stacked in z as one pencil each (cap 1, 2 or
 * 4), or, with cap 0 (the default at creation), the length per leaf list
 * whose tiles, dealt to the device's workgroup slots, finish first.
 * Rewrites the column tables on the mesh's stream (waits).  Errors:
 * HYDRO_EINVAL (NULL handle, cap not 0, 1, 2 or 4), HYDRO_EDEVICE. */
int hydro_amr_set_columns(hydro_amr *a, int cap);
int hydro_amr_free(hydro_amr *a);

#ifdef __cplusplus
}
#endif
#endif
