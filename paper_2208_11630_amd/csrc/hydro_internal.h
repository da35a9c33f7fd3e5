// Internal interface between the C-ABI host code (api.cpp) and the HIP
// kernels (hydro_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hydro {

// Device workspace header, at the start of the caller's workspace buffer.
// sig[] hold the bit patterns of the maximum CFL signal speed (non-negative
// doubles order like their unsigned bit patterns), triple-buffered by step
// number s: a step reads sig[s%3] (device-side dt), reduces the new state
// into sig[(s+1)%3] and clears sig[(s+2)%3] for the step after next.
struct WorkHeader {
  unsigned long long sig[3];
  unsigned long long cnt[3];  // floor hits, fallbacks, nonphysical cells
  double dt_last;             // dt of the most recent step
  unsigned long long pad[25];
};
static_assert(sizeof(WorkHeader) == 256, "workspace header is 256 bytes");

// Geometry and physics shared by every kernel of one grid.
struct GridGeom {
  int nb[3];          // blocks per axis
  int bc[3];          // 0 periodic, 1 outflow
  double inv_dx[3];   // 1/dx per axis
  double gamma;
  double small_p;
};

// Per-launch arguments of the step kernel.
struct StepArgs {
  const double* Uin;  // input state (compact layout, see hydro.h)
  double* Uout;       // output state
  WorkHeader* ws;
  double dt;          // used when cfl <= 0
  double cfl;         // > 0: dt = cfl / max signal speed in ws->sig[slot]
  int slot;           // step number mod 3
};

// One method-of-lines stage of an SSP Runge-Kutta step: the result is
// a0*U0 + a1*(Uin - dt div F), or Uin - dt div F when U0 is NULL.
struct StageArgs {
  const double* U0;   // base state of the step (may be the stage's output buffer)
  double a0, a1;
  int stage;          // 0: first stage (takes and records dt); > 0: uses the recorded dt
  int last;           // nonzero: reduce the result's signal speed for the next dt
};

// One member grid of a batch (device table entry).
struct BatchSim {
  double* U0;         // state buffer 0
  double* U1;         // state buffer 1
  WorkHeader* ws;     // the grid's workspace header
  GridGeom geom;
  int nxb;
  int parity0;        // buffer holding the state at batch step 0 (0: U0, 1: U1)
  int slot0;          // signal slot of the state at batch step 0
  int pad;
};

// One unit of batch work: a z pencil of a column tile of one grid.
struct BatchItem {
  int sim;
  int tile;           // pencil index inside the grid (see tile_step)
};

// The library's static device scratch (a file-scope array in
// hydro_kernels.hip, one copy per device, held until the process ends): the
// member table and work list of allocation-free batch steps.  Sizes are the
// limits hydro.h states (HYDRO_STATIC_MAX_GRIDS, HYDRO_STATIC_MAX_ITEMS).
constexpr size_t kStaticMaxGrids = 4096;
constexpr size_t kStaticMaxItems = size_t(1) << 19;
constexpr size_t kStaticSimsBytes = (kStaticMaxGrids * sizeof(BatchSim) + 255) / 256 * 256;
constexpr size_t kStaticScratchBytes = kStaticSimsBytes + kStaticMaxItems * sizeof(BatchItem);
// Device address of the scratch on the current device (looked up through
// hipGetSymbolAddress on a device's first call, then kept per device).
hipError_t static_scratch(void** ptr);

// st == NULL: predictor-corrector step; else one method-of-lines stage.
// tile: edge of the column tiles (8 for nxb 8; 8 or 16 otherwise).
// plen: planes per z pencil (>= 2, divides the grid's z extent).
hipError_t launch_step(int nxb, int tile, const GridGeom& g, const StepArgs& a, const StageArgs* st, int plen,
                       hipStream_t s);
// items: the work-list range of the members with blocks of nxb^3 cells
// (8, 16 or 32), listed with column tiles of edge `tile`; nseg: pencils
// per column for that size.
hipError_t launch_batch_step(const BatchSim* sims, const BatchItem* items, int nitems, long step, double cfl,
                             int nxb, int tile, int nseg, int grid, hipStream_t s);
hipError_t launch_fill_guards(int nxb, const GridGeom& g, const double* U, double* out, hipStream_t s);
// dir: the per-direction signal max_d (|u_d|+c)/dx_d of the CTU step
// instead of the summed one.
hipError_t launch_signal(int nxb, const GridGeom& g, const double* U, WorkHeader* ws, int slot, bool dir,
                         hipStream_t s);
// Corner-transport-upwind step (z-marching 8 x 8 column tiles, no scratch);
// trace: the normal predictor traces characteristics.
hipError_t launch_ctu(int nxb, const GridGeom& g, const StepArgs& a, bool trace, hipStream_t s);
hipError_t launch_clear_slot(WorkHeader* ws, int slot, hipStream_t s);
hipError_t launch_copy(const double* src, double* dst, long n, hipStream_t s);

// Block-structured AMR (see hydro_kernels.hip): an octree of blocks, level
// 0 the root grid, level l+1 the children of level l's refined blocks.
constexpr int AMR_MAX_LEVELS = 8;
// Doubles per block of a level's leaf views.  n = 8, 16 (the leaf step's
// tile spans the block plane): plane halos, the two guard layers only, plane
// by plane -- planes 0..n-1 the ring of width two around the interior,
// planes -2, -1, n, n+1 whole (the kernels' PlaneHalo<n>); n = 32: whole
// views of (n + 4)^3 cells.  Five variables.
constexpr long amr_view_doubles(int n) {
  return n == 32 ? 5L * (n + 4) * (n + 4) * (n + 4)
                 : 5L * ((long)n * ((n + 4) * (n + 4) - n * n) + 4L * (n + 4) * (n + 4));
}
struct AmrLevel {
  GridGeom g;                 // nb = root nb << l, inv_dx = root inv_dx * 2^l
  double* U;                  // the level's state (compact), updated in place
  double* G;                  // leaf views (amr_view_doubles per block), every block of the level
  double* flux;               // face fluxes per block (those at fine-coarse faces are used)
  const int* lookup;          // block index at each level-l block position, or -1
  const int4* pos;            // block positions (x, y, z, 0)
  const int* parent;          // parent block on level l-1 (level >= 1)
  const int* child_base;      // first child on level l+1, or -1
  const int* refined;         // refined blocks
  const int* leaves;          // unrefined blocks
  const int* leaf_plain;      // leaves without a refined face neighbour
  const int* rx_blocks;       // leaves with one (the reflux groups' blocks, in group order)
  const int4* reflux;         // (leaf, d, side, refined neighbour), grouped by leaf
  const int* reflux_first;    // ngroups + 1 offsets into reflux
  const int4* cols_plain;     // leaf_plain as columns of up to 4 z-stacked blocks (bottom first, -1 unused)
  const int4* cols_rx;        // rx_blocks likewise
  const int* roct;            // restriction octants 8 r + c of the pass (child c of refined block r is
                              // refined or takes refluxing; the other children's leaf steps restrict)
  const int* zneed;           // per block (n = 8, 16): the whole halo planes its fill writes, bit 0 planes
                              // -2, -1, bit 1 planes n, n+1 (those its column's pencil or a face flux reads)
  long nblk, nrefined, nleaves, nleaf_plain, nreflux, ngroups, ncols_plain, ncols_rx, nroct;
  int kmax_plain, kmax_rx;    // longest column of each list (blocks)
};
// Leaf steps over views: the restriction of the new state into the parent
// block, fused into the update (U null: none; see tile_step).
struct ParentOut {
  double* U;           // the parent level's state
  const int* parent;   // parent block of each block of the leaf's level
  const int4* pos;     // block positions of the leaf's level
};
// One column list of an AMR step's leaf-step launch: the launch's
// workgroups first .. first + ncols * (column tiles per block) - 1 step the
// columns of `cols` on level geometry g.
struct AmrSeg {
  GridGeom g;
  const double* G;     // the level's leaf views
  double* U;           // the level's state
  const int4* cols;
  ParentOut po;
  long first;
  int emit;            // reduce the new state's signal speed
  int pad;
};
constexpr int AMR_MAX_SEGS = 2 * AMR_MAX_LEVELS;
// The segments, passed by value as a kernel argument (kernel-argument
// memory is constant, so their fields stay loaded across barriers).
struct AmrSegs {
  AmrSeg s[AMR_MAX_SEGS];
  int n;
  long tiles;                 // the launch's workgroups
};
struct AmrLaunch {
  AmrLevel lev[AMR_MAX_LEVELS];
  int nlev;
  AmrSegs segs;               // the leaf-step launch (amr_segments)
  WorkHeader* ws;
  double dt;                  // used when cfl <= 0
  double cfl;                 // > 0: dt = cfl / ws->sig[slot]
  int slot;                   // step number mod 3
};
hipError_t launch_amr_step(int nxb, const AmrLaunch& L, hipStream_t s);
// The leaf-step launch's segments: every nonempty column list of every
// level, longest columns first.
void amr_segments(int nxb, const AmrLaunch& L, AmrSegs& out);
hipError_t launch_amr_signal(int nxb, const AmrLaunch& L, int slot, hipStream_t s);
// Refinement indicator per root block into E2[nroot] (device).
hipError_t launch_amr_indicator(int nxb, const AmrLaunch& L, double eps, double* E2, hipStream_t s);
// Per-leaf refinement indicator of every level into E2_levels[l][block].
hipError_t launch_amr_leaf_indicator(int nxb, const AmrLaunch& L, double eps, double* const* E2_levels,
                                     hipStream_t s);
// State of mesh `to` (levels >= 1) from mesh `from` (same root grid; to's
// root state in place): same-position blocks copied, new ones prolonged,
// level by level; then the restriction of to's refined blocks.
hipError_t launch_amr_transfer(int nxb, const AmrLaunch& from, const AmrLaunch& to, hipStream_t s);

}  // namespace hydro
