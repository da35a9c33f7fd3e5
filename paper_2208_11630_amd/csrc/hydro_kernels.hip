// HIP kernels (gfx950) of the unsplit second-order Godunov hydro step.
//
// The step follows the explicit finite-volume method the paper names (§2:
// explicit shock-capturing methods, block-by-block update with guard cells;
// §2.2 Hydrodynamics: the predictor-corrector unsplit compressible solver;
// §2.2 Equations of State: perfect gas).  The formulas are the ones listed
// in include/hydro.h.
//
// Design (MI355X):
//  * The state is stored compact, interior cells only ([block][var][z][y][x]):
//    streaming a guarded layout (guard rows and planes skipped, partial
//    ECC-word writes) measured 40% below a compact one on MI355X HBM3E.
//  * One workgroup owns a T x T column tile of one block and marches it along
//    z.  The same-level guard fill is fused: the tile's halo (faces two deep,
//    edges one deep) is gathered straight from the neighbouring blocks'
//    interiors through the periodic/outflow index map, so each interior value
//    crosses HBM once per step.  hydro_fill_guards materialises the guarded
//    Flash-X-style view (4 layers) only when a caller asks for it.
//  * Each thread owns one tile cell and keeps that column's primitives for
//    planes j, j+1 and the difference to plane j-1 in registers (z slopes,
//    z face states and z fluxes
//    never touch LDS).  The in-plane neighbours, the x/y face states and the
//    x/y fluxes go through LDS, so every face flux is computed exactly once
//    per tile; the one-cell ring around the tile is predicted as a second
//    item of one wavefront.
//  * The CFL signal speed of the new state is reduced in the epilogue
//    (wavefront shuffles, then one atomicMax per workgroup on the bit
//    pattern), so the next dt needs no extra pass over the state.
#include "hydro_internal.h"

#include <math.h>

#include <algorithm>

#include <mutex>

namespace hydro {
namespace {

constexpr int G = 4;   // guard layers per side of the guarded view
constexpr int VG = 2;  // guard layers of the internal views the AMR step fills (the stencil's depth)

// Compact state layout: block b, variable v, cell (i, j, k).
template <int N>
struct Layout {
  static constexpr long PS = (long)N * N;
  static constexpr long VS = PS * N;
  static constexpr long BS = 5 * VS;
  // offset of cell (i, j, k) of block b, variable 0
  __device__ static long at(long b, int i, int j, int k) { return b * BS + (long)k * PS + (long)j * N + i; }
};

// Guarded view: [block][var][P][P][P], P = N + 2GW, interior at offset GW.
template <int N, int GW = G>
struct Guarded {
  static constexpr int P = N + 2 * GW;
  static constexpr long PS = (long)P * P;
  static constexpr long VS = PS * P;
  static constexpr long BS = 5 * VS;
};

// Plane halos of a block (AMR leaf views for N = 8, 16, where the leaf
// step's tile spans the block plane and reads the block's interior from its
// state): the cells of the two guard layers, plane by plane, so that a fill
// writes whole rows.  Planes k = 0..N-1 hold the ring of width two around
// the interior -- rows -2, -1 whole, then the four guard cells of rows
// 0..N-1, then rows N, N+1 whole -- and planes -2, -1, N, N+1 are whole.
// Per variable VS doubles; block b's variable v at b*BS + v*VS.
template <int N>
struct PlaneHalo {
  static constexpr int P = N + 2 * VG;
  static constexpr int RP = P * P - N * N;  // ring plane
  static constexpr int FP = P * P;          // whole plane
  static constexpr long VS = (long)N * RP + 4L * FP;
  static constexpr long BS = 5 * VS;
  // slot of (i, j) in a ring plane; (i, j) outside [0, N)^2
  __device__ static int ring_index(int i, int j) {
    if (j < 0) return (j + VG) * P + (i + VG);
    if (j >= N) return 2 * P + 4 * N + (j - N) * P + (i + VG);
    return 2 * P + 4 * j + (i < 0 ? i + VG : i - N + VG);
  }
  // slot of (i, j) in a whole plane
  __device__ static int full_index(int i, int j) { return (j + VG) * P + (i + VG); }
  // slot of a guard cell (i, j, k), block-local indices, not in the interior
  __device__ static long slot(int i, int j, int k) {
    if (k >= 0 && k < N) return (long)k * RP + ring_index(i, j);
    return (long)N * RP + (long)(k < 0 ? k + VG : k - N + VG) * FP + full_index(i, j);
  }
  // the cell of slot s
  __device__ static void cell(int s, int& i, int& j, int& k) {
    if (s < N * RP) {
      k = s / RP;
      const int r = s - k * RP;
      if (r < 2 * P) {
        j = r / P - VG;
        i = r % P - VG;
      } else if (r < 2 * P + 4 * N) {
        const int q = r - 2 * P, c = q % 4;
        j = q / 4;
        i = c < 2 ? c - VG : N + c - VG;
      } else {
        const int q = r - 2 * P - 4 * N;
        j = N + q / P;
        i = q % P - VG;
      }
    } else {
      const int q = s - N * RP, kk = q / FP, r = q - kk * FP;
      k = kk < 2 ? kk - VG : N + kk - VG;
      j = r / P - VG;
      i = r % P - VG;
    }
  }
};
static_assert(PlaneHalo<16>::BS == amr_view_doubles(16) && PlaneHalo<8>::BS == amr_view_doubles(8) &&
                  Guarded<32, VG>::BS == amr_view_doubles(32),
              "leaf view sizes");

__device__ __forceinline__ int map_axis(int I, int n, int bc) {
  // n = cells along the axis; |offset| beyond the domain is at most 2 < n
  if (bc == 0) return I < 0 ? I + n : (I >= n ? I - n : I);
  return I < 0 ? 0 : (I >= n ? n - 1 : I);
}

// Offset (variable 0) of the cell at global index (I, J, K), any of which may
// lie up to two cells outside the domain; boundary conditions applied.
template <int N>
__device__ __forceinline__ long cell_offset(const GridGeom& g, int I, int J, int K) {
  I = map_axis(I, g.nb[0] * N, g.bc[0]);
  J = map_axis(J, g.nb[1] * N, g.bc[1]);
  K = map_axis(K, g.nb[2] * N, g.bc[2]);
  const long b = (long)(I / N) + (long)g.nb[0] * ((J / N) + (long)g.nb[1] * (K / N));
  return Layout<N>::at(b, I % N, J % N, K % N);
}

template <int N>
__device__ __forceinline__ void load_cons(const double* __restrict__ U, long off, double (&u)[5]) {
#pragma unroll
  for (int v = 0; v < 5; ++v) u[v] = U[off + v * Layout<N>::VS];
}

// Same, from a workgroup-uniform base P and a 32-bit per-cell byte offset
// (a scalar base plus a vector offset in the load itself).
// GVW: P points into an internal view (variable stride Guarded<N, VG>::VS).
// LAST: the workgroup's last read of these cells (nontemporal load).
template <int N, bool GVW = false, bool LAST = false>
__device__ __forceinline__ void load_cons_at(const double* P, unsigned xyb, double (&u)[5]) {
  constexpr long VSX = GVW ? (long)(N + 2 * VG) * (N + 2 * VG) * (N + 2 * VG) : (long)N * N * N;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const double* a = (const double*)((const char*)(P + v * VSX) + xyb);
    if constexpr (LAST) u[v] = __builtin_nontemporal_load(a);
    else u[v] = *a;
  }
}

// Same, with the variable stride VSX (plane halos).
template <long VSX>
__device__ __forceinline__ void load_cons_vs(const double* P, unsigned xyb, double (&u)[5]) {
#pragma unroll
  for (int v = 0; v < 5; ++v) u[v] = *(const double*)((const char*)(P + v * VSX) + xyb);
}

// Maximum over a workgroup of a non-negative double, folded into *slot with
// one atomicMax on the bit pattern.  red must hold one entry per wavefront.
__device__ __forceinline__ void wg_max_to(double v, unsigned long long* red, unsigned long long* slot) {
  unsigned long long bits = __double_as_longlong(v);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long other = __shfl_xor(bits, o, 64);
    bits = other > bits ? other : bits;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = bits;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = red[0];
#pragma unroll
    for (int w = 1; w < (int)(blockDim.x + 63) / 64; ++w) m = red[w] > m ? red[w] : m;
    atomicMax(slot, m);
  }
}

// ---------------------------------------------------------------------------
// Fast FP64 building blocks.  The hardware reciprocal / reciprocal square root
// (about 5e-8 relative) refined by one Newton step gives about 2^-48
// relative error: well inside the step's 1e-12 tolerance, at roughly half
// the instruction count of IEEE division and square root.

__device__ __forceinline__ double rcp_nr(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

// n / d with one Newton correction of the quotient
__device__ __forceinline__ double div_nr(double n, double d) {
  const double r = __builtin_amdgcn_rcp(d);
  const double q = n * r;
  return fma(fma(-d, q, n), r, q);
}

// t^(-1/2)
__device__ __forceinline__ double rsq_nr(double t) {
  const double y = __builtin_amdgcn_rsq(t);
  return fma(0.5 * y, fma(-(t * y), y, 1.0), y);
}

// Primitive state of a cell plus 1/rho (shared by the predictor).
__device__ __forceinline__ int prim(const double (&u)[5], double gamma, double small_p, double (&w)[5],
                                         double& inv) {
#pragma clang fp contract(off)  // the same bits in every inlined copy (own column, ring, halo cells)
  const double rho = u[0];
  inv = rcp_nr(rho);
  const double vx = u[1] * inv, vy = u[2] * inv, vz = u[3] * inv;
  const double kin = 0.5 * rho * ((vx * vx + vy * vy) + vz * vz);
  double p = (gamma - 1.0) * (u[4] - kin);
  int fl = 0;
  if (p < small_p) {
    p = small_p;
    fl = 1;
  }
  w[0] = rho;
  w[1] = vx;
  w[2] = vy;
  w[3] = vz;
  w[4] = p;
  return fl;
}

// HLLC flux normal to axis D between primitive states L and R (Davis wave
// speeds S_L, S_R; Batten contact speed S*).  Branches: S_L >= 0 -> F_L;
// S* >= 0 -> F*_L; S_R > 0 -> F*_R; else F_R.  The star state of the upwind
// side K uses one reciprocal q = 1/(S_K - S*), m = rho_K (S_K - u_K):
//   rho* = m q,  (rho u_n)* = m q S*,  (rho u_t)* = m q u_t,
//   E* = q ((S_K - u_K) E_K + (S* - u_K)(m S* + p_K)).
template <int D>
__device__ __forceinline__ void hllc(const double (&L)[5], const double (&R)[5], double gamma,
                                          double gm1inv, double (&F)[5]) {
  // No implicit contraction: every fused multiply-add is written out, so
  // every inlined copy of the solver rounds the same way (a face computed by
  // a tile's interior thread or by its boundary role gives the same bits),
  // and the kinetic term is symmetric in the velocity components (a y face
  // solved as an x face with u and v exchanged gives the same bits).
#pragma clang fp contract(off)
  const double rL = L[0], uL = L[1 + D], pL = L[4];
  const double rR = R[0], uR = R[1 + D], pR = R[4];
  const double gpL = gamma * pL, gpR = gamma * pR;
  const double cL = gpL * rsq_nr(gpL * rL);
  const double cR = gpR * rsq_nr(gpR * rR);
  const double SL = fmin(uL - cL, uR - cR);
  const double SR = fmax(uL + cL, uR + cR);
  const double mL = rL * (SL - uL), mR = rR * (SR - uR);
  const double Ss = div_nr(fma(-mR, uR, fma(mL, uL, pR - pL)), mL - mR);
  const bool left = (SL >= 0.0) || (Ss >= 0.0);
  const double S = left ? SL : SR;
  const double m = left ? mL : mR;
  const bool corr = left ? (SL < 0.0) : (SR > 0.0);  // not supersonic on the upwind side
  double W[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) W[v] = left ? L[v] : R[v];
  const double rho = W[0], un = W[1 + D], p = W[4];
  const double ke = (W[1] * W[1] + W[2] * W[2]) + W[3] * W[3];
  const double E = fma(0.5 * rho, ke, p * gm1inv);
  const double mass = rho * un;
  F[0] = mass;
  F[1] = mass * W[1];
  F[2] = mass * W[2];
  F[3] = mass * W[3];
  F[1 + D] = fma(mass, W[1 + D], p);
  F[4] = un * (E + p);
  if (corr) {
    const double q = rcp_nr(S - Ss);
    const double factor = m * q;
    const double d0 = factor - rho;
    double dU[5];
    dU[0] = d0;
    dU[1] = d0 * W[1];
    dU[2] = d0 * W[2];
    dU[3] = d0 * W[3];
    dU[1 + D] = fma(factor, Ss, -mass);
    dU[4] = fma(q, fma(S - un, E, (Ss - un) * fma(m, Ss, p)), -E);
#pragma unroll
    for (int v = 0; v < 5; ++v) F[v] = fma(S, dU[v], F[v]);
  }
}

// Per-direction CFL signal of the corner-transport-upwind step:
// max_d (|u_d| + c)/dx_d.
__device__ __forceinline__ double signal_speed_dir(const double (&u)[5], const GridGeom& g) {
  double w[5], inv;
  prim(u, g.gamma, g.small_p, w, inv);
  const double gp = g.gamma * w[4];
  const double c = gp * rsq_nr(gp * w[0]);
  return fmax(fmax((fabs(w[1]) + c) * g.inv_dx[0], (fabs(w[2]) + c) * g.inv_dx[1]), (fabs(w[3]) + c) * g.inv_dx[2]);
}

__device__ __forceinline__ double signal_speed(const double (&u)[5], const GridGeom& g) {
  double w[5], inv;
  prim(u, g.gamma, g.small_p, w, inv);
  const double gp = g.gamma * w[4];
  const double c = gp * rsq_nr(gp * w[0]);
  return ((fabs(w[1]) + c) * g.inv_dx[0] + (fabs(w[2]) + c) * g.inv_dx[1]) + (fabs(w[3]) + c) * g.inv_dx[2];
}

// Workgroup -> tile map that keeps spatially consecutive tiles on one XCD
// (workgroups are dealt to the 8 XCDs round-robin, each XCD has its own L2):
// XCD x takes the contiguous range [x*per, (x+1)*per) of tiles.
__device__ __forceinline__ long xcd_tile(long w, long total) {
  const long per = (total + 7) / 8;
  return (w % 8) * per + w / 8;
}

// ---------------------------------------------------------------------------
// Fused step.  Workgroups of whole wavefront quartets (256 threads for T =
// 16) so that two of them share a CU evenly across its four SIMDs (a 320-
// thread workgroup, one thread per predictor cell, packed only one per CU).
// Thread t owns tile cell (t % T, t / T) and keeps that column's primitives
// for planes j, j+1 and their difference to plane j-1 in registers.  The one-cell ring around the tile
// (4T cells) is a second item of roles 0..4T-1 whose z windows live in LDS;
// the two-deep halo cells that only feed ring slopes (4T+4 cells) are a
// second item of the next roles.  Each thread computes the x
// and y fluxes of its own low faces and its z flux; the last 2T roles also
// take the tile's high x and y boundary faces.  The ring is on the first
// wavefront of the role order and the boundary faces on the last, so no
// wavefront carries both extra items.
template <int T>
struct Tile {
  static constexpr int NI = T * T;   // tile cells
  static constexpr int NR = 4 * T;   // ring cells
  static constexpr int NE = 4 * T + 4;
  static constexpr int NT = (NI > ((NR + NE + 63) / 64) * 64) ? NI : ((NR + NE + 63) / 64) * 64;
  static constexpr int WS = T + 4;    // sW row pitch (x = -2 .. T+1)
  static constexpr int NQ = (T + 1) * T;
  // ring cell r: side r/T: 0 x=-1, 1 x=T, 2 y=-1, 3 y=T
  __device__ static void ring_of(int r, int& x, int& y) {
    const int side = r / T, s = r % T;
    x = side == 0 ? -1 : side == 1 ? T : s;
    y = side == 2 ? -1 : side == 3 ? T : s;
  }
  __device__ static void extra_of(int e, int& x, int& y) {
    if (e < 4 * T) {
      const int side = e / T, s = e % T;
      x = side == 0 ? -2 : side == 1 ? T + 1 : s;
      y = side == 2 ? -2 : side == 3 ? T + 1 : s;
      return;
    }
    const int c = e - 4 * T;
    x = (c & 1) ? T : -1;
    y = (c & 2) ? T : -1;
  }
};

// van Leer's harmonic slope without a branch: (a|b| + |a|b) / (|a| + |b|)
// equals 2ab/(a+b) when ab > 0 and 0 otherwise; the denominator is kept
// positive by the smallest normal double.  The two products are rounded
// separately (no contraction into an fma): for ab < 0 they are exact
// negatives of each other, so the numerator is exactly zero (an fma would
// leave the rounding error of one product).  Costs 0.8% of the step.
__device__ __forceinline__ double van_leer_sf(double a, double b) {
#pragma clang fp contract(off)
  const double num = a * fabs(b) + fabs(a) * b;
  const double den = (fabs(a) + fabs(b)) + 2.2250738585072014e-308;
  return div_nr(num, den);
}

// Positivity check of the six face states t +- s_d/2 of one cell: their
// densities and pressures are all positive exactly when t > |s_d|/2 for every
// d.  On exit wt is the state the face states extrapolate from and h the
// half-slope factor: (t, 0.5), or for the first-order fallback (wc, 0).
__device__ __forceinline__ bool face_check(const double (&t)[5], const double (&wc)[5], const double (&sx)[5],
                                           const double (&sy)[5], const double (&sz)[5], double (&wt)[5],
                                           double& h) {
  const double hr = 0.5 * fmax(fmax(fabs(sx[0]), fabs(sy[0])), fabs(sz[0]));
  const double hp = 0.5 * fmax(fmax(fabs(sx[4]), fabs(sy[4])), fabs(sz[4]));
  const bool ok = (t[0] - hr > 0.0) && (t[0] + hr > 0.0) && (t[4] - hp > 0.0) && (t[4] + hp > 0.0);
#pragma unroll
  for (int v = 0; v < 5; ++v) wt[v] = t[v];
  h = 0.5;
  if (__builtin_expect(!ok, 0)) {  // rare: a branch the wavefront skips, not selects
#pragma unroll
    for (int v = 0; v < 5; ++v) wt[v] = wc[v];
    h = 0.0;
  }
  return ok;
}

// Predictor of one cell: half step with all three directions, then the
// positivity check of the six face states (face_check).
__device__ __forceinline__ bool predict(const double (&wc)[5], double inv, const double (&sx)[5],
                                        const double (&sy)[5], const double (&sz)[5], double gamma,
                                        double lamx, double lamy, double lamz, double (&wt)[5], double& h) {
  const double gp = gamma * wc[4];
  double acc[5];
  {  // x: normal velocity wc[1]
    const double q = lamx * wc[1];
    acc[0] = fma(q, sx[0], (lamx * wc[0]) * sx[1]);
    acc[1] = fma(q, sx[1], (lamx * inv) * sx[4]);
    acc[2] = q * sx[2];
    acc[3] = q * sx[3];
    acc[4] = fma(q, sx[4], (lamx * gp) * sx[1]);
  }
  {  // y
    const double q = lamy * wc[2];
    acc[0] = fma(q, sy[0], fma(lamy * wc[0], sy[2], acc[0]));
    acc[1] = fma(q, sy[1], acc[1]);
    acc[2] = fma(q, sy[2], fma(lamy * inv, sy[4], acc[2]));
    acc[3] = fma(q, sy[3], acc[3]);
    acc[4] = fma(q, sy[4], fma(lamy * gp, sy[2], acc[4]));
  }
  {  // z
    const double q = lamz * wc[3];
    acc[0] = fma(q, sz[0], fma(lamz * wc[0], sz[3], acc[0]));
    acc[1] = fma(q, sz[1], acc[1]);
    acc[2] = fma(q, sz[2], acc[2]);
    acc[3] = fma(q, sz[3], fma(lamz * inv, sz[4], acc[3]));
    acc[4] = fma(q, sz[4], fma(lamz * gp, sz[3], acc[4]));
  }
  double t[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) t[v] = fma(-0.5, acc[v], wc[v]);
  return face_check(t, wc, sx, sy, sz, wt, h);
}

// LDS of one tile step.
template <int T>
struct Smem {
  static constexpr int NT = Tile<T>::NT, NR = Tile<T>::NR, WS = Tile<T>::WS, NQ = Tile<T>::NQ;
  double sW[5][WS * WS];   // primitives of plane j, tile + 2-halo (index (y+2)*WS + x+2)
  double sQx[5][NQ];       // high-x face state of cell (x, y), x = -1..T-1: index y*(T+1) + x+1
  double sQy[5][NQ];       // high-y face state of cell (x, y), y = -1..T-1: index (y+1)*T + x
  double sRx[5][T];        // low-x face state of ring cell (T, y)
  double sRy[5][T];        // low-y face state of ring cell (x, T)
  double sRing[3][5][NR];  // ring z windows (planes mod 3)
  // Conserved state of the own cells, planes mod 3: each thread keeps its
  // column's last three prefetched planes here and takes the old state of
  // the plane it updates from this slot (thread-private, no barrier
  // needed), so the update reloads nothing from global memory.
  double sU[3][5][Tile<T>::NI];
  // The x / y fluxes overwrite the face states: the flux at face (x, y) goes
  // to the slot of the high-side state of its left / lower cell, read only
  // by the thread that computes that face (sQx index y*(T+1) + x, x = 0..T;
  // sQy index y*T + x, y = 0..T).
  unsigned long long sRed[4];  // one per wavefront of a workgroup of up to 256 threads
  int sCnt[3];
};

// Leaf steps over views (GV) may restrict the new state into the parent
// block (ParentOut), fused into the update.  Cell (i, j, k) of a block at
// position (x, y, z) of its level lies in octant (x&1, y&1, z&1) of its
// parent; the parent cell ((x&1) N + i, (y&1) N + j, (z&1) N + k) / 2 takes
// the mean of its eight cells, the 2 x 2 of a plane from neighbouring lanes
// (cells (i, i^1) are lanes t, t^1, rows (j, j^1) lanes t, t^T), then the
// even plane plus the odd one.  For leaves whose state is final after the
// step (refluxing leaves it alone).

// One z pencil of one T x T column tile of an N^3 block, updated from Uin into
// Uout.  A pencil is plen consecutive planes of the global z axis (part of
// a block, or several blocks); tile_in_sim = layer * (column tiles of one
// z layer) + (block_xy * (N/T)^2 + in-plane tile), block_xy = bx + nb0*by,
// so the pencil covers global planes [layer*plen, (layer+1)*plen).  dt is
// cfl / max signal speed (ws->sig[slot]) when cfl > 0, else dt_host.  The
// new state's signal speed goes to ws->sig[(slot+1)%3]; the first pencil of
// the grid also records dt and clears ws->sig[(slot+2)%3].  Must be entered
// by all NT threads of the workgroup.
//
// MOL = false: the predictor-corrector step (face states from the half-step
// predicted centre).  MOL = true: one method-of-lines stage of an SSP
// Runge-Kutta step (face states from the cell centre; result
// a0*U0 + a1*(Uin - dt div F) when st.U0 is set).  A later stage (st.stage
// > 0) takes the dt its first stage recorded; only the last stage reduces
// the signal speed.  Uout may be st.U0 (each cell of U0 is read only by the
// thread that then writes it), never Uin.
//
// GV = true (predictor-corrector only): Uin holds guarded views
// ([block][var][N+2VG]^3, the VG guard layers filled) and the pencil is the
// whole z extent of the blocks of column gv_cols[tile_in_sim / (N/T)^2]:
// up to four blocks of one level stacked in z, bottom first, unused entries
// -1 (or the one block of that index when gv_cols is null).  Plane k is
// read from the view of the block that holds it, the planes below the
// first block and above the last from their guard layers; since a block's
// guard planes toward the next block of its column hold copies of that
// block's cells, the pencil reads exactly what one pencil per block reads.
// With a tile spanning the block plane (T == N) Uin holds plane halos
// (PlaneHalo<N>: the guard cells only) and the own column's interior
// planes come from the blocks' states in Uout, which this workgroup reads
// before it writes them.
// The result goes to the blocks in compact layout in Uout, dt is the one
// recorded in ws->dt_last, and the new state's signal speed goes to
// ws->sig[(slot+1)%3] only when gv_emit is set (event counters always).
// With po.U set, the new state's restriction also goes to the parent
// blocks (ParentOut above), the even planes' 2 x 2 sums held in psum
// (LDS, 5 (T/2)^2 doubles, each slot used by one thread only).
template <int N, int T, bool MOL = false, bool GV = false>
__device__ __forceinline__ void tile_step(const GridGeom& g, const double* __restrict__ Uin, double* Uout,
                                          WorkHeader* ws, double dt_host, double cfl, int slot,
                                          long tile_in_sim, int plen, Smem<T>& sm,
                                          const StageArgs& st = StageArgs{nullptr, 0.0, 0.0, 0, 1},
                                          const int4* gv_cols = nullptr, bool gv_emit = false,
                                          ParentOut po = ParentOut{nullptr, nullptr, nullptr},
                                          double* psum = nullptr) {
  static_assert(!(GV && MOL), "guarded-view input is for the predictor-corrector step");
  using TL = Tile<T>;
  constexpr int NT = TL::NT, NI = TL::NI, NR = TL::NR, NE = TL::NE, WS = TL::WS;
  constexpr int TPB = (N / T) * (N / T);
  constexpr long VS = Layout<N>::VS;
  constexpr long PS = Layout<N>::PS;
  constexpr int GP = Guarded<N, VG>::P;

  const int tid = threadIdx.x;
  const long nxy = GV ? 1 : (long)g.nb[0] * g.nb[1] * TPB;  // column tiles of one z layer
  const int NZ = g.nb[2] * N;
  const long layer = GV ? 0 : tile_in_sim / nxy;
  const long cxy = GV ? tile_in_sim : tile_in_sim % nxy;
  int4 gcol = make_int4(0, -1, -1, -1);  // GV: the blocks of the pencil, bottom first
  if constexpr (GV) gcol = gv_cols ? gv_cols[cxy / TPB] : make_int4((int)(cxy / TPB), -1, -1, -1);
  const int ncolb = GV ? 1 + (gcol.y >= 0) + (gcol.z >= 0) + (gcol.w >= 0) : 1;
  const int z0 = GV ? 0 : (int)(layer * plen), z1 = GV ? N * ncolb : z0 + plen;  // planes of the pencil
  const long bxy = GV ? (long)gcol.x : cxy / TPB;  // block (bx, by, 0), or the first block
  const int tile = (int)(cxy % TPB);
  const int bx = (int)(bxy % g.nb[0]);
  const int by = (int)(bxy / g.nb[0]);
  const int lx0 = (tile % (N / T)) * T, ly0 = (tile / (N / T)) * T;  // tile origin inside the block
  const int X0 = bx * N + lx0, Y0 = by * N + ly0;

  if (tid < 3) sm.sCnt[tid] = 0;

  double dt = dt_host;
  if constexpr (GV) {
    dt = ws->dt_last;
  } else {
    if (MOL && st.stage > 0) {
      if (cfl > 0.0) dt = ws->dt_last;
    } else {
      if (cfl > 0.0) dt = cfl / __longlong_as_double(ws->sig[slot]);
      if (tile_in_sim == 0 && tid == 0) {
        ws->dt_last = dt;
        ws->sig[(slot + 2) % 3] = 0ull;
      }
    }
  }
  const bool emit = GV ? gv_emit : (!MOL || st.last);
  const double lamx = dt * g.inv_dx[0], lamy = dt * g.inv_dx[1], lamz = dt * g.inv_dx[2];
  const double gamma = g.gamma, gm1inv = 1.0 / (g.gamma - 1.0);

  // roles; the second items (ring, halo) and the boundary faces sit on the
  // wavefronts starting at rotation r so the busier wavefront moves between
  // SIMDs from one workgroup to the next: r steps by one between the
  // consecutive workgroups of an XCD (workgroups are dealt to the 8 XCDs in
  // turn) and by two between workgroups b and b + 256, the two a CU
  // receives first (measured: 1.2% faster than without the second term,
  // 3% slower with a step of one there)
  // (a workgroup may be wider than NT, e.g. 8^3 tiles in a 256-thread batch
  // launch: the threads beyond NT only take part in the barriers)
  const bool member = tid < NT;
  const int rot = (int)(((blockIdx.x >> 3) + (blockIdx.x >> 8) * 2) & 3);
  const int role = member ? (tid + 64 * rot) % NT : NT;
  const bool inner = tid < NI;
  const int cx = tid % T, cy = tid / T;                // valid when inner
  const int cidx = (cy + 2) * WS + (cx + 2);
  const bool is_ring = role < NR;
  const bool ring_wave = role < 64;                     // uniform over a wavefront
  const bool is_extra = role >= NR && role < NR + NE;
  const int ring_id = role;                             // valid when is_ring
  int sx2 = 0, sy2 = 0;                                 // second item position
  if (is_ring) TL::ring_of(role, sx2, sy2);
  if (is_extra) TL::extra_of(role - NR, sx2, sy2);
  const int sidx2 = (sy2 + 2) * WS + (sx2 + 2);
  const int rside = role / T;                           // ring side (valid when is_ring)
  // offsets of plane 0 of the own column and of the second item, for the
  // planes that lie inside the block (z halo planes go through the map)
  // Addressing: a cell of global plane k sits at plane(U, k)[xy + v*VS],
  // where plane(U, k) is uniform over the workgroup (the plane's offset in
  // the z layer of blocks that holds it, after the z boundary map) and xy is
  // the cell's 32-bit offset inside its z layer (x/y boundary map applied
  // once, below).  Loads then take a scalar base and a vector offset.
  const long BZS = (long)g.nb[0] * g.nb[1] * Layout<N>::BS;  // size of a z layer of blocks
  auto plane_off = [&](int k) -> long {
    if constexpr (GV) {
      const int kb = k < 0 ? 0 : min(k / N, ncolb - 1);
      const int b = kb == 0 ? gcol.x : kb == 1 ? gcol.y : kb == 2 ? gcol.z : gcol.w;
      return (long)b * Guarded<N, VG>::BS + (long)(k - kb * N + VG) * Guarded<N, VG>::PS;
    } else {
      const int K = map_axis(k, NZ, g.bc[2]);
      return (long)((unsigned)K / N) * BZS + (long)((unsigned)K % N) * PS;
    }
  };
  // output plane k (compact layout)
  auto out_off = [&](int k) -> long {
    if constexpr (GV) {
      const int kb = k / N;  // k in [0, z1)
      const int b = kb == 0 ? gcol.x : kb == 1 ? gcol.y : kb == 2 ? gcol.z : gcol.w;
      return (long)b * Layout<N>::BS + (long)(k - kb * N) * PS;
    } else {
      return plane_off(k);
    }
  };
  // (byte offsets: a z layer of blocks is below 4 GiB, checked on the host)
  const unsigned own_xy = GV ? 8u * (unsigned)((ly0 + cy + VG) * GP + (lx0 + cx + VG))
                             : 8u * (unsigned)Layout<N>::at(bxy, lx0 + cx, ly0 + cy, 0);
  const unsigned own_out = GV ? 8u * (unsigned)((ly0 + cy) * N + (lx0 + cx)) : own_xy;
  const unsigned sec_xy = !(is_ring || is_extra) ? 0u
                          : GV ? 8u * (unsigned)((ly0 + sy2 + VG) * GP + (lx0 + sx2 + VG))
                               : 8u * (unsigned)cell_offset<N>(g, X0 + sx2, Y0 + sy2, 0);
  // GV with a tile spanning the block plane: Uin holds plane halos, the own
  // column's interior planes come from the state in Uout (each block of the
  // column is read here before this workgroup overwrites it); whole halo
  // planes take the view's in-plane offsets (own_xy, sec_xy)
  constexpr bool GVH = GV && T == N;
  using PH = PlaneHalo<N>;
  const unsigned sec_ring = (GVH && (is_ring || is_extra)) ? 8u * (unsigned)PH::ring_index(sx2, sy2) : 0u;
  // block of the column holding plane k, and the plane's index in it
  auto col_block = [&](int k, int& kl) -> int {
    const int kb = k < 0 ? 0 : min(k / N, ncolb - 1);
    kl = k - kb * N;
    return kb == 0 ? gcol.x : kb == 1 ? gcol.y : kb == 2 ? gcol.z : gcol.w;
  };
  auto halo_plane = [&](int kl) -> long {  // whole halo plane kl (kl < 0 or kl >= N)
    return (long)N * PH::RP + (long)(kl < 0 ? kl + VG : kl - N + VG) * PH::FP;
  };
  // own column, plane k
  auto load_own = [&](int k, double (&u)[5]) {
    if constexpr (GVH) {
      int kl;
      const int b = col_block(k, kl);
      if (kl >= 0 && kl < N) load_cons_at<N>(Uout + (long)b * Layout<N>::BS + (long)kl * PS, own_out, u);
      else load_cons_vs<PH::VS>(Uin + (long)b * PH::BS + halo_plane(kl), own_xy, u);
    } else {
      load_cons_at<N, GV>(Uin + plane_off(k), own_xy, u);
    }
  };
  // second item (ring or halo cell), plane k
  auto load_sec = [&](int k, double (&u)[5]) {
    if constexpr (GVH) {
      int kl;
      const int b = col_block(k, kl);
      if (kl >= 0 && kl < N) load_cons_vs<PH::VS>(Uin + (long)b * PH::BS + (long)kl * PH::RP, sec_ring, u);
      else load_cons_vs<PH::VS>(Uin + (long)b * PH::BS + halo_plane(kl), sec_xy, u);
    } else {
      load_cons_at<N, GV>(Uin + plane_off(k), sec_xy, u);
    }
  };

  // Wb, Wc: primitives of planes j, j+1; dzm: Wb minus the plane below
  // (the z slope's lower difference, carried instead of that plane)
  double Wb[5], Wc[5], dzm[5], dzp[5];
  double inv_b = 1.0, inv_c = 1.0;  // 1/rho of planes j and j+1, from the primitive recovery
  double un_next[5], u2_next[5];
  // acc: plane j-1's x/y flux divergence minus its lower z flux, carried to
  // the next plane, whose z flux completes the update of plane j-1
  double zp_prev[5], acc[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    Wb[v] = Wc[v] = dzm[v] = dzp[v] = 0.0;
    un_next[v] = u2_next[v] = 0.0;
    zp_prev[v] = acc[v] = 0.0;
  }
  int n_floor = 0, n_fb = 0, n_bad = 0;
  double smax = 0.0;

  // prologue: planes z0-2, z0-1 of the own column, prefetch plane z0
  if (inner) {
    double u[5], tmp;
    load_own(z0 - 2, u);
    prim(u, gamma, g.small_p, dzm, tmp);
    load_own(z0 - 1, u);
    prim(u, gamma, g.small_p, Wb, inv_b);
#pragma unroll
    for (int v = 0; v < 5; ++v) dzm[v] = Wb[v] - dzm[v];
    load_own(z0, un_next);
  }
  if (is_ring) {
    double u[5], w[5], tmp;
    load_sec(z0 - 1, u);
    prim(u, gamma, g.small_p, w, tmp);
#pragma unroll
    for (int v = 0; v < 5; ++v) sm.sRing[(z0 + 2) % 3][v][ring_id] = w[v];
    load_sec(z0, u2_next);
  }
  if (is_extra) load_sec(z0, u2_next);

  for (int j = z0 - 1; j <= z1; ++j) {
    const bool mid = (j >= z0) && (j < z1);
    const int sl_m = (j + 5) % 3, sl_0 = (j + 3) % 3, sl_p = (j + 4) % 3;  // ring slots of planes j-1, j, j+1
    // -- own column: plane j+1 from the prefetch, publish plane j; second
    // item: ring cell window (planes j..j+1) or halo cell (plane j)
    if (inner) {
      const int fl = prim(un_next, gamma, g.small_p, Wc, inv_c);
      if (j + 1 >= z0 && j + 1 < z1) n_floor += fl;
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        sm.sW[v][cidx] = Wb[v];
        sm.sU[(j + 1) % 3][v][tid] = un_next[v];
      }
    }
    if (is_ring) {
      double w[5], tmp;
      prim(u2_next, gamma, g.small_p, w, tmp);
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        sm.sRing[sl_p][v][ring_id] = w[v];
        sm.sW[v][sidx2] = sm.sRing[sl_0][v][ring_id];
      }
    }
    if (is_extra && mid) {
      double w[5], tmp;
      prim(u2_next, gamma, g.small_p, w, tmp);
#pragma unroll
      for (int v = 0; v < 5; ++v) sm.sW[v][sidx2] = w[v];
    }
    // -- prefetches for the next planes, issued only after the current
    // values are consumed: they then land in the same registers, and nothing
    // waits for them until the next plane
    __builtin_amdgcn_sched_barrier(0);
    if (inner && j + 2 <= z1 + 1) load_own(j + 2, un_next);
    if (is_ring && j + 2 <= z1 + 1) load_sec(j + 2, u2_next);
    if (is_extra && mid && j + 1 < z1) load_sec(j + 1, u2_next);
    __syncthreads();

    // -- predictor: own cell (every plane), ring cell (pencil planes)
    double xm[5], ym[5], zm[5], zp[5];
    if (inner) {
      double sx[5], sy[5], sz[5], wt[5], h;
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const double c = Wb[v];
        sx[v] = van_leer_sf(c - sm.sW[v][cidx - 1], sm.sW[v][cidx + 1] - c);
        sy[v] = van_leer_sf(c - sm.sW[v][cidx - WS], sm.sW[v][cidx + WS] - c);
        dzp[v] = Wc[v] - c;
        sz[v] = van_leer_sf(dzm[v], dzp[v]);
      }
      bool ok;
      if constexpr (MOL)
        ok = face_check(Wb, Wb, sx, sy, sz, wt, h);
      else
        ok = predict(Wb, inv_b, sx, sy, sz, gamma, lamx, lamy, lamz, wt, h);
      if (mid && !ok) ++n_fb;
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        xm[v] = fma(-h, sx[v], wt[v]);
        ym[v] = fma(-h, sy[v], wt[v]);
        zm[v] = fma(-h, sz[v], wt[v]);
        zp[v] = fma(h, sz[v], wt[v]);
      }
      if (mid) {
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          sm.sQx[v][cy * (T + 1) + cx + 1] = fma(h, sx[v], wt[v]);
          sm.sQy[v][(cy + 1) * T + cx] = fma(h, sy[v], wt[v]);
        }
      }
    }
    if (is_ring && mid) {
      // the ring's wavefront is the last to reach the next barrier: let it
      // issue ahead of the other workgroup's wavefront on its SIMD
      __builtin_amdgcn_s_setprio(2);
      double wc[5], sx[5], sy[5], sz[5], wt[5], h;
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        wc[v] = sm.sRing[sl_0][v][ring_id];
        sx[v] = van_leer_sf(wc[v] - sm.sW[v][sidx2 - 1], sm.sW[v][sidx2 + 1] - wc[v]);
        sy[v] = van_leer_sf(wc[v] - sm.sW[v][sidx2 - WS], sm.sW[v][sidx2 + WS] - wc[v]);
        sz[v] = van_leer_sf(wc[v] - sm.sRing[sl_m][v][ring_id], sm.sRing[sl_p][v][ring_id] - wc[v]);
      }
      if constexpr (MOL)
        face_check(wc, wc, sx, sy, sz, wt, h);
      else
        predict(wc, rcp_nr(wc[0]), sx, sy, sz, gamma, lamx, lamy, lamz, wt, h);
      // the one face state of this ring cell that a tile face uses
      const int r = ring_id % T;
      if (rside == 0) {
#pragma unroll
        for (int v = 0; v < 5; ++v) sm.sQx[v][r * (T + 1)] = fma(h, sx[v], wt[v]);  // (-1, r) high x
      } else if (rside == 1) {
#pragma unroll
        for (int v = 0; v < 5; ++v) sm.sRx[v][r] = fma(-h, sx[v], wt[v]);           // (T, r) low x
      } else if (rside == 2) {
#pragma unroll
        for (int v = 0; v < 5; ++v) sm.sQy[v][r] = fma(h, sy[v], wt[v]);            // (r, -1) high y
      } else {
#pragma unroll
        for (int v = 0; v < 5; ++v) sm.sRy[v][r] = fma(-h, sy[v], wt[v]);           // (r, T) low y
      }
    }
    // z faces of the own column; the ring's wavefront, which predicted a
    // second cell, takes its z faces after the barrier
    double fz[5];
    if (inner && j >= z0 && !ring_wave) hllc<2>(zp_prev, zm, gamma, gm1inv, fz);
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();

    // -- x and y fluxes: own low faces, plus the tile's high boundary faces
    // the ring's wavefront is the busiest of this phase too (its z faces
    // besides the x / y ones): it keeps the issue priority here
    if (ring_wave) __builtin_amdgcn_s_setprio(2);
    if (inner && j >= z0 && ring_wave) hllc<2>(zp_prev, zm, gamma, gm1inv, fz);
    if (mid) {
      if (inner) {
        double WL[5], F[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) WL[v] = sm.sQx[v][cy * (T + 1) + cx];
        hllc<0>(WL, xm, gamma, gm1inv, F);
#pragma unroll
        for (int v = 0; v < 5; ++v) sm.sQx[v][cy * (T + 1) + cx] = F[v];
#pragma unroll
        for (int v = 0; v < 5; ++v) WL[v] = sm.sQy[v][cy * T + cx];
        hllc<1>(WL, ym, gamma, gm1inv, F);
#pragma unroll
        for (int v = 0; v < 5; ++v) sm.sQy[v][cy * T + cx] = F[v];
      }
      if (role >= NT - 2 * T) {  // on the last wavefront, away from the ring's
        // x faces at (T, r) and y faces at (r, T) in one HLLC call: a y face
        // is an x face of the state with u and v exchanged (the flux is
        // exchanged back), which gives the same operations in the same order
        const int r = (role - (NT - 2 * T)) % T;
        const bool yface = role >= NT - T;
        const double* qL = yface ? (const double*)sm.sQy + (T * T + r) : (const double*)sm.sQx + (r * (T + 1) + T);
        const double* qR = yface ? (const double*)sm.sRy + r : (const double*)sm.sRx + r;
        double* fo = yface ? (double*)sm.sQy + (T * T + r) : (double*)sm.sQx + (r * (T + 1) + T);
        double WL[5], WR[5], F[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          WL[v] = qL[v * TL::NQ];
          WR[v] = qR[v * T];
        }
        if (yface) {
          const double a = WL[1], b = WR[1];
          WL[1] = WL[2];
          WL[2] = a;
          WR[1] = WR[2];
          WR[2] = b;
        }
        hllc<0>(WL, WR, gamma, gm1inv, F);
        if (yface) {
          const double a = F[1];
          F[1] = F[2];
          F[2] = a;
        }
#pragma unroll
        for (int v = 0; v < 5; ++v) fo[v * TL::NQ] = F[v];
      }
    }
    __builtin_amdgcn_s_setprio(0);
    // the base state of a stage is fetched before the barrier, so its
    // latency overlaps the wait (the old state comes from sU)
    const long off_u = plane_off(j - 1);
    double base[5];
    if constexpr (MOL) {
      if (inner && j >= z0 + 1 && st.U0) load_cons_at<N>(st.U0 + off_u, own_xy, base);
    }
    __syncthreads();

    // -- update plane j-1, carry plane j's divergence
    if (inner) {
      double dxy[5];
      if (mid) {
        const int qx = cy * (T + 1) + cx, qy = cy * T + cx;
#pragma unroll
        for (int v = 0; v < 5; ++v)
          dxy[v] = lamx * (sm.sQx[v][qx + 1] - sm.sQx[v][qx]) + lamy * (sm.sQy[v][qy + T] - sm.sQy[v][qy]);
      }
      if (j >= z0 + 1) {
        double un[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) un[v] = sm.sU[(j - 1) % 3][v][tid] - fma(lamz, fz[v], acc[v]);
        if constexpr (MOL) {
          if (st.U0) {
#pragma unroll
            for (int v = 0; v < 5; ++v) un[v] = st.a0 * base[v] + st.a1 * un[v];
          }
        }
        // stored at once (holding the values for the next plane's store
        // phase cost registers and measured 4% slower)
        const long oo = GV ? out_off(j - 1) : off_u;
#pragma unroll
        for (int v = 0; v < 5; ++v)
          __builtin_nontemporal_store(un[v], (double*)((char*)(Uout + oo + v * VS) + own_out));
        bool good = un[0] > 0.0 && un[4] > 0.0;
#pragma unroll
        for (int v = 0; v < 5; ++v) good = good && isfinite(un[v]);
        if (!good) ++n_bad;
        if (emit) {
          const double s = signal_speed(un, g);
          smax = (s > smax || !(s == s)) ? s : smax;
        }
        if constexpr (GV) {
          if (po.U) {  // (uniform; every lane of the wavefront is an inner cell)
            double q[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) q[v] = un[v] + __shfl_xor(un[v], 1, 64);
#pragma unroll
            for (int v = 0; v < 5; ++v) q[v] = q[v] + __shfl_xor(q[v], T, 64);
            int kl;
            const int b = col_block(j - 1, kl);
            if (((cx | cy) & 1) == 0) {  // one lane per 2 x 2; psum: its even-plane sums (LDS, own slot)
              double* ps = psum + (cy >> 1) * (T / 2) + (cx >> 1);
              if ((kl & 1) == 0) {
#pragma unroll
                for (int v = 0; v < 5; ++v) ps[v * (NI / 4)] = q[v];
              } else {
                const int4 bp = po.pos[b];
                const long pc = Layout<N>::at(po.parent[b], ((bp.x & 1) * N + lx0 + cx) >> 1,
                                              ((bp.y & 1) * N + ly0 + cy) >> 1, ((bp.z & 1) * N + kl) >> 1);
#pragma unroll
                for (int v = 0; v < 5; ++v) po.U[pc + v * VS] = (ps[v * (NI / 4)] + q[v]) * 0.125;
              }
            }
          }
        }
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        if (mid) acc[v] = fma(-lamz, fz[v], dxy[v]);
        zp_prev[v] = zp[v];
        dzm[v] = dzp[v];
        Wb[v] = Wc[v];
      }
      inv_b = inv_c;
    }
  }

  if (n_floor) atomicAdd(&sm.sCnt[0], n_floor);
  if (n_fb) atomicAdd(&sm.sCnt[1], n_fb);
  if (n_bad) atomicAdd(&sm.sCnt[2], n_bad);
  if (emit) wg_max_to(smax, sm.sRed, &ws->sig[(slot + 1) % 3]);
  else __syncthreads();  // sCnt is complete
  if (tid == 0) {
    for (int c = 0; c < 3; ++c)
      if (sm.sCnt[c]) atomicAdd(&ws->cnt[c], (unsigned long long)sm.sCnt[c]);
  }
}

// One grid: one workgroup per pencil, XCD-aware order.
template <int N, int T>
__global__ __launch_bounds__(Tile<T>::NT, 2) void step_kernel(GridGeom g, StepArgs a, long ntiles, int plen) {
  __shared__ Smem<T> sm;
  const long tile_id = xcd_tile(blockIdx.x, ntiles);
  if (tile_id >= ntiles) return;
  tile_step<N, T>(g, a.Uin, a.Uout, a.ws, a.dt, a.cfl, a.slot, tile_id, plen, sm);
}

// One method-of-lines stage of one grid (same launch shape as step_kernel).
template <int N, int T>
__global__ __launch_bounds__(Tile<T>::NT, 2) void stage_kernel(GridGeom g, StepArgs a, StageArgs st, long ntiles,
                                                               int plen) {
  __shared__ Smem<T> sm;
  const long tile_id = xcd_tile(blockIdx.x, ntiles);
  if (tile_id >= ntiles) return;
  tile_step<N, T, true>(g, a.Uin, a.Uout, a.ws, a.dt, a.cfl, a.slot, tile_id, plen, sm, st);
}

// Many grids in one persistent launch: workgroup w takes items w, w + G,
// w + 2G, ... of the work list (G workgroups).  The item sequence depends
// only on the launch shape, so the loop and every barrier in it are in
// uniform control flow.  (A shared atomic counter broadcast through LDS was
// compiled into a loop whose lanes reached the barrier without the fetching
// lane's store, and never ended.)  Every grid uses its own device dt (cfl /
// its own maximum signal speed).  N: the block size of every member whose
// items are listed — the host launches one kernel per size class over that
// class's range of the work list — so the kernel holds one instance of the
// tile step (a kernel holding all three spilled registers and ran 8% slower
// on a mixed ensemble).  An item of a member of another size would be
// skipped, never misread.
template <int N, int T>
__global__ __launch_bounds__(Tile<T>::NT, 2) void batch_step_kernel(const BatchSim* __restrict__ sims,
                                                                    const BatchItem* __restrict__ items, int nitems,
                                                                    long step, double cfl, int nseg) {
  __shared__ Smem<T> sm;
  // The items in 8 contiguous ranges, one per XCD (workgroups are dealt to
  // the 8 XCDs in turn), so tiles next to each other in the work list --
  // neighbours in a grid -- share an L2; a grid of workgroups that is not a
  // multiple of 8 takes the items in plain stride.
  const int G = (int)gridDim.x;
  const bool by_xcd = G % 8 == 0;
  const int nx = by_xcd ? G / 8 : G;
  const int x = by_xcd ? (int)blockIdx.x % 8 : 0;
  const int l = by_xcd ? (int)blockIdx.x / 8 : (int)blockIdx.x;
  const int per = by_xcd ? (nitems + 7) / 8 : nitems;
  const int end = min(nitems, (x + 1) * per);
  for (int it = x * per + l; it < end; it += nx) {
    const BatchItem w = items[it];
    const BatchSim d = sims[w.sim];  // a copy: its fields stay loaded across the tile step's barriers
    const int par = (int)((d.parity0 + step) & 1);
    const int slot = (int)((d.slot0 + step) % 3);
    const double* Uin = par ? d.U1 : d.U0;
    double* Uout = par ? d.U0 : d.U1;
    if (d.nxb == N) tile_step<N, T>(d.geom, Uin, Uout, d.ws, 0.0, cfl, slot, w.tile, N / nseg, sm);
    __syncthreads();  // the next item reuses the LDS
  }
}

// ---------------------------------------------------------------------------
// Corner-transport-upwind (CTU) step: the corner-coupled form of the unsplit
// predictor-corrector solver (§2.2 Hydrodynamics), twelve HLLC solves per
// cell: normal predictor per direction, 1-D fluxes, corner states with
// lam_t/3 transverse corrections and their fluxes, final states with lam/2
// cross corrections and their fluxes, update (ctu_tile_kernel below).

// HLLC along a runtime direction (the solver is specialised per direction).
__device__ __forceinline__ void hllc_dir(int d, const double (&L)[5], const double (&R)[5], double gamma,
                                         double gm1inv, double (&F)[5]) {
  if (d == 0)
    hllc<0>(L, R, gamma, gm1inv, F);
  else if (d == 1)
    hllc<1>(L, R, gamma, gm1inv, F);
  else
    hllc<2>(L, R, gamma, gm1inv, F);
}

__device__ __forceinline__ void to_cons(const double* w, double gm1inv, double (&u)[5]) {
  u[0] = w[0];
  u[1] = w[0] * w[1];
  u[2] = w[0] * w[2];
  u[3] = w[0] * w[3];
  u[4] = w[4] * gm1inv + 0.5 * w[0] * ((w[1] * w[1] + w[2] * w[2]) + w[3] * w[3]);
}

// Primitive of a corrected conserved state; false when rho <= 0 or p <= 0.
__device__ __forceinline__ bool corrected_prim(const double (&u)[5], double gamma, double (&w)[5]) {
  if (!(u[0] > 0.0)) return false;
  const double inv = rcp_nr(u[0]);
  w[0] = u[0];
  w[1] = u[1] * inv;
  w[2] = u[2] * inv;
  w[3] = u[3] * inv;
  w[4] = (gamma - 1.0) * (u[4] - 0.5 * u[0] * ((w[1] * w[1] + w[2] * w[2]) + w[3] * w[3]));
  return w[4] > 0.0;
}

// Characteristic tracing of the normal predictor along d (the upwind
// projection of Colella 1990 / Stone et al. 2008): the primitive slope S is
// split over the waves of the primitive Jacobian A_d(W) -- with c the sound
// speed and u the normal velocity,
//   u - c:  amplitude a_- = S_p/(2c^2) - rho S_u/(2c), vector (1, -c/rho, 0, 0, c^2)
//   u:      entropy and shear, (S_rho - S_p/c^2, 0, S_t1, S_t2, 0)
//   u + c:  amplitude a_+ = S_p/(2c^2) + rho S_u/(2c), vector (1,  c/rho, 0, 0, c^2)
// -- and each face keeps the waves moving toward it within the step:
//   high face  W + sum over speeds s > 0 of (1 - lam s)/2 times the wave,
//   low face   W - sum over speeds s < 0 of (1 + lam s)/2 times the wave.
__device__ __forceinline__ void trace_faces(int d, const double (&w)[5], const double (&S)[5], double lam,
                                            double gamma, double inv_rho, double (&lo)[5], double (&hi)[5]) {
  const double rho = w[0], un = w[1 + d];
  const double c2 = gamma * w[4] * inv_rho;
  const double ic = rsq_nr(c2);                 // 1/c
  const double c = c2 * ic;
  const double ic2 = ic * ic;
  const double a = 0.5 * S[4] * ic2, b = 0.5 * rho * S[1 + d] * ic;
  const double am = a - b, ap = a + b;
  const double cr = c * inv_rho;
  double wm[5], w0[5], wp[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) wm[v] = w0[v] = wp[v] = 0.0;
  wm[0] = am;
  wm[1 + d] = -am * cr;
  wm[4] = am * c2;
  wp[0] = ap;
  wp[1 + d] = ap * cr;
  wp[4] = ap * c2;
  w0[0] = S[0] - S[4] * ic2;
#pragma unroll
  for (int v = 1; v < 4; ++v)
    if (v != 1 + d) w0[v] = S[v];
  const double sm = un - c, s0 = un, sp = un + c;
  const double hm = sm > 0.0 ? 0.5 * (1.0 - lam * sm) : 0.0, lm = sm < 0.0 ? 0.5 * (1.0 + lam * sm) : 0.0;
  const double h0 = s0 > 0.0 ? 0.5 * (1.0 - lam * s0) : 0.0, l0 = s0 < 0.0 ? 0.5 * (1.0 + lam * s0) : 0.0;
  const double hp = sp > 0.0 ? 0.5 * (1.0 - lam * sp) : 0.0, lp = sp < 0.0 ? 0.5 * (1.0 + lam * sp) : 0.0;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    hi[v] = w[v] + ((hm * wm[v] + h0 * w0[v]) + hp * wp[v]);
    lo[v] = w[v] - ((lm * wm[v] + l0 * w0[v]) + lp * wp[v]);
  }
}

// ---------------------------------------------------------------------------
// Corner-transport-upwind step as a z-marching column tile.  A workgroup of 128
// threads owns an 8 x 8 column tile of one block and marches it through the
// block's planes.  Thread t < 100 owns position (i, j) = (t % 10 - 1,
// t / 10 - 1) of the tile plus its one-cell ring; threads 100..127 gather
// the primitives of the 44 cells two deep around it (two cells each).
// Iteration p predicts plane k1 = p + 1 and finishes plane p:
//   A  primitives of plane p + 2 (own column), plane p + 1 published
//   B  normal predictor of plane k1 (face states), z 1-D flux at face k1
//   C  x / y 1-D fluxes of plane k1; corner fluxes F_{x|z}, F_{y|z} of p
//   D  corner fluxes F_{x|y}, F_{y|x} of plane k1, F_{z|x}, F_{z|y} at face k1
//   E  final fluxes: x / y of plane p, z at face k1
//   F  update of plane p
// Each position keeps what it needs from the plane below in registers (its
// z window of primitives, low x / y face states, high z face state, 1-D z
// flux, transverse 1-D flux differences, z corner fluxes, the combined
// z-face correction and the final z flux); neighbours exchange values
// through LDS.  Fallbacks are counted over exactly the faces the per-block
// step counts: a tile counts its high boundary faces only where they are
// the block's, and rows or columns one cell outside only at the block's
// border.
struct CtuTile {
  static constexpr int T = 8;
  static constexpr int P = T + 2;          // positions per row: cells -1..T
  static constexpr int NP = P * P;         // 100
  static constexpr int R = T + 4;          // plane rows of the primitives: cells -2..T+1
  static constexpr int NR = R * R;         // 144
  static constexpr int NO = NR - NP;       // 44 cells two deep
  static constexpr int NT = 128;
  __device__ static void outer_of(int e, int& x, int& y) {
    if (e < R) { x = e - 2; y = -2; return; }
    if (e < 2 * R) { x = e - R - 2; y = T + 1; return; }
    if (e < 2 * R + P) { x = -2; y = e - 2 * R - 1; return; }
    x = T + 1;
    y = e - 2 * R - P - 1;
  }
};

struct CtuTileSmem {
  double sW[5][CtuTile::NR];                      // primitives of plane k1, cells -2..T+1
  double sXh[2][5][CtuTile::NP];                  // high x face states, by plane parity
  double sYh[2][5][CtuTile::NP];                  // high y face states, by plane parity
  double sF1x[5][CtuTile::NP], sF1y[5][CtuTile::NP];   // 1-D x / y fluxes of k1, then the final x / y fluxes of p
  double sFxz[5][CtuTile::NP], sFyz[5][CtuTile::NP];   // F_{x|z}, F_{y|z} of plane p
  double sFxy[5][CtuTile::NP], sFyx[5][CtuTile::NP];   // z 1-D flux differences of p (phase B-C), then F_{x|y}, F_{y|x} of k1
  double sDzx[5][CtuTile::NP], sDzy[5][CtuTile::NP];   // F_{z|x}, F_{z|y} differences over plane p
  unsigned long long sRed[2];
  int sCnt[3];
};

// A corrected face state: the conserved form of the primitive face state w
// minus coef * d (d a flux difference, or a combination of them), back to
// primitives; falls back to w when the result has rho <= 0 or p <= 0
// (returns true then).
__device__ __forceinline__ bool corrected_state(const double (&w)[5], double coef, const double (&d)[5],
                                                double gamma, double gm1inv, double (&out)[5]) {
  double u[5];
  to_cons(w, gm1inv, u);
#pragma unroll
  for (int v = 0; v < 5; ++v) u[v] -= coef * d[v];
  const bool ok = corrected_prim(u, gamma, out);
  if (!ok) {
#pragma unroll
    for (int v = 0; v < 5; ++v) out[v] = w[v];
  }
  return !ok;
}

template <int N, bool TRACE>
__global__ __launch_bounds__(CtuTile::NT) void ctu_tile_kernel(GridGeom g, StepArgs a, long ntiles) {
  using C = CtuTile;
  constexpr int T = C::T, P = C::P, R = C::R;
  constexpr int TPB = (N / T) * (N / T);
  constexpr long PS = Layout<N>::PS, VS = Layout<N>::VS;
  __shared__ CtuTileSmem sm;
  const long tile_id = xcd_tile(blockIdx.x, ntiles);
  if (tile_id >= ntiles) return;
  const int tid = threadIdx.x;
  const long blk = tile_id / TPB;
  const int tile = (int)(tile_id % TPB);
  const int lx0 = (tile % (N / T)) * T, ly0 = (tile / (N / T)) * T;
  const int bx = (int)(blk % g.nb[0]), by = (int)((blk / g.nb[0]) % g.nb[1]);
  const int bz = (int)(blk / ((long)g.nb[0] * g.nb[1]));
  const int X0 = bx * N + lx0, Y0 = by * N + ly0, Z0 = bz * N;
  const int NZ = g.nb[2] * N;
  const long BZS = (long)g.nb[0] * g.nb[1] * Layout<N>::BS;
  WorkHeader* ws = a.ws;
  const int slot = a.slot;
  if (tid < 3) sm.sCnt[tid] = 0;
  double dt = a.dt;
  if (a.cfl > 0.0) dt = a.cfl / __longlong_as_double(ws->sig[slot]);
  if (tile_id == 0 && tid == 0) {
    ws->dt_last = dt;
    ws->sig[(slot + 2) % 3] = 0ull;
  }
  const double lx = dt * g.inv_dx[0], ly = dt * g.inv_dx[1], lz = dt * g.inv_dx[2];
  const double gamma = g.gamma, gm1inv = 1.0 / (g.gamma - 1.0);

  // roles
  const bool pos = tid < C::NP;
  const int i = pos ? tid % P - 1 : 0, j = pos ? tid / P - 1 : 0;
  const int q = tid;                                  // position index (when pos)
  const int rq = (j + 2) * R + (i + 2);               // own cell in sW
  const bool inner = pos && i >= 0 && i < T && j >= 0 && j < T;
  const int e0 = 2 * (tid - C::NP), e1 = e0 + 1;
  const bool out0 = !pos && e0 < C::NO, out1 = !pos && e1 < C::NO;
  int ox0 = 0, oy0 = 0, ox1 = 0, oy1 = 0;
  if (out0) C::outer_of(e0, ox0, oy0);
  if (out1) C::outer_of(e1, ox1, oy1);
  const int r0 = (oy0 + 2) * R + (ox0 + 2), r1 = (oy1 + 2) * R + (ox1 + 2);
  // which faces this tile counts fallbacks on (the per-block step's sets)
  const bool xhi_blk = lx0 + T == N, yhi_blk = ly0 + T == N;
  const bool cfx = i < T || xhi_blk;                   // x face i (low face of position i), i in [0, T]
  const bool cfy = j < T || yhi_blk;
  const bool crx = (i >= 0 && i < T) || (i == -1 && lx0 == 0) || (i == T && xhi_blk);   // column i in [-1, T]
  const bool cry = (j >= 0 && j < T) || (j == -1 && ly0 == 0) || (j == T && yhi_blk);
  // addresses: a cell of global plane k at plane_off(k) + its column's 32-bit byte offset
  auto plane_off = [&](int k) -> long {
    const int K = map_axis(k, NZ, g.bc[2]);
    return (long)((unsigned)K / N) * BZS + (long)((unsigned)K % N) * PS;
  };
  const unsigned own_xy = pos ? 8u * (unsigned)cell_offset<N>(g, X0 + i, Y0 + j, 0) : 0u;
  const unsigned o0_xy = out0 ? 8u * (unsigned)cell_offset<N>(g, X0 + ox0, Y0 + oy0, 0) : 0u;
  const unsigned o1_xy = out1 ? 8u * (unsigned)cell_offset<N>(g, X0 + ox1, Y0 + oy1, 0) : 0u;
  const double* Uin = a.Uin;

  double Wz0[5], Wz1[5], pre[5], pre1[5];
  double xlo[5], ylo[5], zhi[5], f1z[5], d1x[5], d1y[5], fzx[5], fzy[5], dzl[5], ffz[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    Wz0[v] = Wz1[v] = pre[v] = pre1[v] = 0.0;
    xlo[v] = ylo[v] = zhi[v] = f1z[v] = d1x[v] = d1y[v] = fzx[v] = fzy[v] = dzl[v] = ffz[v] = 0.0;
  }
  int n_floor = 0, n_fb = 0, n_bad = 0;
  double smax = 0.0;

  // prologue: own column planes Z0-2, Z0-1 and the prefetch of Z0; the
  // outer cells' plane Z0-1
  if (pos) {
    double u[5], tmp;
    load_cons_at<N>(Uin + plane_off(Z0 - 2), own_xy, u);
    prim(u, gamma, g.small_p, Wz0, tmp);
    load_cons_at<N>(Uin + plane_off(Z0 - 1), own_xy, u);
    prim(u, gamma, g.small_p, Wz1, tmp);
    load_cons_at<N>(Uin + plane_off(Z0), own_xy, pre);
  }
  if (out0) load_cons_at<N>(Uin + plane_off(Z0 - 1), o0_xy, pre);
  if (out1) load_cons_at<N>(Uin + plane_off(Z0 - 1), o1_xy, pre1);

  for (int p = Z0 - 2; p < Z0 + N; ++p) {
    const int k1 = p + 1;
    const bool mid = p >= Z0;                          // plane p is updated (and its x / y corner fluxes formed)
    const int par1 = k1 & 1, par0 = p & 1;
    // ---- A: primitives
    double Wz2[5];
    if (pos) {
      double tmp;
      const int fl = prim(pre, gamma, g.small_p, Wz2, tmp);
      if (inner && p + 2 < Z0 + N) n_floor += fl;
#pragma unroll
      for (int v = 0; v < 5; ++v) sm.sW[v][rq] = Wz1[v];
    }
    if (out0) {
      double w[5], tmp;
      prim(pre, gamma, g.small_p, w, tmp);
#pragma unroll
      for (int v = 0; v < 5; ++v) sm.sW[v][r0] = w[v];
    }
    if (out1) {
      double w[5], tmp;
      prim(pre1, gamma, g.small_p, w, tmp);
#pragma unroll
      for (int v = 0; v < 5; ++v) sm.sW[v][r1] = w[v];
    }
    __builtin_amdgcn_sched_barrier(0);
    if (pos && p + 3 <= Z0 + N + 1) load_cons_at<N>(Uin + plane_off(p + 3), own_xy, pre);
    if (out0 && p + 2 <= Z0 + N) load_cons_at<N>(Uin + plane_off(p + 2), o0_xy, pre);
    if (out1 && p + 2 <= Z0 + N) load_cons_at<N>(Uin + plane_off(p + 2), o1_xy, pre1);
    __syncthreads();

    // ---- B: normal predictor of plane k1; z 1-D flux at face k1
    double xl[5], xh[5], yl[5], yh[5], zl[5], zh[5];
    if (pos) {
      double sl[3][5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const double c = Wz1[v];
        sl[0][v] = van_leer_sf(c - sm.sW[v][rq - 1], sm.sW[v][rq + 1] - c);
        sl[1][v] = van_leer_sf(c - sm.sW[v][rq - R], sm.sW[v][rq + R] - c);
        sl[2][v] = van_leer_sf(c - Wz0[v], Wz2[v] - c);
      }
      const double inv = rcp_nr(Wz1[0]);
      double fs[6][5];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        if constexpr (TRACE) {
          trace_faces(d, Wz1, sl[d], d == 0 ? lx : d == 1 ? ly : lz, gamma, inv, fs[2 * d], fs[2 * d + 1]);
        } else {
          const double lam = d == 0 ? lx : d == 1 ? ly : lz;
          const double un = Wz1[1 + d];
          double A[5];
          A[0] = un * sl[d][0] + Wz1[0] * sl[d][1 + d];
          A[1] = un * sl[d][1];
          A[2] = un * sl[d][2];
          A[3] = un * sl[d][3];
          A[1 + d] += sl[d][4] * inv;
          A[4] = (gamma * Wz1[4]) * sl[d][1 + d] + un * sl[d][4];
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            const double wt = Wz1[v] - 0.5 * lam * A[v];
            fs[2 * d][v] = wt - 0.5 * sl[d][v];
            fs[2 * d + 1][v] = wt + 0.5 * sl[d][v];
          }
        }
      }
      bool ok = true;
#pragma unroll
      for (int s = 0; s < 6; ++s) ok = ok && fs[s][0] > 0.0 && fs[s][4] > 0.0;
      if (!ok && inner && k1 >= Z0 && k1 < Z0 + N) ++n_fb;
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        xl[v] = ok ? fs[0][v] : Wz1[v];
        xh[v] = ok ? fs[1][v] : Wz1[v];
        yl[v] = ok ? fs[2][v] : Wz1[v];
        yh[v] = ok ? fs[3][v] : Wz1[v];
        zl[v] = ok ? fs[4][v] : Wz1[v];
        zh[v] = ok ? fs[5][v] : Wz1[v];
        sm.sXh[par1][v][q] = xh[v];
        sm.sYh[par1][v][q] = yh[v];
      }
      if (p >= Z0 - 1) {                               // face k1 in [Z0, Z0 + N]
        double F[5];
        hllc<2>(zhi, zl, gamma, gm1inv, F);
        if (mid) {
#pragma unroll
          for (int v = 0; v < 5; ++v) sm.sFxy[v][q] = F[v] - f1z[v];   // the z 1-D flux difference over plane p
        }
#pragma unroll
        for (int v = 0; v < 5; ++v) f1z[v] = F[v];
      }
    }
    __syncthreads();

    // ---- C: x / y 1-D fluxes of plane k1; F_{x|z}, F_{y|z} of plane p
    if (pos) {
      double F[5], L[5], Rt[5];
      if (i >= 0) {
#pragma unroll
        for (int v = 0; v < 5; ++v) L[v] = sm.sXh[par1][v][q - 1];
        hllc<0>(L, xl, gamma, gm1inv, F);
#pragma unroll
        for (int v = 0; v < 5; ++v) sm.sF1x[v][q] = F[v];
      }
      if (j >= 0) {
#pragma unroll
        for (int v = 0; v < 5; ++v) L[v] = sm.sYh[par1][v][q - P];
        hllc<1>(L, yl, gamma, gm1inv, F);
#pragma unroll
        for (int v = 0; v < 5; ++v) sm.sF1y[v][q] = F[v];
      }
      if (mid) {
        double w[5], d[5];
        if (i >= 0) {                                  // x face i, rows -1..T
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            w[v] = sm.sXh[par0][v][q - 1];
            d[v] = sm.sFxy[v][q - 1];
          }
          const bool b0 = corrected_state(w, lz * (1.0 / 3.0), d, gamma, gm1inv, L);
#pragma unroll
          for (int v = 0; v < 5; ++v) d[v] = sm.sFxy[v][q];
          const bool b1 = corrected_state(xlo, lz * (1.0 / 3.0), d, gamma, gm1inv, Rt);
          if (cfx && cry) n_fb += (int)b0 + (int)b1;
          hllc<0>(L, Rt, gamma, gm1inv, F);
#pragma unroll
          for (int v = 0; v < 5; ++v) sm.sFxz[v][q] = F[v];
        }
        if (j >= 0) {                                  // y face j, columns -1..T
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            w[v] = sm.sYh[par0][v][q - P];
            d[v] = sm.sFxy[v][q - P];
          }
          const bool b0 = corrected_state(w, lz * (1.0 / 3.0), d, gamma, gm1inv, L);
#pragma unroll
          for (int v = 0; v < 5; ++v) d[v] = sm.sFxy[v][q];
          const bool b1 = corrected_state(ylo, lz * (1.0 / 3.0), d, gamma, gm1inv, Rt);
          if (cfy && crx) n_fb += (int)b0 + (int)b1;
          hllc<1>(L, Rt, gamma, gm1inv, F);
#pragma unroll
          for (int v = 0; v < 5; ++v) sm.sFyz[v][q] = F[v];
        }
      }
    }
    __syncthreads();

    // ---- D: F_{x|y}, F_{y|x} of plane k1; F_{z|x}, F_{z|y} at face k1
    double nd1x[5], nd1y[5];
    if (pos) {
      const bool hx = i >= 0 && i < T, hy = j >= 0 && j < T;   // own transverse 1-D flux differences exist
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        nd1x[v] = hx ? sm.sF1x[v][q + 1] - sm.sF1x[v][q] : 0.0;
        nd1y[v] = hy ? sm.sF1y[v][q + P] - sm.sF1y[v][q] : 0.0;
      }
      double F[5], L[5], Rt[5], w[5], d[5];
      if (i >= 0 && hy) {                              // x face i of an inner row
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          w[v] = sm.sXh[par1][v][q - 1];
          d[v] = sm.sF1y[v][q - 1 + P] - sm.sF1y[v][q - 1];
        }
        const bool b0 = corrected_state(w, ly * (1.0 / 3.0), d, gamma, gm1inv, L);
        const bool b1 = corrected_state(xl, ly * (1.0 / 3.0), nd1y, gamma, gm1inv, Rt);
        if (cfx) n_fb += (int)b0 + (int)b1;
        hllc<0>(L, Rt, gamma, gm1inv, F);
#pragma unroll
        for (int v = 0; v < 5; ++v) sm.sFxy[v][q] = F[v];
      }
      if (j >= 0 && hx) {                              // y face j of an inner column
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          w[v] = sm.sYh[par1][v][q - P];
          d[v] = sm.sF1x[v][q - P + 1] - sm.sF1x[v][q - P];
        }
        const bool b0 = corrected_state(w, lx * (1.0 / 3.0), d, gamma, gm1inv, L);
        const bool b1 = corrected_state(yl, lx * (1.0 / 3.0), nd1x, gamma, gm1inv, Rt);
        if (cfy) n_fb += (int)b0 + (int)b1;
        hllc<1>(L, Rt, gamma, gm1inv, F);
#pragma unroll
        for (int v = 0; v < 5; ++v) sm.sFyx[v][q] = F[v];
      }
      if (p >= Z0 - 1) {                               // z face k1
        if (hx) {                                      // F_{z|x}: inner columns, rows -1..T
          const bool b0 = corrected_state(zhi, lx * (1.0 / 3.0), d1x, gamma, gm1inv, L);
          const bool b1 = corrected_state(zl, lx * (1.0 / 3.0), nd1x, gamma, gm1inv, Rt);
          if (cry) n_fb += (int)b0 + (int)b1;
          hllc<2>(L, Rt, gamma, gm1inv, F);
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            if (mid) sm.sDzx[v][q] = F[v] - fzx[v];
            fzx[v] = F[v];
          }
        }
        if (hy) {                                      // F_{z|y}: inner rows, columns -1..T
          const bool b0 = corrected_state(zhi, ly * (1.0 / 3.0), d1y, gamma, gm1inv, L);
          const bool b1 = corrected_state(zl, ly * (1.0 / 3.0), nd1y, gamma, gm1inv, Rt);
          if (crx) n_fb += (int)b0 + (int)b1;
          hllc<2>(L, Rt, gamma, gm1inv, F);
#pragma unroll
          for (int v = 0; v < 5; ++v) {
            if (mid) sm.sDzy[v][q] = F[v] - fzy[v];
            fzy[v] = F[v];
          }
        }
      }
    }
    __syncthreads();

    // ---- E: final fluxes (x / y of plane p, z at face k1); the old state of p
    double nffz[5], uold[5];
    if (pos) {
      double F[5], L[5], Rt[5], w[5], d[5];
      const bool hx = i >= 0 && i < T, hy = j >= 0 && j < T;
      if (mid && i >= 0 && hy) {                       // x face i of an inner row
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          w[v] = sm.sXh[par0][v][q - 1];
          d[v] = ly * (sm.sFyz[v][q - 1 + P] - sm.sFyz[v][q - 1]) + lz * sm.sDzy[v][q - 1];
        }
        const bool b0 = corrected_state(w, 0.5, d, gamma, gm1inv, L);
#pragma unroll
        for (int v = 0; v < 5; ++v) d[v] = ly * (sm.sFyz[v][q + P] - sm.sFyz[v][q]) + lz * sm.sDzy[v][q];
        const bool b1 = corrected_state(xlo, 0.5, d, gamma, gm1inv, Rt);
        if (cfx) n_fb += (int)b0 + (int)b1;
        hllc<0>(L, Rt, gamma, gm1inv, F);
#pragma unroll
        for (int v = 0; v < 5; ++v) sm.sF1x[v][q] = F[v];
      }
      if (mid && j >= 0 && hx) {                       // y face j of an inner column
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          w[v] = sm.sYh[par0][v][q - P];
          d[v] = lx * (sm.sFxz[v][q - P + 1] - sm.sFxz[v][q - P]) + lz * sm.sDzx[v][q - P];
        }
        const bool b0 = corrected_state(w, 0.5, d, gamma, gm1inv, L);
#pragma unroll
        for (int v = 0; v < 5; ++v) d[v] = lx * (sm.sFxz[v][q + 1] - sm.sFxz[v][q]) + lz * sm.sDzx[v][q];
        const bool b1 = corrected_state(ylo, 0.5, d, gamma, gm1inv, Rt);
        if (cfy) n_fb += (int)b0 + (int)b1;
        hllc<1>(L, Rt, gamma, gm1inv, F);
#pragma unroll
        for (int v = 0; v < 5; ++v) sm.sF1y[v][q] = F[v];
      }
      if (inner) {                                     // z face k1: the correction of plane k1's side
#pragma unroll
        for (int v = 0; v < 5; ++v)
          d[v] = lx * (sm.sFxy[v][q + 1] - sm.sFxy[v][q]) + ly * (sm.sFyx[v][q + P] - sm.sFyx[v][q]);
        if (p >= Z0 - 1) {
          const bool b0 = corrected_state(zhi, 0.5, dzl, gamma, gm1inv, L);
          const bool b1 = corrected_state(zl, 0.5, d, gamma, gm1inv, Rt);
          n_fb += (int)b0 + (int)b1;
          hllc<2>(L, Rt, gamma, gm1inv, nffz);
        }
#pragma unroll
        for (int v = 0; v < 5; ++v) dzl[v] = d[v];
        if (mid) load_cons_at<N, false, true>(Uin + plane_off(p), own_xy, uold);
      }
    }
    __syncthreads();

    // ---- F: update of plane p
    if (inner && mid) {
      double un[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const double div = (lx * (sm.sF1x[v][q + 1] - sm.sF1x[v][q]) + ly * (sm.sF1y[v][q + P] - sm.sF1y[v][q])) +
                           lz * (nffz[v] - ffz[v]);
        un[v] = uold[v] - div;
      }
      const long oo = plane_off(p);
#pragma unroll
      for (int v = 0; v < 5; ++v)
        __builtin_nontemporal_store(un[v], (double*)((char*)(a.Uout + oo + v * VS) + own_xy));
      bool good = un[0] > 0.0 && un[4] > 0.0;
#pragma unroll
      for (int v = 0; v < 5; ++v) good = good && isfinite(un[v]);
      if (!good) ++n_bad;
      const double s = signal_speed_dir(un, g);
      smax = (s > smax || !(s == s)) ? s : smax;
    }
    // the plane below for the next iteration
    if (pos) {
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        Wz0[v] = Wz1[v];
        Wz1[v] = Wz2[v];
        xlo[v] = xl[v];
        ylo[v] = yl[v];
        zhi[v] = zh[v];
        d1x[v] = nd1x[v];
        d1y[v] = nd1y[v];
        if (inner && p >= Z0 - 1) ffz[v] = nffz[v];
      }
    }
  }
  if (n_floor) atomicAdd(&sm.sCnt[0], n_floor);
  if (n_fb) atomicAdd(&sm.sCnt[1], n_fb);
  if (n_bad) atomicAdd(&sm.sCnt[2], n_bad);
  wg_max_to(smax, sm.sRed, &ws->sig[(slot + 1) % 3]);
  if (tid == 0) {
    for (int c = 0; c < 3; ++c)
      if (sm.sCnt[c]) atomicAdd(&ws->cnt[c], (unsigned long long)sm.sCnt[c]);
  }
}

// ---------------------------------------------------------------------------
// Block-structured AMR (the Grid unit's refinement): an octree of blocks,
// level 0 the root grid, level l+1 the eight children (half the cell size)
// of each refined block of level l.  Kernels: the leaves' guard views
// (copies of same-level cells, prolongation from the level above), the
// fluxes at fine-coarse faces that refluxing uses (formed before the leaf
// steps), the leaf steps of every level in one launch (the fused tile step
// over the views; a leaf that refluxing leaves alone also restricts its new
// state into its parent), refluxing, the restriction of the parent octants
// over refined or refluxed children, the refinement indicators and the
// regrid transfer.

template <int N>
struct AmrStep {
  static constexpr long NF = 6L * 5 * N * N;      // boundary fluxes per block: [face 2d+side][v][a1][a0]
};

// Offset of the cell at global index (I, J, K) of one level (each may lie
// up to two cells outside the domain; boundary conditions applied), its
// block found through the level's lookup (every position read here holds a
// block: the host checks the nesting; a missing one would read block 0).
template <int N>
__device__ __forceinline__ long level_offset(const GridGeom& g, const int* __restrict__ lookup, int I, int J,
                                             int K) {
  I = map_axis(I, g.nb[0] * N, g.bc[0]);
  J = map_axis(J, g.nb[1] * N, g.bc[1]);
  K = map_axis(K, g.nb[2] * N, g.bc[2]);
  const int b = lookup[(I / N) + g.nb[0] * ((J / N) + g.nb[1] * (K / N))];
  return Layout<N>::at(b < 0 ? 0 : b, I % N, J % N, K % N);
}

// Conserved state prolonged from level p to the level-(p+1) cell at global
// index (I, J, K) (inside the domain): U_c + sum_d S_d * (+-1/4), S_d the van
// Leer slope of the conserved variable over level-p cells (level-p map and
// lookup), keeping U_c if the result has rho <= 0 or p <= 0.
template <int N>
__device__ __forceinline__ void prolong_cell(const GridGeom& gp, const int* __restrict__ lookup,
                                             const double* __restrict__ Up, int I, int J, int K, double (&val)[5]) {
  const int Ic = I / 2, Jc = J / 2, Kc = K / 2;
  double uc[5];
  load_cons<N>(Up, level_offset<N>(gp, lookup, Ic, Jc, Kc), uc);
#pragma unroll
  for (int v = 0; v < 5; ++v) val[v] = uc[v];
  const int off[3] = {(I & 1) * 2 - 1, (J & 1) * 2 - 1, (K & 1) * 2 - 1};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double um[5], up[5];
    load_cons<N>(Up, level_offset<N>(gp, lookup, Ic - (d == 0), Jc - (d == 1), Kc - (d == 2)), um);
    load_cons<N>(Up, level_offset<N>(gp, lookup, Ic + (d == 0), Jc + (d == 1), Kc + (d == 2)), up);
#pragma unroll
    for (int v = 0; v < 5; ++v) val[v] += van_leer_sf(uc[v] - um[v], up[v] - uc[v]) * (0.25 * off[d]);
  }
  const double rho = val[0];
  const double kin = 0.5 * ((val[1] * val[1] + val[2] * val[2]) + val[3] * val[3]) / (rho > 0.0 ? rho : 1.0);
  const double p = (gp.gamma - 1.0) * (val[4] - kin);
  if (!(rho > 0.0 && p > 0.0)) {
#pragma unroll
    for (int v = 0; v < 5; ++v) val[v] = uc[v];
  }
}

// Views of the listed blocks of level l >= 1 (two guard layers): a position
// (mapped at level l) inside a block of level l copies its cell; otherwise it
// is prolonged from level l-1.
template <int N>
__global__ __launch_bounds__(256) void amr_fill_level_kernel(GridGeom g, GridGeom gp,
                                                             const int* __restrict__ lookup,
                                                             const int* __restrict__ lookup_p,
                                                             const int4* __restrict__ pos,
                                                             const double* __restrict__ U,
                                                             const double* __restrict__ Up,
                                                             double* __restrict__ G,
                                                             const int* __restrict__ list) {
  constexpr int P = Guarded<N, VG>::P;
  const int f = list[blockIdx.x];
  const int4 q = pos[f];
  const int X0 = q.x * N, Y0 = q.y * N, Z0 = q.z * N;
  const int NX = g.nb[0] * N, NY = g.nb[1] * N, NZ = g.nb[2] * N;
  double* out = G + (long)f * Guarded<N, VG>::BS;
  for (int t = threadIdx.x; t < P * P * P; t += blockDim.x) {
    const int I = map_axis(X0 + t % P - VG, NX, g.bc[0]);
    const int J = map_axis(Y0 + (t / P) % P - VG, NY, g.bc[1]);
    const int K = map_axis(Z0 + t / (P * P) - VG, NZ, g.bc[2]);
    const int b = lookup[(I / N) + g.nb[0] * ((J / N) + g.nb[1] * (K / N))];
    double val[5];
    if (b >= 0)
      load_cons<N>(U, Layout<N>::at(b, I % N, J % N, K % N), val);
    else
      prolong_cell<N>(gp, lookup_p, Up, I, J, K, val);
#pragma unroll
    for (int v = 0; v < 5; ++v) out[v * Guarded<N, VG>::VS + t] = val[v];
  }
}

// Plane halos (PlaneHalo<N>) of the listed blocks of level l, slot after
// slot, so each workgroup writes whole rows: a position (mapped at level l)
// inside a block of level l copies its cell, otherwise (level l >= 1) it is
// prolonged from level l-1.  Every level-0 position has a block.  The ring
// planes are always written, the whole planes -2, -1 only when bit 0 of
// zneed[block] is set and N, N+1 only with bit 1: a block inside a column
// of z-stacked blocks has neither read (the column's pencil reads the
// next block's own cells there).
template <int N>
__global__ __launch_bounds__(256) void amr_fill_halo_kernel(GridGeom g, GridGeom gp, const int* __restrict__ lookup,
                                                            const int* __restrict__ lookup_p,
                                                            const int4* __restrict__ pos,
                                                            const double* __restrict__ U,
                                                            const double* __restrict__ Up,
                                                            double* __restrict__ H, const int* __restrict__ list,
                                                            const int* __restrict__ zneed) {
  using PH = PlaneHalo<N>;
  constexpr int NRP = N * PH::RP, FP2 = 2 * PH::FP;
  const int f = list[blockIdx.x];
  const int4 q = pos[f];
  const int need = zneed[f];
  const int lowp = (need & 1) ? FP2 : 0, count = NRP + lowp + ((need & 2) ? FP2 : 0);
  const int X0 = q.x * N, Y0 = q.y * N, Z0 = q.z * N;
  const int NX = g.nb[0] * N, NY = g.nb[1] * N, NZ = g.nb[2] * N;
  double* out = H + (long)f * PH::BS;
  for (int u = threadIdx.x; u < count; u += blockDim.x) {
    const int t = u < NRP + lowp ? u : u + (FP2 - lowp);  // slot: skip the low planes when not written
    int i, j, k;
    PH::cell(t, i, j, k);
    const int I = map_axis(X0 + i, NX, g.bc[0]);
    const int J = map_axis(Y0 + j, NY, g.bc[1]);
    const int K = map_axis(Z0 + k, NZ, g.bc[2]);
    const int b = lookup[(I / N) + g.nb[0] * ((J / N) + g.nb[1] * (K / N))];
    double val[5];
    if (b >= 0)
      load_cons<N>(U, Layout<N>::at(b, I % N, J % N, K % N), val);
    else
      prolong_cell<N>(gp, lookup_p, Up, I, J, K, val);
#pragma unroll
    for (int v = 0; v < 5; ++v) out[v * PH::VS + t] = val[v];
  }
}

// Start of an AMR step: dt = cfl / ws->sig[slot] (cfl > 0) or dt_host,
// recorded in ws->dt_last for every later kernel of the step; the signal
// slot of the step after next is cleared.
__global__ void amr_begin_kernel(WorkHeader* ws, double dt_host, double cfl, int slot) {
  ws->dt_last = cfl > 0.0 ? cfl / __longlong_as_double(ws->sig[slot]) : dt_host;
  ws->sig[(slot + 2) % 3] = 0ull;
}

// Leaf steps of every level in one launch: workgroup w steps column tile
// w - first of the segment holding w (segments in order of `first`), the
// fused tile step over that level's leaf views (the whole z extent of a
// column of z-stacked blocks, tile_step's gv_cols).  Segments with the
// longest columns come first, so the longest workgroups start first.  The
// leaf steps are independent of each other (each reads its own views and
// cells and writes its own cells and parent octant), so one launch holds
// them all.
template <int N, int T>
__global__ __launch_bounds__(Tile<T>::NT, 2) void amr_tile_kernel(AmrSegs S, int slot, WorkHeader* ws) {
  __shared__ Smem<T> sm;
  __shared__ double psum[5 * Tile<T>::NI / 4];  // fused restriction: even-plane 2 x 2 sums
  const long w = blockIdx.x;
  if (w >= S.tiles) return;
  int q = 0;
  while (q + 1 < S.n && w >= S.s[q + 1].first) ++q;
  const AmrSeg& a = S.s[q];
  tile_step<N, T, false, true>(a.g, a.G, a.U, ws, 0.0, 0.0, slot, w - a.first, N, sm,
                               StageArgs{nullptr, 0.0, 0.0, 0, 1}, a.cols, a.emit != 0, a.po, psum);
}

// Face state of cell (i, j, k) of a block on its low (hi = 0) or high
// (hi = 1) d face, formed as the leaf step forms it: primitives of the cell
// and its six neighbours, van Leer slopes, predictor with fallback.  Cells
// of the block come from its state Ub (compact, not yet stepped), the
// others from its leaf view V (plane halo for N = 8, 16, whole view for 32).
template <int N>
__device__ __forceinline__ void amr_face_state(const double* V, const double* Ub, int i, int j, int k, int d,
                                               int hi, const GridGeom& g, double lamx, double lamy, double lamz,
                                               double (&out)[5]) {
  constexpr bool HALO = N != 32;
  constexpr int P = Guarded<N, VG>::P;
  constexpr long VSv = HALO ? PlaneHalo<N>::VS : Guarded<N, VG>::VS;
  auto w_at = [&](int a, int b, int c, double (&w)[5]) {
    const bool in = a >= 0 && a < N && b >= 0 && b < N && c >= 0 && c < N;
    const double* src;
    long vs;
    if (in) {
      src = Ub + ((long)c * N + b) * N + a;
      vs = Layout<N>::VS;
    } else {
      long o;
      if constexpr (HALO) o = PlaneHalo<N>::slot(a, b, c);
      else o = ((long)(c + VG) * P + (b + VG)) * P + (a + VG);
      src = V + o;
      vs = VSv;
    }
    double u[5], inv;
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = src[v * vs];
    prim(u, g.gamma, g.small_p, w, inv);
  };
  double wc[5], wm[5], wp[5], sx[5], sy[5], sz[5], wt[5], h;
  w_at(i, j, k, wc);
  w_at(i - 1, j, k, wm);
  w_at(i + 1, j, k, wp);
#pragma unroll
  for (int v = 0; v < 5; ++v) sx[v] = van_leer_sf(wc[v] - wm[v], wp[v] - wc[v]);
  w_at(i, j - 1, k, wm);
  w_at(i, j + 1, k, wp);
#pragma unroll
  for (int v = 0; v < 5; ++v) sy[v] = van_leer_sf(wc[v] - wm[v], wp[v] - wc[v]);
  w_at(i, j, k - 1, wm);
  w_at(i, j, k + 1, wp);
#pragma unroll
  for (int v = 0; v < 5; ++v) sz[v] = van_leer_sf(wc[v] - wm[v], wp[v] - wc[v]);
  predict(wc, rcp_nr(wc[0]), sx, sy, sz, g.gamma, lamx, lamy, lamz, wt, h);
  const double hs = hi ? h : -h;
#pragma unroll
  for (int v = 0; v < 5; ++v) out[v] = fma(hs, d == 0 ? sx[v] : (d == 1 ? sy[v] : sz[v]), wt[v]);
}

// Fluxes on the faces that refluxing uses, computed before the leaf steps
// from the old states and the leaf views with the leaf step's arithmetic:
// workgroup 5e + part of reflux
// entry e = (coarse leaf b, d, side, refined r): part 0 is b's face 2d+side
// (level 0), parts 1..4 the faces 2d+(1-side) of r's four children on the
// side toward b (level 1).  Output flux[block][face][v][a1][a0], a0 / a1 the
// faster / slower transverse index.
template <int N>
__global__ __launch_bounds__(256) void amr_face_flux_kernel(GridGeom g0, GridGeom g1,
                                                            const int4* __restrict__ entries,
                                                            const int* __restrict__ child_base,
                                                            const double* __restrict__ G0,
                                                            const double* __restrict__ G1,
                                                            const double* __restrict__ U0,
                                                            const double* __restrict__ U1, double* flux0,
                                                            double* flux1, const WorkHeader* ws) {
  using A = AmrStep<N>;
  const double dt = ws->dt_last;
  const int part = blockIdx.x % 5;
  const int4 e = entries[blockIdx.x / 5];
  const int d = e.y;
  const int t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;   // faster, slower transverse axes
  int blk, fs;
  if (part == 0) {
    blk = e.x;
    fs = e.z;
  } else {
    fs = e.z ? 0 : 1;
    int co[3];
    co[d] = fs;
    co[t0] = (part - 1) & 1;
    co[t1] = (part - 1) >> 1;
    blk = child_base[e.w] + co[0] + 2 * co[1] + 4 * co[2];
  }
  const GridGeom& g = part ? g1 : g0;
  const double* V = (part ? G1 : G0) + (long)blk * amr_view_doubles(N);
  const double* Ub = (part ? U1 : U0) + (long)blk * Layout<N>::BS;
  double* out = (part ? flux1 : flux0) + (long)blk * A::NF + (long)(2 * d + fs) * 5 * N * N;
  const double lamx = dt * g.inv_dx[0], lamy = dt * g.inv_dx[1], lamz = dt * g.inv_dx[2];
  const double gm1inv = 1.0 / (g.gamma - 1.0);
  for (int t = threadIdx.x; t < N * N; t += blockDim.x) {
    const int a1 = t / N, a0 = t % N;
    int c[3];
    c[d] = fs ? N : 0;     // the cell on the face's high side
    c[t0] = a0;
    c[t1] = a1;
    double L[5], R[5], F[5];
    amr_face_state<N>(V, Ub, c[0] - (d == 0), c[1] - (d == 1), c[2] - (d == 2), d, 1, g, lamx, lamy, lamz, L);
    amr_face_state<N>(V, Ub, c[0], c[1], c[2], d, 0, g, lamx, lamy, lamz, R);
    hllc_dir(d, L, R, g.gamma, gm1inv, F);
#pragma unroll
    for (int v = 0; v < 5; ++v) out[(long)v * N * N + t] = F[v];
  }
}

// Refluxing: entry e = (coarse leaf b, direction d, side, refined neighbour
// r).  The root cell of b next to the face replaces its face flux by the mean
// of the four fine fluxes over it: U += lam_d (F_c - <F_f>) on the high face
// (side 1), U -= lam_d (F_c - <F_f>) on the low face.  Entries of one coarse
// block are contiguous (first[w] .. first[w+1]) and one workgroup applies
// them in order: faces of one block share their edge and corner cells.
// Then it reduces the block's final signal speed into ws->sig[(slot+1)%3]
// (the leaf step left these blocks out).
template <int N>
__global__ __launch_bounds__(256) void amr_reflux_kernel(GridGeom g0, const int4* __restrict__ entries,
                                                         const int* __restrict__ first,
                                                         const double* __restrict__ flux0,
                                                         const double* __restrict__ flux1,
                                                         const int* __restrict__ child_base, double* Ur,
                                                         WorkHeader* ws, int slot) {
  using A = AmrStep<N>;
  constexpr int H = N / 2;
  __shared__ unsigned long long sRed[4];
  const double dt = ws->dt_last;
  const int e_end = first[blockIdx.x + 1];
  for (int q = first[blockIdx.x]; q < e_end; ++q) {
    const int4 e = entries[q];
    const int b = e.x, d = e.y, side = e.z, r = e.w;
    const double lam = dt * g0.inv_dx[d];
    const int t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;   // faster, slower transverse axes
    const double* fc = flux0 + (long)b * A::NF + (long)(2 * d + side) * 5 * N * N;
    const int fside = side ? 0 : 1;                        // the refined block's face toward b
    for (int t = threadIdx.x; t < N * N; t += blockDim.x) {
      const int a1 = t / N, a0 = t % N;                    // slower, faster transverse index
      int co[3];
      co[d] = fside;
      co[t0] = a0 / H;
      co[t1] = a1 / H;
      const int fb = child_base[r] + co[0] + 2 * co[1] + 4 * co[2];
      const double* ff = flux1 + (long)fb * A::NF + (long)(2 * d + fside) * 5 * N * N;
      const int f1 = 2 * (a1 % H), f0 = 2 * (a0 % H);
      int c3[3];
      c3[d] = side ? N - 1 : 0;
      c3[t0] = a0;
      c3[t1] = a1;
      const long off = Layout<N>::at(b, c3[0], c3[1], c3[2]);
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const double* fv = ff + (long)v * N * N;
        const double mean =
            0.25 * ((fv[f1 * N + f0] + fv[f1 * N + f0 + 1]) + (fv[(f1 + 1) * N + f0] + fv[(f1 + 1) * N + f0 + 1]));
        const double corr = lam * (fc[(long)v * N * N + t] - mean);
        Ur[off + v * Layout<N>::VS] += side ? corr : -corr;
      }
    }
    __syncthreads();
  }
  const int b = entries[first[blockIdx.x]].x;
  double smax = 0.0;
  for (int t = threadIdx.x; t < N * N * N; t += blockDim.x) {
    double u[5];
    load_cons<N>(Ur, Layout<N>::at(b, t % N, (t / N) % N, t / (N * N)), u);
    const double sp = signal_speed(u, g0);
    smax = (sp > smax || !(sp == sp)) ? sp : smax;
  }
  wg_max_to(smax, sRed, &ws->sig[(slot + 1) % 3]);
}

// Refinement indicator of root block b (one workgroup each): the largest,
// over its cells, of Loehner's squared second-derivative ratio of density
// and of pressure, E^2 = sum_d num_d^2 / sum_d den_d^2 with
// num_d = (fR - f0) - (f0 - fL), den_d = (|fR - f0| + |f0 - fL|) +
// eps ((|fR| + 2|f0|) + |fL|) over the cell and its neighbours along d (root
// map); 0 where the denominator is 0.  Every operation is rounded as
// written (no fused multiply-adds), so refinement decisions taken from it
// are reproducible bit for bit.
__device__ __forceinline__ double amr_pressure(const double (&u)[5], double gamma) {
#pragma clang fp contract(off)
  const double kin = 0.5 * ((u[1] * u[1] + u[2] * u[2]) + u[3] * u[3]) / u[0];
  return (gamma - 1.0) * (u[4] - kin);
}

template <int N>
__global__ __launch_bounds__(256) void amr_indicator_kernel(GridGeom g0, const double* __restrict__ Ur, double eps,
                                                            double* __restrict__ out) {
#pragma clang fp contract(off)
  __shared__ double sRed[4];
  const int b = blockIdx.x;
  const int bx = b % g0.nb[0], by = (b / g0.nb[0]) % g0.nb[1], bz = b / (g0.nb[0] * g0.nb[1]);
  double emax = 0.0;
  for (int t = threadIdx.x; t < N * N * N; t += blockDim.x) {
    const int I = bx * N + t % N, J = by * N + (t / N) % N, K = bz * N + t / (N * N);
    double u[5];
    load_cons<N>(Ur, cell_offset<N>(g0, I, J, K), u);
    const double r0 = u[0], p0 = amr_pressure(u, g0.gamma);
    double nr = 0.0, dr = 0.0, np_ = 0.0, dp = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double um[5], up[5];
      load_cons<N>(Ur, cell_offset<N>(g0, I - (d == 0), J - (d == 1), K - (d == 2)), um);
      load_cons<N>(Ur, cell_offset<N>(g0, I + (d == 0), J + (d == 1), K + (d == 2)), up);
      const double rL = um[0], rR = up[0], pL = amr_pressure(um, g0.gamma), pR = amr_pressure(up, g0.gamma);
      const double an = (rR - r0) - (r0 - rL);
      const double ad = (fabs(rR - r0) + fabs(r0 - rL)) + eps * ((fabs(rR) + 2.0 * fabs(r0)) + fabs(rL));
      const double bn = (pR - p0) - (p0 - pL);
      const double bd = (fabs(pR - p0) + fabs(p0 - pL)) + eps * ((fabs(pR) + 2.0 * fabs(p0)) + fabs(pL));
      if (d == 0) {
        nr = an * an;
        dr = ad * ad;
        np_ = bn * bn;
        dp = bd * bd;
      } else {
        nr = nr + an * an;
        dr = dr + ad * ad;
        np_ = np_ + bn * bn;
        dp = dp + bd * bd;
      }
    }
    const double er = dr > 0.0 ? nr / dr : 0.0;
    const double ep = dp > 0.0 ? np_ / dp : 0.0;
    const double e = fmax(er, ep);
    emax = fmax(emax, e);
  }
  // workgroup maximum (non-negative values; wavefront shuffles then LDS)
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) emax = fmax(emax, __shfl_xor(emax, o, 64));
  if ((threadIdx.x & 63) == 0) sRed[threadIdx.x >> 6] = emax;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = sRed[0];
    for (int w = 1; w < (int)(blockDim.x + 63) / 64; ++w) m = fmax(m, sRed[w]);
    out[b] = m;
  }
}

// Refinement indicator of the listed leaves of one level (one workgroup
// each), into E2[block]: the per-cell quantity of amr_indicator_kernel with
// neighbours read at the leaf's own level through the level's lookup; a
// neighbour position holding no block of that level (a coarser region)
// takes the cell's own state.  Rounded as written, like that kernel.
template <int N>
__global__ __launch_bounds__(256) void amr_leaf_indicator_kernel(GridGeom g, const int* __restrict__ lookup,
                                                                 const double* __restrict__ U,
                                                                 const int* __restrict__ leaves,
                                                                 const int4* __restrict__ pos, double eps,
                                                                 double* __restrict__ E2) {
#pragma clang fp contract(off)
  __shared__ double sRed[4];
  const int b = leaves[blockIdx.x];
  const int4 q = pos[b];
  const int NX = g.nb[0] * N, NY = g.nb[1] * N, NZ = g.nb[2] * N;
  auto load_or_self = [&](int I, int J, int K, const double (&own)[5], double (&u)[5]) {
    I = map_axis(I, NX, g.bc[0]);
    J = map_axis(J, NY, g.bc[1]);
    K = map_axis(K, NZ, g.bc[2]);
    const int nb = lookup[(I / N) + g.nb[0] * ((J / N) + g.nb[1] * (K / N))];
    if (nb >= 0) {
      load_cons<N>(U, Layout<N>::at(nb, I % N, J % N, K % N), u);
    } else {
#pragma unroll
      for (int v = 0; v < 5; ++v) u[v] = own[v];
    }
  };
  double emax = 0.0;
  for (int t = threadIdx.x; t < N * N * N; t += blockDim.x) {
    const int I = q.x * N + t % N, J = q.y * N + (t / N) % N, K = q.z * N + t / (N * N);
    double u[5];
    load_cons<N>(U, Layout<N>::at(b, t % N, (t / N) % N, t / (N * N)), u);
    const double r0 = u[0], p0 = amr_pressure(u, g.gamma);
    double nr = 0.0, dr = 0.0, np_ = 0.0, dp = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      double um[5], up[5];
      load_or_self(I - (d == 0), J - (d == 1), K - (d == 2), u, um);
      load_or_self(I + (d == 0), J + (d == 1), K + (d == 2), u, up);
      const double rL = um[0], rR = up[0], pL = amr_pressure(um, g.gamma), pR = amr_pressure(up, g.gamma);
      const double an = (rR - r0) - (r0 - rL);
      const double ad = (fabs(rR - r0) + fabs(r0 - rL)) + eps * ((fabs(rR) + 2.0 * fabs(r0)) + fabs(rL));
      const double bn = (pR - p0) - (p0 - pL);
      const double bd = (fabs(pR - p0) + fabs(p0 - pL)) + eps * ((fabs(pR) + 2.0 * fabs(p0)) + fabs(pL));
      if (d == 0) {
        nr = an * an;
        dr = ad * ad;
        np_ = bn * bn;
        dp = bd * bd;
      } else {
        nr = nr + an * an;
        dr = dr + ad * ad;
        np_ = np_ + bn * bn;
        dp = dp + bd * bd;
      }
    }
    const double er = dr > 0.0 ? nr / dr : 0.0;
    const double ep = dp > 0.0 ? np_ / dp : 0.0;
    emax = fmax(emax, fmax(er, ep));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) emax = fmax(emax, __shfl_xor(emax, o, 64));
  if ((threadIdx.x & 63) == 0) sRed[threadIdx.x >> 6] = emax;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = sRed[0];
    for (int w = 1; w < (int)(blockDim.x + 63) / 64; ++w) m = fmax(m, sRed[w]);
    E2[b] = m;
  }
}

// Regridding, level l >= 1 of the new mesh: block f copies the block at the
// same position of the old mesh's level l (old_lookup, when that level
// exists), else is prolonged cell by cell from the new mesh's level l-1
// (already final).
template <int N>
__global__ __launch_bounds__(256) void amr_transfer_level_kernel(GridGeom g, GridGeom gp,
                                                                 const int* __restrict__ old_lookup,
                                                                 const double* __restrict__ U_old,
                                                                 const int* __restrict__ lookup_p,
                                                                 const double* __restrict__ Up,
                                                                 const int4* __restrict__ pos,
                                                                 double* __restrict__ U) {
  const int f = blockIdx.x;
  const int4 q = pos[f];
  double* out = U + (long)f * Layout<N>::BS;
  const int ob = old_lookup ? old_lookup[q.x + g.nb[0] * (q.y + g.nb[1] * q.z)] : -1;
  if (ob >= 0) {
    const double* src = U_old + (long)ob * Layout<N>::BS;
    for (int t = threadIdx.x; t < 5 * N * N * N; t += blockDim.x) out[t] = src[t];
    return;
  }
  for (int t = threadIdx.x; t < N * N * N; t += blockDim.x) {
    double val[5];
    prolong_cell<N>(gp, lookup_p, Up, q.x * N + t % N, q.y * N + (t / N) % N, q.z * N + t / (N * N), val);
#pragma unroll
    for (int v = 0; v < 5; ++v) out[v * Layout<N>::VS + t] = val[v];
  }
}

// Restriction: each cell of a refined block takes the mean of the eight
// cells of its child that cover it: the 2 x 2 sums of the child's two
// planes, each in the order (0,0), (1,0), (0,1), (1,1), added -- the
// order of the leaf step's fused restriction.  Workgroup w covers octant
// oct[w] = 8 r + c, the part of refined block r over its child c (child
// cx + 2cy + 4cz covers cells (cx N/2.., cy N/2.., cz N/2..)), or with oct
// null the octant w % 8 of block refined[w / 8].  The two cells of a fine
// row that one parent cell takes are one 16-byte load.
template <int N>
__global__ __launch_bounds__(256) void amr_restrict_kernel(const int* __restrict__ oct,
                                                           const int* __restrict__ refined,
                                                           const int* __restrict__ child_base,
                                                           const double* __restrict__ Uf, double* __restrict__ Ur) {
  constexpr int H = N / 2;
  const int w = oct ? oct[blockIdx.x] : 8 * refined[blockIdx.x >> 3] + (int)(blockIdx.x & 7);
  const int r = w >> 3;
  const int c = w & 7;
  const long fb = child_base[r] + c;
  const int i0 = (c & 1) * H, j0 = ((c >> 1) & 1) * H, k0 = (c >> 2) * H;
  for (int t = threadIdx.x; t < H * H * H; t += blockDim.x) {
    const int ii = t % H, jj = (t / H) % H, kk = t / (H * H);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const double* f = Uf + Layout<N>::at(fb, 2 * ii, 2 * jj, 2 * kk) + v * Layout<N>::VS;
      const double2 a = *(const double2*)f;
      const double2 b = *(const double2*)(f + N);
      const double2 e = *(const double2*)(f + N * N);
      const double2 h = *(const double2*)(f + N * N + N);
      const double s0 = (a.x + a.y) + (b.x + b.y), s1 = (e.x + e.y) + (h.x + h.y);
      Ur[Layout<N>::at(r, i0 + ii, j0 + jj, k0 + kk) + v * Layout<N>::VS] = (s0 + s1) * 0.125;
    }
  }
}

// Summed signal speed over the listed blocks (all when list is null).
template <int N>
__global__ __launch_bounds__(256) void amr_signal_kernel(GridGeom g, const double* __restrict__ U,
                                                         const int* __restrict__ list, unsigned long long* slot) {
  __shared__ unsigned long long sRed[4];
  const long blk = list ? list[blockIdx.x] : blockIdx.x;
  double smax = 0.0;
  for (int t = threadIdx.x; t < N * N * N; t += 256) {
    double u[5];
    load_cons<N>(U, Layout<N>::at(blk, t % N, (t / N) % N, t / (N * N)), u);
    const double s = signal_speed(u, g);
    smax = (s > smax || !(s == s)) ? s : smax;
  }
  wg_max_to(smax, sRed, slot);
}

// ---------------------------------------------------------------------------
// Guard fill: one workgroup per (block, plane of the guarded view); every
// cell of the guarded view (interior and guard layers, faces, edges and
// corners) receives the state value at its mapped global index.
template <int N, int GW = G>
__global__ __launch_bounds__(256) void fill_guards_kernel(GridGeom g, const double* __restrict__ U,
                                                          double* __restrict__ out,
                                                          const int* __restrict__ list = nullptr) {
  constexpr int P = Guarded<N, GW>::P;
  constexpr long VS = Layout<N>::VS;
  const long blk = list ? (long)list[blockIdx.x / P] : (long)(blockIdx.x / P);
  const int k = (int)(blockIdx.x % P) - GW;
  const int bx = (int)(blk % g.nb[0]);
  const int by = (int)((blk / g.nb[0]) % g.nb[1]);
  const int bz = (int)(blk / ((long)g.nb[0] * g.nb[1]));
  const int nx = g.nb[0] * N, ny = g.nb[1] * N, nz = g.nb[2] * N;
  for (int t = threadIdx.x; t < P * P; t += blockDim.x) {
    const int i = t % P - GW, j = t / P - GW;
    // global index, mapped per axis (guards reach up to G cells out)
    int I = bx * N + i, J = by * N + j, K = bz * N + k;
    I = g.bc[0] == 0 ? ((I % nx) + nx) % nx : min(max(I, 0), nx - 1);
    J = g.bc[1] == 0 ? ((J % ny) + ny) % ny : min(max(J, 0), ny - 1);
    K = g.bc[2] == 0 ? ((K % nz) + nz) % nz : min(max(K, 0), nz - 1);
    const long sb = (long)(I / N) + (long)g.nb[0] * ((J / N) + (long)g.nb[1] * (K / N));
    const long src = Layout<N>::at(sb, I % N, J % N, K % N);
    const long dst = blk * Guarded<N, GW>::BS + (long)(k + GW) * Guarded<N, GW>::PS + (long)(j + GW) * P + (i + GW);
#pragma unroll
    for (int v = 0; v < 5; ++v) out[dst + v * Guarded<N, GW>::VS] = U[src + v * VS];
  }
}

// Standalone CFL signal-speed reduction: one workgroup per block.
template <int N, bool DIR>
__global__ __launch_bounds__(256) void signal_kernel(GridGeom g, const double* __restrict__ U,
                                                     unsigned long long* slot) {
  __shared__ unsigned long long sRed[4];
  const long blk = blockIdx.x;
  double smax = 0.0;
  for (int t = threadIdx.x; t < N * N * N; t += 256) {
    const int i = t % N, j = (t / N) % N, k = t / (N * N);
    double u[5];
    load_cons<N>(U, Layout<N>::at(blk, i, j, k), u);
    const double s = DIR ? signal_speed_dir(u, g) : signal_speed(u, g);
    smax = (s > smax || !(s == s)) ? s : smax;
  }
  wg_max_to(smax, sRed, slot);
}

__global__ void clear_slot_kernel(WorkHeader* ws, int slot) { ws->sig[slot] = 0ull; }

// Streaming copy of n doubles (bandwidth probe): each workgroup moves one
// contiguous chunk with 16-byte accesses, four independent loads in flight
// per thread, nontemporal in both directions (measured 5.4 TB/s against
// 5.1 with one plain load at a time).
typedef double copy_v2 __attribute__((ext_vector_type(2)));
constexpr long COPY_CHUNK = 20480;  // doubles per workgroup (160 KiB)
__global__ __launch_bounds__(256) void copy_kernel(const double* __restrict__ src, double* __restrict__ dst,
                                                   long n) {
  const long base = (long)blockIdx.x * COPY_CHUNK;
  const long end = base + COPY_CHUNK < n ? base + COPY_CHUNK : n;
  long i = base + 2 * (long)threadIdx.x;
  for (; i + 512 * 3 + 1 < end; i += 512 * 4) {
    copy_v2 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = __builtin_nontemporal_load((const copy_v2*)(src + i + 512 * u));
#pragma unroll
    for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(v[u], (copy_v2*)(dst + i + 512 * u));
  }
  for (; i + 1 < end; i += 512) *(double2*)(dst + i) = *(const double2*)(src + i);
  if (i < end) dst[i] = src[i];
}

template <int N, int T>
hipError_t launch_step_t(const GridGeom& g, const StepArgs& a, const StageArgs* st, int plen, hipStream_t s) {
  const long layers = (long)g.nb[2] * N / plen;
  const long ntiles = (long)g.nb[0] * g.nb[1] * (N / T) * (N / T) * layers;
  const long grid = 8 * ((ntiles + 7) / 8);
  if (st)
    hipLaunchKernelGGL((stage_kernel<N, T>), dim3((unsigned)grid), dim3(Tile<T>::NT), 0, s, g, a, *st, ntiles,
                       plen);
  else
    hipLaunchKernelGGL((step_kernel<N, T>), dim3((unsigned)grid), dim3(Tile<T>::NT), 0, s, g, a, ntiles, plen);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_step(int nxb, int tile, const GridGeom& g, const StepArgs& a, const StageArgs* st, int plen,
                       hipStream_t s) {
  const long nz = (long)g.nb[2] * nxb;
  if (plen < 2 || plen > nz || nz % plen) return hipErrorInvalidValue;
  switch (nxb * 100 + tile) {
    case 808: return launch_step_t<8, 8>(g, a, st, plen, s);
    case 1616: return launch_step_t<16, 16>(g, a, st, plen, s);
    case 1608: return launch_step_t<16, 8>(g, a, st, plen, s);
    case 3216: return launch_step_t<32, 16>(g, a, st, plen, s);
    case 3208: return launch_step_t<32, 8>(g, a, st, plen, s);
  }
  return hipErrorInvalidValue;
}

template <int N>
hipError_t launch_amr_t(const AmrLaunch& L, hipStream_t s) {
  constexpr int T = N == 8 ? 8 : 16;
  const int slot = L.slot;
  hipLaunchKernelGGL(amr_begin_kernel, dim3(1), dim3(1), 0, s, L.ws, L.dt, L.cfl, slot);
  // 1. views: level 0 by the same-level map, deeper levels by copies and
  //    prolongation from the level above (states only: any order)
  const AmrLevel& R = L.lev[0];
  // (views of leaves only: the leaf steps and the face fluxes read no
  // others; plane halos when the leaf step's tile spans the block plane)
  constexpr bool HALO = T == N;
  if (R.nleaves) {
    if constexpr (HALO)
      hipLaunchKernelGGL(amr_fill_halo_kernel<N>, dim3((unsigned)R.nleaves), dim3(256), 0, s, R.g, R.g, R.lookup,
                         R.lookup, R.pos, R.U, R.U, R.G, R.leaves, R.zneed);
    else
      hipLaunchKernelGGL((fill_guards_kernel<N, VG>), dim3((unsigned)(R.nleaves * Guarded<N, VG>::P)), dim3(256),
                         0, s, R.g, R.U, R.G, R.leaves);
  }
  for (int l = 1; l < L.nlev; ++l) {
    const AmrLevel& A = L.lev[l];
    const AmrLevel& B = L.lev[l - 1];
    if (!A.nleaves) continue;
    if constexpr (HALO)
      hipLaunchKernelGGL(amr_fill_halo_kernel<N>, dim3((unsigned)A.nleaves), dim3(256), 0, s, A.g, B.g, A.lookup,
                         B.lookup, A.pos, A.U, B.U, A.G, A.leaves, A.zneed);
    else
      hipLaunchKernelGGL(amr_fill_level_kernel<N>, dim3((unsigned)A.nleaves), dim3(256), 0, s, A.g, B.g, A.lookup,
                         B.lookup, A.pos, A.U, B.U, A.G, A.leaves);
  }
  // 2. fluxes at the fine-coarse faces, from the old states and the views,
  //    before the leaf steps write the new states over them
  for (int l = 0; l + 1 < L.nlev; ++l) {
    const AmrLevel& A = L.lev[l];
    const AmrLevel& B = L.lev[l + 1];
    if (A.nreflux)
      hipLaunchKernelGGL(amr_face_flux_kernel<N>, dim3((unsigned)(5 * A.nreflux)), dim3(256), 0, s, A.g, B.g,
                         A.reflux, A.child_base, A.G, B.G, A.U, B.U, A.flux, B.flux, (const WorkHeader*)L.ws);
  }
  // 3. leaf steps (fused tile step over the views, one launch for every
  //    level: amr_segments), written over the state: every read of another
  //    block's old state goes to the views.  Leaves next to a refined block
  //    reduce their signal speed after refluxing instead.  The other leaves
  //    of levels >= 1 also write the restriction of their new state into
  //    their parent octant.
  if (L.segs.tiles)
    hipLaunchKernelGGL((amr_tile_kernel<N, T>), dim3((unsigned)L.segs.tiles), dim3(Tile<T>::NT), 0, s, L.segs, slot,
                       L.ws);
  // 4. refluxing
  for (int l = 0; l + 1 < L.nlev; ++l) {
    const AmrLevel& A = L.lev[l];
    const AmrLevel& B = L.lev[l + 1];
    if (!A.nreflux) continue;
    hipLaunchKernelGGL(amr_reflux_kernel<N>, dim3((unsigned)A.ngroups), dim3(256), 0, s, A.g, A.reflux,
                       A.reflux_first, A.flux, B.flux, A.child_base, A.U, L.ws, slot);
  }
  // 5. restriction of the octants over refined or refluxed children,
  //    finest level first
  for (int l = L.nlev - 2; l >= 0; --l) {
    const AmrLevel& A = L.lev[l];
    if (A.nroct)
      hipLaunchKernelGGL(amr_restrict_kernel<N>, dim3((unsigned)A.nroct), dim3(N == 8 ? 64 : 256), 0, s, A.roct,
                         A.refined, A.child_base, L.lev[l + 1].U, A.U);
  }
  return hipGetLastError();
}

template <int N>
void launch_amr_adapt_t(const AmrLaunch& L, double eps, double* E2, double* const* E2_levels,
                        const AmrLaunch* from, hipStream_t s) {
  const AmrLevel& R = L.lev[0];
  if (E2) hipLaunchKernelGGL(amr_indicator_kernel<N>, dim3((unsigned)R.nblk), dim3(256), 0, s, R.g, R.U, eps, E2);
  if (E2_levels)
    for (int l = 0; l < L.nlev; ++l) {
      const AmrLevel& A = L.lev[l];
      if (A.nleaves)
        hipLaunchKernelGGL(amr_leaf_indicator_kernel<N>, dim3((unsigned)A.nleaves), dim3(256), 0, s, A.g, A.lookup,
                           A.U, A.leaves, A.pos, eps, E2_levels[l]);
    }
  if (from) {
    for (int l = 1; l < L.nlev; ++l) {
      const AmrLevel& A = L.lev[l];
      const AmrLevel& B = L.lev[l - 1];
      const bool has = l < from->nlev;
      hipLaunchKernelGGL(amr_transfer_level_kernel<N>, dim3((unsigned)A.nblk), dim3(256), 0, s, A.g, B.g,
                         has ? from->lev[l].lookup : (const int*)nullptr,
                         has ? (const double*)from->lev[l].U : (const double*)nullptr, B.lookup, B.U, A.pos, A.U);
    }
    for (int l = L.nlev - 2; l >= 0; --l) {
      const AmrLevel& A = L.lev[l];
      if (A.nrefined)
        hipLaunchKernelGGL(amr_restrict_kernel<N>, dim3((unsigned)(8 * A.nrefined)), dim3(N == 8 ? 64 : 256), 0, s,
                           (const int*)nullptr, A.refined, A.child_base, L.lev[l + 1].U, A.U);
    }
  }
}

hipError_t launch_amr_indicator(int nxb, const AmrLaunch& L, double eps, double* E2, hipStream_t s) {
  switch (nxb) {
    case 8: launch_amr_adapt_t<8>(L, eps, E2, nullptr, nullptr, s); break;
    case 16: launch_amr_adapt_t<16>(L, eps, E2, nullptr, nullptr, s); break;
    case 32: launch_amr_adapt_t<32>(L, eps, E2, nullptr, nullptr, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_amr_leaf_indicator(int nxb, const AmrLaunch& L, double eps, double* const* E2_levels,
                                     hipStream_t s) {
  switch (nxb) {
    case 8: launch_amr_adapt_t<8>(L, eps, nullptr, E2_levels, nullptr, s); break;
    case 16: launch_amr_adapt_t<16>(L, eps, nullptr, E2_levels, nullptr, s); break;
    case 32: launch_amr_adapt_t<32>(L, eps, nullptr, E2_levels, nullptr, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

void amr_segments(int nxb, const AmrLaunch& L, AmrSegs& out) {
  const int T = nxb == 8 ? 8 : 16;
  const long tpb = (long)(nxb / T) * (nxb / T);
  struct Cand {
    AmrSeg s;
    int k;
    long ntiles;
  };
  Cand c[AMR_MAX_SEGS];
  int n = 0;
  for (int l = 0; l < L.nlev; ++l) {
    const AmrLevel& A = L.lev[l];
    const ParentOut none{nullptr, nullptr, nullptr};
    const ParentOut po = l ? ParentOut{L.lev[l - 1].U, A.parent, A.pos} : none;
    if (A.ncols_plain) c[n++] = Cand{AmrSeg{A.g, A.G, A.U, A.cols_plain, po, 0, 1, 0}, A.kmax_plain, A.ncols_plain * tpb};
    if (A.ncols_rx) c[n++] = Cand{AmrSeg{A.g, A.G, A.U, A.cols_rx, none, 0, 0, 0}, A.kmax_rx, A.ncols_rx * tpb};
  }
  std::stable_sort(c, c + n, [](const Cand& a, const Cand& b) { return a.k > b.k; });
  long first = 0;
  for (int i = 0; i < n; ++i) {
    out.s[i] = c[i].s;
    out.s[i].first = first;
    first += c[i].ntiles;
  }
  out.n = n;
  out.tiles = first;
}

hipError_t launch_amr_transfer(int nxb, const AmrLaunch& from, const AmrLaunch& to, hipStream_t s) {
  switch (nxb) {
    case 8: launch_amr_adapt_t<8>(to, 0.0, nullptr, nullptr, &from, s); break;
    case 16: launch_amr_adapt_t<16>(to, 0.0, nullptr, nullptr, &from, s); break;
    case 32: launch_amr_adapt_t<32>(to, 0.0, nullptr, nullptr, &from, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_amr_step(int nxb, const AmrLaunch& L, hipStream_t s) {
  switch (nxb) {
    case 8: return launch_amr_t<8>(L, s);
    case 16: return launch_amr_t<16>(L, s);
    case 32: return launch_amr_t<32>(L, s);
  }
  return hipErrorInvalidValue;
}

template <int N>
void launch_amr_signal_t(const AmrLaunch& L, unsigned long long* dst, hipStream_t s) {
  for (int l = 0; l < L.nlev; ++l) {
    const AmrLevel& A = L.lev[l];
    if (A.nleaves)
      hipLaunchKernelGGL(amr_signal_kernel<N>, dim3((unsigned)A.nleaves), dim3(256), 0, s, A.g, A.U, A.leaves, dst);
  }
}

hipError_t launch_amr_signal(int nxb, const AmrLaunch& L, int slot, hipStream_t s) {
  unsigned long long* dst = &L.ws->sig[slot];
  hipLaunchKernelGGL(clear_slot_kernel, dim3(1), dim3(1), 0, s, L.ws, slot);
  switch (nxb) {
    case 8: launch_amr_signal_t<8>(L, dst, s); break;
    case 16: launch_amr_signal_t<16>(L, dst, s); break;
    case 32: launch_amr_signal_t<32>(L, dst, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <bool TRACE>
hipError_t launch_ctu_t(int nxb, const GridGeom& g, const StepArgs& a, hipStream_t s) {
  const long nblk = (long)g.nb[0] * g.nb[1] * g.nb[2];
  const long ntiles = nblk * (nxb / CtuTile::T) * (nxb / CtuTile::T);
  const unsigned grid = (unsigned)(8 * ((ntiles + 7) / 8));
  switch (nxb) {
    case 8: hipLaunchKernelGGL((ctu_tile_kernel<8, TRACE>), dim3(grid), dim3(CtuTile::NT), 0, s, g, a, ntiles); break;
    case 16: hipLaunchKernelGGL((ctu_tile_kernel<16, TRACE>), dim3(grid), dim3(CtuTile::NT), 0, s, g, a, ntiles); break;
    case 32: hipLaunchKernelGGL((ctu_tile_kernel<32, TRACE>), dim3(grid), dim3(CtuTile::NT), 0, s, g, a, ntiles); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_ctu(int nxb, const GridGeom& g, const StepArgs& a, bool trace, hipStream_t s) {
  return trace ? launch_ctu_t<true>(nxb, g, a, s) : launch_ctu_t<false>(nxb, g, a, s);
}

hipError_t launch_batch_step(const BatchSim* sims, const BatchItem* items, int nitems, long step, double cfl,
                             int nxb, int tile, int nseg, int grid, hipStream_t s) {
  // 8x8 tiles: 128-thread workgroups (the 8x8 tile's roles), twice as many
  // of them, so a CU holds the same number of wavefronts
  const unsigned g16 = (unsigned)grid, g8 = (unsigned)(2 * grid);
  switch (nxb * 100 + tile) {
    case 808:
      hipLaunchKernelGGL((batch_step_kernel<8, 8>), dim3(g8), dim3(Tile<8>::NT), 0, s, sims, items, nitems, step, cfl,
                         nseg);
      break;
    case 1616:
      hipLaunchKernelGGL((batch_step_kernel<16, 16>), dim3(g16), dim3(Tile<16>::NT), 0, s, sims, items, nitems, step,
                         cfl, nseg);
      break;
    case 1608:
      hipLaunchKernelGGL((batch_step_kernel<16, 8>), dim3(g8), dim3(Tile<8>::NT), 0, s, sims, items, nitems, step, cfl,
                         nseg);
      break;
    case 3216:
      hipLaunchKernelGGL((batch_step_kernel<32, 16>), dim3(g16), dim3(Tile<16>::NT), 0, s, sims, items, nitems, step,
                         cfl, nseg);
      break;
    case 3208:
      hipLaunchKernelGGL((batch_step_kernel<32, 8>), dim3(g8), dim3(Tile<8>::NT), 0, s, sims, items, nitems, step, cfl,
                         nseg);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fill_guards(int nxb, const GridGeom& g, const double* U, double* out, hipStream_t s) {
  const long nblk = (long)g.nb[0] * g.nb[1] * g.nb[2];
  switch (nxb) {
    case 8:
      hipLaunchKernelGGL(fill_guards_kernel<8>, dim3((unsigned)(nblk * Guarded<8>::P)), dim3(256), 0, s, g, U, out);
      break;
    case 16:
      hipLaunchKernelGGL(fill_guards_kernel<16>, dim3((unsigned)(nblk * Guarded<16>::P)), dim3(256), 0, s, g, U, out);
      break;
    case 32:
      hipLaunchKernelGGL(fill_guards_kernel<32>, dim3((unsigned)(nblk * Guarded<32>::P)), dim3(256), 0, s, g, U, out);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int N>
void launch_signal_t(const GridGeom& g, const double* U, unsigned long long* dst, bool dir, hipStream_t s) {
  const long nblk = (long)g.nb[0] * g.nb[1] * g.nb[2];
  if (dir)
    hipLaunchKernelGGL((signal_kernel<N, true>), dim3((unsigned)nblk), dim3(256), 0, s, g, U, dst);
  else
    hipLaunchKernelGGL((signal_kernel<N, false>), dim3((unsigned)nblk), dim3(256), 0, s, g, U, dst);
}

hipError_t launch_signal(int nxb, const GridGeom& g, const double* U, WorkHeader* ws, int slot, bool dir,
                         hipStream_t s) {
  unsigned long long* dst = &ws->sig[slot];
  hipLaunchKernelGGL(clear_slot_kernel, dim3(1), dim3(1), 0, s, ws, slot);
  switch (nxb) {
    case 8: launch_signal_t<8>(g, U, dst, dir, s); break;
    case 16: launch_signal_t<16>(g, U, dst, dir, s); break;
    case 32: launch_signal_t<32>(g, U, dst, dir, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_copy(const double* src, double* dst, long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long grid = (n + COPY_CHUNK - 1) / COPY_CHUNK;
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)grid), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

// Static scratch of the allocation-free batch step.  Host code never passes
// the array's name to a kernel (on the host it is only a stand-in for the
// symbol): it looks the device address up once per device and passes that.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

hipError_t static_scratch(void** ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

hipError_t launch_clear_slot(WorkHeader* ws, int slot, hipStream_t s) {
  hipLaunchKernelGGL(clear_slot_kernel, dim3(1), dim3(1), 0, s, ws, slot);
  return hipGetLastError();
}

}  // namespace hydro
