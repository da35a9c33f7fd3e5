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
//  * Each thread owns one cell of the predictor footprint (the tile plus one
//    ring) and keeps that column's primitives for planes j-1, j, j+1 in
//    registers (z slopes, z face states and z fluxes never touch LDS).  The
//    in-plane neighbours, the x/y face states and the x/y fluxes go through
//    LDS, so every face flux is computed exactly once per tile.
//  * The CFL signal speed of the new state is reduced in the epilogue
//    (wavefront shuffles, then one atomicMax per workgroup on the bit
//    pattern), so the next dt needs no extra pass over the state.
#include "hydro_internal.h"

#include <math.h>

namespace hydro {
namespace {

constexpr int G = 4;  // guard layers per side of the guarded view

// Compact state layout: block b, variable v, cell (i, j, k).
template <int N>
struct Layout {
  static constexpr long PS = (long)N * N;
  static constexpr long VS = PS * N;
  static constexpr long BS = 5 * VS;
  // offset of cell (i, j, k) of block b, variable 0
  __device__ static long at(long b, int i, int j, int k) { return b * BS + (long)k * PS + (long)j * N + i; }
};

// Guarded view: [block][var][P][P][P], P = N + 2G, interior at offset G.
template <int N>
struct Guarded {
  static constexpr int P = N + 2 * G;
  static constexpr long PS = (long)P * P;
  static constexpr long VS = PS * P;
  static constexpr long BS = 5 * VS;
};

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

// Conservative -> primitive, gamma-law EOS, pressure floor.  Returns 1 if the
// floor was applied.
__device__ __forceinline__ int cons_to_prim(const double (&u)[5], double gamma, double small_p,
                                            double (&w)[5]) {
  const double rho = u[0];
  const double vx = u[1] / rho, vy = u[2] / rho, vz = u[3] / rho;
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

__device__ __forceinline__ double van_leer(double a, double b) {
  const double ab = a * b;
  return ab > 0.0 ? (2.0 * ab) / (a + b) : 0.0;
}

// out += lam * A_D(w) * d  (primitive-form Euler Jacobian along axis D)
template <int D>
__device__ __forceinline__ void add_jacobian(const double (&w)[5], const double (&d)[5], double gamma,
                                             double lam, double (&out)[5]) {
  const double un = w[1 + D];
  double t[5];
  t[0] = un * d[0] + w[0] * d[1 + D];
  t[1] = un * d[1];
  t[2] = un * d[2];
  t[3] = un * d[3];
  t[1 + D] += d[4] / w[0];
  t[4] = gamma * w[4] * d[1 + D] + un * d[4];
#pragma unroll
  for (int v = 0; v < 5; ++v) out[v] += lam * t[v];
}

// HLLC flux normal to axis D between primitive states L and R.
template <int D>
__device__ __forceinline__ void hllc(const double (&L)[5], const double (&R)[5], double gamma,
                                     double (&F)[5]) {
  const double rL = L[0], uL = L[1 + D], pL = L[4];
  const double rR = R[0], uR = R[1 + D], pR = R[4];
  const double cL = sqrt(gamma * pL / rL);
  const double cR = sqrt(gamma * pR / rR);
  const double SL = fmin(uL - cL, uR - cR);
  const double SR = fmax(uL + cL, uR + cR);
  const double Ss = (pR - pL + rL * uL * (SL - uL) - rR * uR * (SR - uR)) /
                    (rL * (SL - uL) - rR * (SR - uR));
  // Upwind side K and whether the star correction applies:
  //   SL >= 0 -> F_L;  S* >= 0 -> F*_L;  SR > 0 -> F*_R;  else F_R.
  const bool left = (SL >= 0.0) || (Ss >= 0.0);
  const double S = left ? SL : SR;
  const bool corr = left ? (SL < 0.0) : (SR > 0.0);
  double W[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) W[v] = left ? L[v] : R[v];
  const double rho = W[0], un = W[1 + D], p = W[4];
  const double E = p / (gamma - 1.0) + 0.5 * rho * ((W[1] * W[1] + W[2] * W[2]) + W[3] * W[3]);
  const double mass = rho * un;
  F[0] = mass;
  F[1] = mass * W[1];
  F[2] = mass * W[2];
  F[3] = mass * W[3];
  F[1 + D] += p;
  F[4] = un * (E + p);
  if (corr) {
    const double factor = rho * (S - un) / (S - Ss);
    double dU[5];
    dU[0] = factor - rho;
    dU[1] = factor * W[1] - rho * W[1];
    dU[2] = factor * W[2] - rho * W[2];
    dU[3] = factor * W[3] - rho * W[3];
    dU[1 + D] = factor * Ss - rho * un;
    dU[4] = factor * (E / rho + (Ss - un) * (Ss + p / (rho * (S - un)))) - E;
#pragma unroll
    for (int v = 0; v < 5; ++v) F[v] += S * dU[v];
  }
}

// Maximum over a workgroup of a non-negative double, folded into *slot with
// one atomicMax on the bit pattern.  red must hold one entry per wavefront.
template <int NT>
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
    for (int w = 1; w < (NT + 63) / 64; ++w) m = red[w] > m ? red[w] : m;
    atomicMax(slot, m);
  }
}

__device__ __forceinline__ double signal_speed(const double (&u)[5], const GridGeom& g) {
  double w[5];
  cons_to_prim(u, g.gamma, g.small_p, w);
  const double c = sqrt(g.gamma * w[4] / w[0]);
  return ((fabs(w[1]) + c) * g.inv_dx[0] + (fabs(w[2]) + c) * g.inv_dx[1]) +
         (fabs(w[3]) + c) * g.inv_dx[2];
}

// ---------------------------------------------------------------------------
// Fused step kernel.  Template: N block edge, T tile edge (N % T == 0).
// Thread roles (NP = (T+2)^2 - 4 predictor cells):
//   tid <  T*T      : tile cell (x, y) = (tid % T, tid / T)
//   tid <  NP       : ring cell, side r/T: x=-1 | x=T | y=-1 | y=T
// Extra cells, primitives only (x/y slopes of the ring): x=-2 | x=T+1 |
// y=-2 | y=T+1 rows, then the 4 edge cells (+-1 corners of the ring).
template <int T>
struct Tile {
  static constexpr int NP = (T + 2) * (T + 2) - 4;
  static constexpr int NT = ((NP + 63) / 64) * 64;
  static constexpr int NE = 4 * T + 4;
  static constexpr int WS = T + 4;  // sW row pitch
  static constexpr int PSP = T + 2; // sP row pitch
  static constexpr int NFX = (T + 1) * T;

  __device__ static void cell_of(int t, int& x, int& y) {
    if (t < T * T) {
      x = t % T;
      y = t / T;
      return;
    }
    const int r = t - T * T, side = r / T, s = r % T;
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

template <int N, int T>
__global__ __launch_bounds__(Tile<T>::NT) void step_kernel(GridGeom g, StepArgs a) {
  using TL = Tile<T>;
  constexpr int NT = TL::NT, NP = TL::NP, NE = TL::NE, WS = TL::WS, PSP = TL::PSP;
  constexpr int TPB = (N / T) * (N / T);  // tiles per block
  constexpr long VS = Layout<N>::VS;

  __shared__ double sW[5][WS * WS];         // primitives of plane j (tile + 2-halo)
  __shared__ double sP[15][PSP * PSP];      // predicted centre, x slope, y slope
  __shared__ int sFB[PSP * PSP];            // first-order fallback flags
  __shared__ double sFx[5][TL::NFX];        // x fluxes: face (x, y) between x-1 and x
  __shared__ double sFy[5][TL::NFX];        // y fluxes: face (x, y) between y-1 and y
  __shared__ unsigned long long sRed[NT / 64];
  __shared__ int sCnt[3];

  const int tid = threadIdx.x;
  const long blk = blockIdx.x / TPB;
  const int tile = blockIdx.x % TPB;
  const int bx = (int)(blk % g.nb[0]);
  const int by = (int)((blk / g.nb[0]) % g.nb[1]);
  const int bz = (int)(blk / ((long)g.nb[0] * g.nb[1]));
  const int X0 = bx * N + (tile % (N / T)) * T;  // global index of the tile origin
  const int Y0 = by * N + (tile / (N / T)) * T;
  const int Z0 = bz * N;

  if (tid < 3) sCnt[tid] = 0;

  double dt = a.dt;
  if (a.cfl > 0.0) dt = a.cfl / __longlong_as_double(a.ws->sig[a.slot]);
  if (blockIdx.x == 0 && tid == 0) {
    a.ws->dt_last = dt;
    a.ws->sig[(a.slot + 2) % 3] = 0ull;
  }
  const double lamx = dt * g.inv_dx[0], lamy = dt * g.inv_dx[1], lamz = dt * g.inv_dx[2];
  const double gamma = g.gamma;

  // own cell
  const bool pred = tid < NP;
  const bool inner = tid < T * T;
  int cx = 0, cy = 0;
  if (pred) TL::cell_of(tid, cx, cy);
  const int cidx = (cy + 2) * WS + (cx + 2);
  const int pidx = (cy + 1) * PSP + (cx + 1);

  // window of own-cell primitives: Wa = plane j-1, Wb = plane j, Wc = plane j+1
  double Wa[5], Wb[5], Wc[5];
  double zp_prev[5], fz_prev[5], dxy_prev[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    Wa[v] = Wb[v] = Wc[v] = 0.0;
    zp_prev[v] = fz_prev[v] = dxy_prev[v] = 0.0;
  }
  int n_floor = 0, n_fb = 0, n_bad = 0;
  double smax = 0.0;

  if (pred) {
    double u[5];
    load_cons<N>(a.Uin, cell_offset<N>(g, X0 + cx, Y0 + cy, Z0 - 2), u);
    cons_to_prim(u, gamma, g.small_p, Wa);
    load_cons<N>(a.Uin, cell_offset<N>(g, X0 + cx, Y0 + cy, Z0 - 1), u);
    cons_to_prim(u, gamma, g.small_p, Wb);
  }

  for (int j = -1; j <= N; ++j) {
    const bool mid = (j >= 0) && (j < N);
    // -- load plane j+1 (own cell), publish plane j primitives
    if (pred) {
      double u[5];
      load_cons<N>(a.Uin, cell_offset<N>(g, X0 + cx, Y0 + cy, Z0 + j + 1), u);
      const int fl = cons_to_prim(u, gamma, g.small_p, Wc);
      if (inner && j + 1 >= 0 && j + 1 < N) n_floor += fl;
#pragma unroll
      for (int v = 0; v < 5; ++v) sW[v][cidx] = Wb[v];
    }
    if (mid) {
      for (int e = (tid + NT - NP) % NT; e < NE; e += NT) {
        int ex, ey;
        TL::extra_of(e, ex, ey);
        double u[5], w[5];
        load_cons<N>(a.Uin, cell_offset<N>(g, X0 + ex, Y0 + ey, Z0 + j), u);
        cons_to_prim(u, gamma, g.small_p, w);
#pragma unroll
        for (int v = 0; v < 5; ++v) sW[v][(ey + 2) * WS + (ex + 2)] = w[v];
      }
    }
    __syncthreads();

    // -- predictor at plane j
    double zm[5], zp[5];
    const bool active = mid ? pred : inner;
    if (active) {
      double sx[5], sy[5], sz[5], wt[5];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const double c = Wb[v];
        sx[v] = van_leer(c - sW[v][cidx - 1], sW[v][cidx + 1] - c);
        sy[v] = van_leer(c - sW[v][cidx - WS], sW[v][cidx + WS] - c);
        sz[v] = van_leer(c - Wa[v], Wc[v] - c);
      }
      double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
      add_jacobian<0>(Wb, sx, gamma, lamx, acc);
      add_jacobian<1>(Wb, sy, gamma, lamy, acc);
      add_jacobian<2>(Wb, sz, gamma, lamz, acc);
#pragma unroll
      for (int v = 0; v < 5; ++v) wt[v] = Wb[v] - 0.5 * acc[v];
      const bool ok = (wt[0] + 0.5 * sx[0] > 0.0) && (wt[0] - 0.5 * sx[0] > 0.0) &&
                      (wt[0] + 0.5 * sy[0] > 0.0) && (wt[0] - 0.5 * sy[0] > 0.0) &&
                      (wt[0] + 0.5 * sz[0] > 0.0) && (wt[0] - 0.5 * sz[0] > 0.0) &&
                      (wt[4] + 0.5 * sx[4] > 0.0) && (wt[4] - 0.5 * sx[4] > 0.0) &&
                      (wt[4] + 0.5 * sy[4] > 0.0) && (wt[4] - 0.5 * sy[4] > 0.0) &&
                      (wt[4] + 0.5 * sz[4] > 0.0) && (wt[4] - 0.5 * sz[4] > 0.0);
      if (mid) {
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          sP[v][pidx] = wt[v];
          sP[5 + v][pidx] = sx[v];
          sP[10 + v][pidx] = sy[v];
        }
        sFB[pidx] = ok ? 0 : 1;
        if (inner && !ok) ++n_fb;
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        zm[v] = ok ? wt[v] - 0.5 * sz[v] : Wb[v];
        zp[v] = ok ? wt[v] + 0.5 * sz[v] : Wb[v];
      }
    }
    // -- z flux at j-1/2 (tile cells)
    double fz[5];
    if (inner && j >= 0) hllc<2>(zp_prev, zm, gamma, fz);
    __syncthreads();

    // -- x and y fluxes of plane j
    if (mid) {
      for (int f = tid; f < 2 * TL::NFX; f += NT) {
        const bool isx = f < TL::NFX;
        const int q = isx ? f : f - TL::NFX;
        int fx, fy, lx, ly;
        if (isx) {
          fx = q % (T + 1);
          fy = q / (T + 1);
          lx = fx - 1;
          ly = fy;
        } else {
          fx = q % T;
          fy = q / T;
          lx = fx;
          ly = fy - 1;
        }
        const int pl = (ly + 1) * PSP + (lx + 1), pr = (fy + 1) * PSP + (fx + 1);
        const int wl = (ly + 2) * WS + (lx + 2), wr = (fy + 2) * WS + (fx + 2);
        const int so = isx ? 5 : 10;
        const bool fbl = sFB[pl] != 0, fbr = sFB[pr] != 0;
        double WL[5], WR[5], F[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          WL[v] = fbl ? sW[v][wl] : sP[v][pl] + 0.5 * sP[so + v][pl];
          WR[v] = fbr ? sW[v][wr] : sP[v][pr] - 0.5 * sP[so + v][pr];
        }
        if (isx) {
          hllc<0>(WL, WR, gamma, F);
#pragma unroll
          for (int v = 0; v < 5; ++v) sFx[v][q] = F[v];
        } else {
          hllc<1>(WL, WR, gamma, F);
#pragma unroll
          for (int v = 0; v < 5; ++v) sFy[v][q] = F[v];
        }
      }
    }
    __syncthreads();

    // -- update plane j-1, keep plane j's x/y divergence
    if (inner) {
      double dxy[5];
      if (mid) {
        const int qx = cy * (T + 1) + cx, qy = cy * T + cx;
#pragma unroll
        for (int v = 0; v < 5; ++v)
          dxy[v] = lamx * (sFx[v][qx + 1] - sFx[v][qx]) + lamy * (sFy[v][qy + T] - sFy[v][qy]);
      }
      if (j >= 1) {
        const long off = cell_offset<N>(g, X0 + cx, Y0 + cy, Z0 + j - 1);
        double u[5];
        load_cons<N>(a.Uin, off, u);
        double un[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) un[v] = u[v] - (dxy_prev[v] + lamz * (fz[v] - fz_prev[v]));
#pragma unroll
        for (int v = 0; v < 5; ++v) a.Uout[off + v * VS] = un[v];
        bool good = un[0] > 0.0 && un[4] > 0.0;
#pragma unroll
        for (int v = 0; v < 5; ++v) good = good && isfinite(un[v]);
        if (!good) ++n_bad;
        const double s = signal_speed(un, g);
        smax = (s > smax || !(s == s)) ? s : smax;
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        if (mid) dxy_prev[v] = dxy[v];
        if (j >= 0) fz_prev[v] = fz[v];
        zp_prev[v] = zp[v];
      }
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      Wa[v] = Wb[v];
      Wb[v] = Wc[v];
    }
  }

  // -- epilogue: signal-speed maximum and event counters
  if (n_floor) atomicAdd(&sCnt[0], n_floor);
  if (n_fb) atomicAdd(&sCnt[1], n_fb);
  if (n_bad) atomicAdd(&sCnt[2], n_bad);
  wg_max_to<NT>(smax, sRed, &a.ws->sig[(a.slot + 1) % 3]);
  if (tid == 0) {
    for (int c = 0; c < 3; ++c)
      if (sCnt[c]) atomicAdd(&a.ws->cnt[c], (unsigned long long)sCnt[c]);
  }
}

// ---------------------------------------------------------------------------
// Guard fill: one workgroup per (block, plane of the guarded view); every
// cell of the guarded view (interior and guard layers, faces, edges and
// corners) receives the state value at its mapped global index.
template <int N>
__global__ __launch_bounds__(256) void fill_guards_kernel(GridGeom g, const double* __restrict__ U,
                                                          double* __restrict__ out) {
  constexpr int P = Guarded<N>::P;
  constexpr long VS = Layout<N>::VS;
  const long blk = blockIdx.x / P;
  const int k = (int)(blockIdx.x % P) - G;
  const int bx = (int)(blk % g.nb[0]);
  const int by = (int)((blk / g.nb[0]) % g.nb[1]);
  const int bz = (int)(blk / ((long)g.nb[0] * g.nb[1]));
  const int nx = g.nb[0] * N, ny = g.nb[1] * N, nz = g.nb[2] * N;
  for (int t = threadIdx.x; t < P * P; t += blockDim.x) {
    const int i = t % P - G, j = t / P - G;
    // global index, mapped per axis (guards reach up to G cells out)
    int I = bx * N + i, J = by * N + j, K = bz * N + k;
    I = g.bc[0] == 0 ? ((I % nx) + nx) % nx : min(max(I, 0), nx - 1);
    J = g.bc[1] == 0 ? ((J % ny) + ny) % ny : min(max(J, 0), ny - 1);
    K = g.bc[2] == 0 ? ((K % nz) + nz) % nz : min(max(K, 0), nz - 1);
    const long sb = (long)(I / N) + (long)g.nb[0] * ((J / N) + (long)g.nb[1] * (K / N));
    const long src = Layout<N>::at(sb, I % N, J % N, K % N);
    const long dst = blk * Guarded<N>::BS + (long)(k + G) * Guarded<N>::PS + (long)(j + G) * P + (i + G);
#pragma unroll
    for (int v = 0; v < 5; ++v) out[dst + v * Guarded<N>::VS] = U[src + v * VS];
  }
}

// Standalone CFL signal-speed reduction: one workgroup per block.
template <int N>
__global__ __launch_bounds__(256) void signal_kernel(GridGeom g, const double* __restrict__ U,
                                                     unsigned long long* slot) {
  __shared__ unsigned long long sRed[4];
  const long blk = blockIdx.x;
  double smax = 0.0;
  for (int t = threadIdx.x; t < N * N * N; t += 256) {
    const int i = t % N, j = (t / N) % N, k = t / (N * N);
    double u[5];
    load_cons<N>(U, Layout<N>::at(blk, i, j, k), u);
    const double s = signal_speed(u, g);
    smax = (s > smax || !(s == s)) ? s : smax;
  }
  wg_max_to<256>(smax, sRed, slot);
}

__global__ void clear_slot_kernel(WorkHeader* ws, int slot) { ws->sig[slot] = 0ull; }

// Streaming copy of n doubles (bandwidth probe): each workgroup moves one
// contiguous chunk with 16-byte accesses.
constexpr long COPY_CHUNK = 20480;  // doubles per workgroup (160 KiB)
__global__ __launch_bounds__(256) void copy_kernel(const double* __restrict__ src, double* __restrict__ dst,
                                                   long n) {
  const long base = (long)blockIdx.x * COPY_CHUNK;
  const long end = base + COPY_CHUNK < n ? base + COPY_CHUNK : n;
  long i = base + 2 * (long)threadIdx.x;
  for (; i + 1 < end; i += 512) *(double2*)(dst + i) = *(const double2*)(src + i);
  if (i < end) dst[i] = src[i];
}

template <int N, int T>
hipError_t launch_step_t(const GridGeom& g, const StepArgs& a, hipStream_t s) {
  const long nblk = (long)g.nb[0] * g.nb[1] * g.nb[2];
  const long grid = nblk * (N / T) * (N / T);
  hipLaunchKernelGGL((step_kernel<N, T>), dim3((unsigned)grid), dim3(Tile<T>::NT), 0, s, g, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_step(int nxb, const GridGeom& g, const StepArgs& a, hipStream_t s) {
  switch (nxb) {
    case 8: return launch_step_t<8, 8>(g, a, s);
    case 16: return launch_step_t<16, 16>(g, a, s);
    case 32: return launch_step_t<32, 16>(g, a, s);
  }
  return hipErrorInvalidValue;
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

hipError_t launch_signal(int nxb, const GridGeom& g, const double* U, WorkHeader* ws, int slot,
                         hipStream_t s) {
  const long nblk = (long)g.nb[0] * g.nb[1] * g.nb[2];
  unsigned long long* dst = &ws->sig[slot];
  hipLaunchKernelGGL(clear_slot_kernel, dim3(1), dim3(1), 0, s, ws, slot);
  switch (nxb) {
    case 8: hipLaunchKernelGGL(signal_kernel<8>, dim3((unsigned)nblk), dim3(256), 0, s, g, U, dst); break;
    case 16: hipLaunchKernelGGL(signal_kernel<16>, dim3((unsigned)nblk), dim3(256), 0, s, g, U, dst); break;
    case 32: hipLaunchKernelGGL(signal_kernel<32>, dim3((unsigned)nblk), dim3(256), 0, s, g, U, dst); break;
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

hipError_t launch_clear_slot(WorkHeader* ws, int slot, hipStream_t s) {
  hipLaunchKernelGGL(clear_slot_kernel, dim3(1), dim3(1), 0, s, ws, slot);
  return hipGetLastError();
}

}  // namespace hydro
