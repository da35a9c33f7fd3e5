// C-ABI host side of libhydro: descriptor validation, handles, launches.
// The operation and the conventions are documented in include/hydro.h.
#include "hydro.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <queue>
#include <set>
#include <vector>

#include "hydro_internal.h"

struct hydro_batch;

static_assert(HYDRO_STATIC_MAX_GRIDS == hydro::kStaticMaxGrids, "static scratch: grid limit");
static_assert(HYDRO_STATIC_MAX_ITEMS == hydro::kStaticMaxItems, "static scratch: item limit");

struct hydro_grid {
  hydro_grid_desc d;
  hydro::GridGeom geom;
  int cur;                  // 0: state in d.U, 1: in d.U_alt
  unsigned long long steps; // steps taken; signal slot of the current state = steps % 3
  bool sig_valid;           // slot holds the current state's maximum signal speed
  int plen;                 // planes per z pencil (tuning; results do not depend on it)
  int tile;                 // column tile edge, 8 or 16 (tuning; results do not depend on it)
  hydro_batch* batch;       // batch the grid belongs to (its own step calls are refused meanwhile)
  int scheme;               // HYDRO_SCHEME_*
  double* U_stage;          // third state buffer (third-order Runge-Kutta)
  unsigned long long mark;  // last hydro_batch_step_static call that listed the grid
};

struct hydro_batch {
  std::vector<hydro_grid*> grids;
  std::vector<unsigned char> active;     // member takes part in the next steps
  std::vector<hydro::BatchSim> sims;     // host copy of the device table
  std::vector<hydro::BatchItem> items;   // host copy of the device work list
  hydro::BatchSim* d_sims;
  hydro::BatchItem* d_items;
  size_t max_items;
  void* stream;
  int nseg[3];                           // pencils per column for nxb 8, 16, 32
  int tile[3];                           // column tile edge for nxb 8, 16, 32
  int grid;                              // persistent workgroups
  long cls_begin[3], cls_count[3];       // work-list range of each size class (8, 16, 32)
  int cus;
  long step;                             // steps since the table was last uploaded
  bool dirty;                            // table / list must be rebuilt before the next step
  bool use_graph;
  double graph_cfl;                      // cfl baked into the captured graph
  hipGraph_t graph;
  hipGraphExec_t exec;
};

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(HYDRO_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }


int validate(const hydro_grid_desc* d) {
  if (!d) return fail(HYDRO_EINVAL, "descriptor is NULL");
  if (d->nxb != 8 && d->nxb != 16 && d->nxb != 32)
    return fail(HYDRO_EINVAL, "nxb must be 8, 16 or 32 (got %d)", d->nxb);
  if (d->nguard != HYDRO_NGUARD) return fail(HYDRO_EINVAL, "nguard must be %d (got %d)", HYDRO_NGUARD, d->nguard);
  long long nblk = 1;
  for (int a = 0; a < 3; ++a) {
    if (d->nblk[a] < 1) return fail(HYDRO_EINVAL, "nblk[%d] must be >= 1 (got %d)", a, d->nblk[a]);
    nblk *= d->nblk[a];
    if ((long long)d->nblk[a] * d->nxb > (1 << 24))
      return fail(HYDRO_EINVAL, "axis %d has more than 2^24 cells", a);
    if (!(std::isfinite(d->lo[a]) && std::isfinite(d->hi[a]) && d->hi[a] > d->lo[a]))
      return fail(HYDRO_EINVAL, "domain axis %d needs finite lo < hi", a);
    const double dx = (d->hi[a] - d->lo[a]) / ((double)d->nblk[a] * d->nxb);
    if (!finite_pos(dx)) return fail(HYDRO_EINVAL, "cell width along axis %d is not positive", a);
    if (d->bc[a] != HYDRO_BC_PERIODIC && d->bc[a] != HYDRO_BC_OUTFLOW)
      return fail(HYDRO_EINVAL, "bc[%d] must be HYDRO_BC_PERIODIC or HYDRO_BC_OUTFLOW", a);
  }
  if (nblk > (1LL << 31) / 16) return fail(HYDRO_EINVAL, "too many blocks (%lld)", nblk);
  const long long layer_bytes = (long long)d->nblk[0] * d->nblk[1] * 5 * d->nxb * d->nxb * d->nxb * 8;
  if (layer_bytes >= (1LL << 32))
    return fail(HYDRO_EINVAL, "a z layer of blocks (nblk[0]*nblk[1] blocks) must hold less than 4 GiB");
  if (!(std::isfinite(d->gamma) && d->gamma > 1.0)) return fail(HYDRO_EINVAL, "gamma must be finite and > 1");
  if (!(std::isfinite(d->small_p) && d->small_p >= 0.0)) return fail(HYDRO_EINVAL, "small_p must be finite and >= 0");
  if (!d->U || !d->U_alt) return fail(HYDRO_EINVAL, "state buffers must be non-NULL");
  if (((uintptr_t)d->U | (uintptr_t)d->U_alt) & 255)
    return fail(HYDRO_EINVAL, "state buffers must be 256-byte aligned");
  const size_t bytes = hydro_state_doubles(d) * sizeof(double);
  const uintptr_t a0 = (uintptr_t)d->U, a1 = (uintptr_t)d->U_alt;
  if ((a0 < a1 ? a1 - a0 : a0 - a1) < bytes) return fail(HYDRO_EINVAL, "state buffers overlap");
  if (!d->work) return fail(HYDRO_EINVAL, "workspace must be non-NULL");
  if ((uintptr_t)d->work & 255) return fail(HYDRO_EINVAL, "workspace must be 256-byte aligned");
  if (d->work_bytes < hydro_work_bytes(d))
    return fail(HYDRO_ESIZE, "workspace has %zu bytes, needs %zu", d->work_bytes, hydro_work_bytes(d));
  return HYDRO_OK;
}

hipStream_t stream_of(const hydro_grid* g) { return (hipStream_t)g->d.stream; }
hydro::WorkHeader* ws_of(const hydro_grid* g) { return (hydro::WorkHeader*)g->d.work; }
double* cur_state(const hydro_grid* g) { return g->cur ? g->d.U_alt : g->d.U; }
double* other_state(const hydro_grid* g) { return g->cur ? g->d.U : g->d.U_alt; }
int slot_of(const hydro_grid* g) { return (int)(g->steps % 3); }

bool is_ctu(int scheme) { return scheme == HYDRO_SCHEME_CTU || scheme == HYDRO_SCHEME_CTU_CHAR; }

int check_device() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  hipDeviceProp_t p;
  e = hipGetDeviceProperties(&p, dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  if (strncmp(p.gcnArchName, "gfx950", 6) != 0)
    return fail(HYDRO_EDEVICE, "device %d is %s; this library is built for gfx950", dev, p.gcnArchName);
  return HYDRO_OK;
}

int ensure_signal_on(hydro_grid* g, hipStream_t s) {
  if (g->sig_valid) return HYDRO_OK;
  hipError_t e = hydro::launch_signal(g->d.nxb, g->geom, cur_state(g), ws_of(g), slot_of(g), is_ctu(g->scheme), s);
  if (e != hipSuccess) return hip_fail(e, "signal-speed kernel launch");
  g->sig_valid = true;
  return HYDRO_OK;
}

int ensure_signal(hydro_grid* g) { return ensure_signal_on(g, stream_of(g)); }

// SSP Runge-Kutta step in Shu-Osher form from the current buffer A, with
// B = the other buffer and C = the stage buffer:
//   order 2: A -> B (U1 = U + dt L(U)); (B, A) -> A (1/2 U + 1/2 (U1 + dt L(U1)))
//   order 3: A -> B; (B, A) -> C (3/4 U + 1/4 (...)); (C, A) -> A (1/3 U + 2/3 (...))
// The last stage writes over the base state cell by cell, so the state stays
// in A.
int do_rk_step(hydro_grid* g, double dt, double cfl) {
  double* A = cur_state(g);
  double* B = other_state(g);
  const int order = g->scheme == HYDRO_SCHEME_RK3 ? 3 : 2;
  struct Stage {
    const double* in;
    double* out;
    const double* base;
    double a0, a1;
  };
  const Stage rk2[2] = {{A, B, nullptr, 0.0, 0.0}, {B, A, A, 0.5, 0.5}};
  const Stage rk3[3] = {{A, B, nullptr, 0.0, 0.0}, {B, g->U_stage, A, 0.75, 0.25},
                        {g->U_stage, A, A, 1.0 / 3.0, 2.0 / 3.0}};
  const Stage* stages = order == 3 ? rk3 : rk2;
  for (int k = 0; k < order; ++k) {
    hydro::StepArgs a;
    a.Uin = stages[k].in;
    a.Uout = stages[k].out;
    a.ws = ws_of(g);
    a.dt = dt;
    a.cfl = cfl;
    a.slot = slot_of(g);
    hydro::StageArgs st;
    st.U0 = stages[k].base;
    st.a0 = stages[k].a0;
    st.a1 = stages[k].a1;
    st.stage = k;
    st.last = k == order - 1;
    hipError_t e = hydro::launch_step(g->d.nxb, g->tile, g->geom, a, &st, g->plen, stream_of(g));
    if (e != hipSuccess) return hip_fail(e, "stage kernel launch");
  }
  g->steps += 1;
  g->sig_valid = true;
  return HYDRO_OK;
}

int do_ctu_step(hydro_grid* g, double dt, double cfl) {
  hydro::StepArgs a;
  a.Uin = cur_state(g);
  a.Uout = other_state(g);
  a.ws = ws_of(g);
  a.dt = dt;
  a.cfl = cfl;
  a.slot = slot_of(g);
  hipError_t e = hydro::launch_ctu(g->d.nxb, g->geom, a, g->scheme == HYDRO_SCHEME_CTU_CHAR, stream_of(g));
  if (e != hipSuccess) return hip_fail(e, "CTU kernel launch");
  g->cur ^= 1;
  g->steps += 1;
  g->sig_valid = true;
  return HYDRO_OK;
}

int do_step(hydro_grid* g, double dt, double cfl) {
  if (is_ctu(g->scheme)) return do_ctu_step(g, dt, cfl);
  if (g->scheme != HYDRO_SCHEME_MH) return do_rk_step(g, dt, cfl);
  hydro::StepArgs a;
  a.Uin = cur_state(g);
  a.Uout = other_state(g);
  a.ws = ws_of(g);
  a.dt = dt;
  a.cfl = cfl;
  a.slot = slot_of(g);
  hipError_t e = hydro::launch_step(g->d.nxb, g->tile, g->geom, a, nullptr, g->plen, stream_of(g));
  if (e != hipSuccess) return hip_fail(e, "step kernel launch");
  g->cur ^= 1;
  g->steps += 1;
  g->sig_valid = true;
  return HYDRO_OK;
}

bool overlaps(const void* p, size_t pb, const void* q, size_t qb) {
  const uintptr_t a0 = (uintptr_t)p, a1 = a0 + pb, b0 = (uintptr_t)q, b1 = b0 + qb;
  return a0 < b1 && b0 < a1;
}

int read_header(hydro_grid* g, hydro::WorkHeader* h) {
  hipError_t e = hipMemcpyAsync(h, g->d.work, sizeof *h, hipMemcpyDeviceToHost, stream_of(g));
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync (workspace header)");
  e = hipStreamSynchronize(stream_of(g));
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return HYDRO_OK;
}

}  // namespace

extern "C" {

size_t hydro_state_doubles(const hydro_grid_desc* d) {
  if (!d || d->nxb <= 0 || d->nblk[0] < 1 || d->nblk[1] < 1 || d->nblk[2] < 1) return 0;
  const size_t n = (size_t)d->nxb;
  return (size_t)d->nblk[0] * d->nblk[1] * d->nblk[2] * 5 * n * n * n;
}

size_t hydro_guarded_doubles(const hydro_grid_desc* d) {
  if (!d || d->nxb <= 0 || d->nguard < 0 || d->nblk[0] < 1 || d->nblk[1] < 1 || d->nblk[2] < 1) return 0;
  const size_t P = (size_t)d->nxb + 2 * (size_t)d->nguard;
  return (size_t)d->nblk[0] * d->nblk[1] * d->nblk[2] * 5 * P * P * P;
}

size_t hydro_work_bytes(const hydro_grid_desc* d) {
  (void)d;
  return sizeof(hydro::WorkHeader);
}

int hydro_init_grid(const hydro_grid_desc* d, hydro_grid** out) {
  if (!out) return fail(HYDRO_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(d);
  if (rc) return rc;
  rc = check_device();
  if (rc) return rc;
  hydro_grid* g = new (std::nothrow) hydro_grid;
  if (!g) return fail(HYDRO_EINVAL, "out of host memory");
  g->d = *d;
  for (int a = 0; a < 3; ++a) {
    g->geom.nb[a] = d->nblk[a];
    g->geom.bc[a] = d->bc[a];
    const double dx = (d->hi[a] - d->lo[a]) / ((double)d->nblk[a] * d->nxb);
    g->geom.inv_dx[a] = 1.0 / dx;
  }
  g->geom.gamma = d->gamma;
  g->geom.small_p = d->small_p;
  g->cur = 0;
  g->steps = 0;
  g->sig_valid = false;
  g->plen = d->nxb;
  g->tile = d->nxb == 8 ? 8 : 16;
  g->batch = nullptr;
  g->mark = 0;
  g->scheme = HYDRO_SCHEME_MH;
  g->U_stage = nullptr;
  hipError_t e = hipMemsetAsync(d->work, 0, sizeof(hydro::WorkHeader), (hipStream_t)d->stream);
  if (e != hipSuccess) {
    delete g;
    return hip_fail(e, "hipMemsetAsync (workspace)");
  }
  *out = g;
  return HYDRO_OK;
}

int hydro_fill_guards(hydro_grid* g, double* guarded) {
  if (!g) return fail(HYDRO_EINVAL, "handle is NULL");
  if (!guarded) return fail(HYDRO_EINVAL, "guarded output buffer is NULL");
  if ((uintptr_t)guarded & 7) return fail(HYDRO_EINVAL, "guarded output buffer must be 8-byte aligned");
  const uintptr_t o0 = (uintptr_t)guarded, o1 = o0 + hydro_guarded_doubles(&g->d) * sizeof(double);
  const size_t sb = hydro_state_doubles(&g->d) * sizeof(double);
  const double* states[3] = {g->d.U, g->d.U_alt, g->U_stage};
  for (const double* st : states) {
    if (!st) continue;
    const uintptr_t s0 = (uintptr_t)st, s1 = s0 + sb;
    if (o0 < s1 && s0 < o1) return fail(HYDRO_EINVAL, "guarded output overlaps a state buffer");
  }
  hipError_t e = hydro::launch_fill_guards(g->d.nxb, g->geom, cur_state(g), guarded, stream_of(g));
  if (e != hipSuccess) return hip_fail(e, "guard-fill kernel launch");
  return HYDRO_OK;
}

int hydro_step(hydro_grid* g, double dt) {
  if (!g) return fail(HYDRO_EINVAL, "handle is NULL");
  if (g->batch) return fail(HYDRO_EINVAL, "grid belongs to a batch; step it through the batch");
  if (!finite_pos(dt)) return fail(HYDRO_EINVAL, "dt must be finite and > 0 (got %g)", dt);
  return do_step(g, dt, 0.0);
}

int hydro_step_cfl(hydro_grid* g, double cfl) {
  if (!g) return fail(HYDRO_EINVAL, "handle is NULL");
  if (g->batch) return fail(HYDRO_EINVAL, "grid belongs to a batch; step it through the batch");
  if (!finite_pos(cfl)) return fail(HYDRO_EINVAL, "cfl must be finite and > 0 (got %g)", cfl);
  int rc = ensure_signal(g);
  if (rc) return rc;
  return do_step(g, 0.0, cfl);
}

int hydro_dt(hydro_grid* g, double cfl, double* dt_out) {
  if (!g || !dt_out) return fail(HYDRO_EINVAL, "handle or dt_out is NULL");
  if (!finite_pos(cfl)) return fail(HYDRO_EINVAL, "cfl must be finite and > 0 (got %g)", cfl);
  int rc = ensure_signal(g);
  if (rc) return rc;
  hydro::WorkHeader h;
  rc = read_header(g, &h);
  if (rc) return rc;
  double s;
  const unsigned long long bits = h.sig[slot_of(g)];
  memcpy(&s, &bits, sizeof s);
  const double dt = cfl / s;
  const bool ok = std::isfinite(s) && s > 0.0 && std::isfinite(dt) && dt > 0.0;
  if (ok) *dt_out = dt;
  if (h.cnt[2] != 0)  // takes precedence: a nonphysical state also spoils the signal speed
    return fail(HYDRO_ENONPHYS, "%llu nonphysical cells produced since init", h.cnt[2]);
  if (!ok) return fail(HYDRO_EINVAL, "maximum signal speed %g is not positive and finite", s);
  return HYDRO_OK;
}

int hydro_last_dt(hydro_grid* g, double* dt_out) {
  if (!g || !dt_out) return fail(HYDRO_EINVAL, "handle or dt_out is NULL");
  if (g->steps == 0) return fail(HYDRO_EINVAL, "no step has been taken");
  hydro::WorkHeader h;
  int rc = read_header(g, &h);
  if (rc) return rc;
  *dt_out = h.dt_last;
  return HYDRO_OK;
}

int hydro_state_changed(hydro_grid* g) {
  if (!g) return fail(HYDRO_EINVAL, "handle is NULL");
  g->sig_valid = false;
  return HYDRO_OK;
}

int hydro_current(hydro_grid* g, double** U_cur) {
  if (!g || !U_cur) return fail(HYDRO_EINVAL, "handle or U_cur is NULL");
  *U_cur = cur_state(g);
  return HYDRO_OK;
}

int hydro_counters(hydro_grid* g, long long out[3]) {
  if (!g || !out) return fail(HYDRO_EINVAL, "handle or out is NULL");
  hydro::WorkHeader h;
  int rc = read_header(g, &h);
  if (rc) return rc;
  for (int c = 0; c < 3; ++c) out[c] = (long long)h.cnt[c];
  return HYDRO_OK;
}

int hydro_free_grid(hydro_grid* g) {
  if (g && g->batch) return fail(HYDRO_EINVAL, "grid belongs to a batch; free the batch first");
  delete g;
  return HYDRO_OK;
}

int hydro_set_buffers(hydro_grid* g, double* U, double* U_alt) {
  if (!g) return fail(HYDRO_EINVAL, "handle is NULL");
  if (g->batch) return fail(HYDRO_EINVAL, "grid belongs to a batch");
  hydro_grid_desc d = g->d;
  d.U = U;
  d.U_alt = U_alt;
  int rc = validate(&d);
  if (rc) return rc;
  const size_t sb = hydro_state_doubles(&d) * sizeof(double);
  if (g->U_stage && (overlaps(g->U_stage, sb, U, sb) || overlaps(g->U_stage, sb, U_alt, sb)))
    return fail(HYDRO_EINVAL, "state buffers overlap the stage buffer");
  g->d.U = U;
  g->d.U_alt = U_alt;
  g->cur = 0;
  return HYDRO_OK;
}

int hydro_set_scheme(hydro_grid* g, int scheme, double* U_stage) {
  if (!g) return fail(HYDRO_EINVAL, "handle is NULL");
  if (g->batch) return fail(HYDRO_EINVAL, "grid belongs to a batch");
  if (scheme != HYDRO_SCHEME_MH && scheme != HYDRO_SCHEME_RK2 && scheme != HYDRO_SCHEME_RK3 && !is_ctu(scheme))
    return fail(HYDRO_EINVAL, "unknown scheme %d", scheme);
  if (scheme == HYDRO_SCHEME_RK3) {
    if (!U_stage) return fail(HYDRO_EINVAL, "the third-order scheme needs a stage buffer");
    if ((uintptr_t)U_stage & 255) return fail(HYDRO_EINVAL, "stage buffer must be 256-byte aligned");
    const size_t sb = hydro_state_doubles(&g->d) * sizeof(double);
    if (overlaps(U_stage, sb, g->d.U, sb) || overlaps(U_stage, sb, g->d.U_alt, sb))
      return fail(HYDRO_EINVAL, "stage buffer overlaps a state buffer");
  } else {
    U_stage = nullptr;
  }
  if (is_ctu(scheme) != is_ctu(g->scheme))
    g->sig_valid = false;  // the kept signal speed follows the other CFL rule
  g->scheme = scheme;
  g->U_stage = U_stage;
  return HYDRO_OK;
}

int hydro_set_pencils(hydro_grid* g, int nseg) {
  if (!g) return fail(HYDRO_EINVAL, "handle is NULL");
  if (nseg != 1 && nseg != 2 && nseg != 4) return fail(HYDRO_EINVAL, "pencils per column must be 1, 2 or 4");
  if (g->d.nxb / nseg < 2) return fail(HYDRO_EINVAL, "pencils shorter than 2 planes");
  g->plen = g->d.nxb / nseg;
  return HYDRO_OK;
}

int hydro_set_tile(hydro_grid* g, int tile) {
  if (!g) return fail(HYDRO_EINVAL, "handle is NULL");
  if (g->batch) return fail(HYDRO_EINVAL, "grid belongs to a batch");
  if (tile != 8 && tile != 16) return fail(HYDRO_EINVAL, "column tiles must be 8x8 or 16x16 (got %d)", tile);
  if (tile > g->d.nxb) return fail(HYDRO_EINVAL, "8^3 blocks take 8x8 column tiles");
  g->tile = tile;
  return HYDRO_OK;
}

int hydro_set_pencil_planes(hydro_grid* g, int planes) {
  if (!g) return fail(HYDRO_EINVAL, "handle is NULL");
  const long nz = (long)g->d.nblk[2] * g->d.nxb;
  if (planes < 2 || planes > nz || nz % planes)
    return fail(HYDRO_EINVAL, "planes per pencil must be >= 2 and divide the %ld planes along z", nz);
  g->plen = planes;
  return HYDRO_OK;
}

// ---- batches ---------------------------------------------------------------

namespace {

constexpr int kMaxPencils = 4;

int default_tile(int nxb) { return nxb == 8 ? 8 : 16; }
int size_class(int nxb) { return nxb == 8 ? 0 : nxb == 16 ? 1 : 2; }

// column tiles of a grid's z layers stepped with tiles of edge `tile`
long columns_of(const hydro_grid* g, int tile) {
  const long per = (long)(g->d.nxb / tile) * (g->d.nxb / tile);
  return (long)g->d.nblk[0] * g->d.nblk[1] * g->d.nblk[2] * per;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct BatchLayout {
  size_t sims, items, total, max_items;
};

BatchLayout batch_layout(hydro_grid* const* grids, int n) {
  BatchLayout L;
  size_t maxi = 0;
  for (int i = 0; i < n; ++i) maxi += (size_t)columns_of(grids[i], 8) * kMaxPencils;
  L.max_items = maxi;
  L.sims = 0;
  L.items = align256(sizeof(hydro::BatchSim) * (size_t)n);
  L.total = L.items + align256(sizeof(hydro::BatchItem) * maxi);
  return L;
}

void drop_graph(hydro_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// Member table and work list of the grids (their current buffer and signal
// slot): one contiguous work-list range per block size (32^3 columns, then
// 16^3, then 8^3), each stepped by its own launch; inactive members get a
// table entry but no items.  Launches the signal-speed reduction on `s` for
// active members whose kept value is stale.
int build_tables(hydro_grid* const* grids, int n, const unsigned char* active, const int nseg[3], const int tile[3],
                 hipStream_t s,
                 std::vector<hydro::BatchSim>& sims, std::vector<hydro::BatchItem>& items, long cls_begin[3],
                 long cls_count[3]) {
  sims.resize(n);
  items.clear();
  for (int cls = 2; cls >= 0; --cls) {
    cls_begin[cls] = (long)items.size();
    for (int i = 0; i < n; ++i) {
      hydro_grid* g = grids[i];
      if (!active[i] || size_class(g->d.nxb) != cls) continue;
      const long cols = columns_of(g, tile[cls]) * nseg[cls];
      for (long c = 0; c < cols; ++c) items.push_back(hydro::BatchItem{i, (int)c});
    }
    cls_count[cls] = (long)items.size() - cls_begin[cls];
  }
  for (int i = 0; i < n; ++i) {
    hydro_grid* g = grids[i];
    hydro::BatchSim& m = sims[i];
    m.U0 = g->d.U;
    m.U1 = g->d.U_alt;
    m.ws = ws_of(g);
    m.geom = g->geom;
    m.nxb = g->d.nxb;
    m.parity0 = g->cur;
    m.slot0 = slot_of(g);
    m.pad = 0;
    if (active[i]) {
      int rc = ensure_signal_on(g, s);
      if (rc) return rc;
    }
  }
  return HYDRO_OK;
}

// Rebuild the member table and the work list from the grid handles and
// upload both.
int batch_upload(hydro_batch* b) {
  hipStream_t s = (hipStream_t)b->stream;
  const int n = (int)b->grids.size();
  int rc = build_tables(b->grids.data(), n, b->active.data(), b->nseg, b->tile, s, b->sims, b->items, b->cls_begin,
                        b->cls_count);
  if (rc) return rc;
  hipError_t e = hipMemcpyAsync(b->d_sims, b->sims.data(), sizeof(hydro::BatchSim) * n, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !b->items.empty())
    e = hipMemcpyAsync(b->d_items, b->items.data(), sizeof(hydro::BatchItem) * b->items.size(),
                       hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "batch table upload");
  b->step = 0;
  b->dirty = false;
  drop_graph(b);
  return HYDRO_OK;
}

// One launch per block-size class present, each running the kernel that
// holds that size's tile step only (the classes' work-list ranges are
// disjoint and every member sits in one class, so the launches are
// independent; the stream orders them).
hipError_t class_launches(const hydro::BatchSim* d_sims, const hydro::BatchItem* d_items, const long cls_begin[3],
                          const long cls_count[3], const int nseg[3], const int tile[3], int grid, double cfl,
                          long step, hipStream_t s) {
  for (int cls = 2; cls >= 0; --cls) {
    if (cls_count[cls] == 0) continue;
    hipError_t e = hydro::launch_batch_step(d_sims, d_items + cls_begin[cls], (int)cls_count[cls], step % 6, cfl,
                                            8 << cls, tile[cls], nseg[cls], grid, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t batch_launch(hydro_batch* b, double cfl, long step) {
  return class_launches(b->d_sims, b->d_items, b->cls_begin, b->cls_count, b->nseg, b->tile, b->grid, cfl, step,
                        (hipStream_t)b->stream);
}

void advance_members(hydro_batch* b, int nsteps) {
  for (size_t i = 0; i < b->grids.size(); ++i) {
    if (!b->active[i]) continue;
    hydro_grid* g = b->grids[i];
    g->cur ^= (nsteps & 1);
    g->steps += (unsigned long long)nsteps;
    g->sig_valid = true;
  }
}

}  // namespace

size_t hydro_batch_work_bytes(hydro_grid* const* grids, int n) {
  if (!grids || n <= 0) return 0;
  for (int i = 0; i < n; ++i)
    if (!grids[i]) return 0;
  return batch_layout(grids, n).total;
}

int hydro_batch_create(hydro_grid* const* grids, int n, void* work, size_t work_bytes, void* stream,
                       hydro_batch** out) {
  if (!out) return fail(HYDRO_EINVAL, "out is NULL");
  *out = nullptr;
  if (!grids || n <= 0) return fail(HYDRO_EINVAL, "a batch needs at least one grid");
  for (int i = 0; i < n; ++i) {
    if (!grids[i]) return fail(HYDRO_EINVAL, "grid %d is NULL", i);
    if (grids[i]->batch) return fail(HYDRO_EINVAL, "grid %d already belongs to a batch", i);
    if (grids[i]->scheme != HYDRO_SCHEME_MH)
      return fail(HYDRO_EINVAL, "grid %d uses a Runge-Kutta scheme; batches take predictor-corrector grids", i);
    for (int k = 0; k < i; ++k)
      if (grids[k] == grids[i]) return fail(HYDRO_EINVAL, "grid %d appears twice", i);
  }
  if (!work || ((uintptr_t)work & 255)) return fail(HYDRO_EINVAL, "batch workspace must be non-NULL and 256-byte aligned");
  const BatchLayout L = batch_layout(grids, n);
  if (L.max_items > (size_t)0x7fffffff) return fail(HYDRO_EINVAL, "batch too large");
  if (work_bytes < L.total) return fail(HYDRO_ESIZE, "batch workspace has %zu bytes, needs %zu", work_bytes, L.total);
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "device query");
  hydro_batch* b = new (std::nothrow) hydro_batch;
  if (!b) return fail(HYDRO_EINVAL, "out of host memory");
  b->grids.assign(grids, grids + n);
  b->active.assign(n, 1);
  b->d_sims = (hydro::BatchSim*)((char*)work + L.sims);
  b->d_items = (hydro::BatchItem*)((char*)work + L.items);
  b->max_items = L.max_items;
  b->stream = stream;
  b->nseg[0] = b->nseg[1] = b->nseg[2] = 1;
  b->tile[0] = 8;
  b->tile[1] = b->tile[2] = 16;
  b->cus = cus;
  b->grid = 2 * cus;
  for (int c = 0; c < 3; ++c) b->cls_begin[c] = b->cls_count[c] = 0;
  b->step = 0;
  b->dirty = true;
  b->use_graph = false;
  b->graph = nullptr;
  b->exec = nullptr;
  for (int i = 0; i < n; ++i) grids[i]->batch = b;
  *out = b;
  return HYDRO_OK;
}

int hydro_batch_set_active(hydro_batch* b, const unsigned char* mask) {
  if (!b || !mask) return fail(HYDRO_EINVAL, "batch or mask is NULL");
  for (size_t i = 0; i < b->grids.size(); ++i) b->active[i] = mask[i] ? 1 : 0;
  b->dirty = true;
  return HYDRO_OK;
}

int hydro_batch_set_pencils(hydro_batch* b, const int nseg[3]) {
  if (!b || !nseg) return fail(HYDRO_EINVAL, "batch or nseg is NULL");
  const int sizes[3] = {8, 16, 32};
  for (int c = 0; c < 3; ++c) {
    if (nseg[c] != 1 && nseg[c] != 2 && nseg[c] != 4) return fail(HYDRO_EINVAL, "pencils per column must be 1, 2 or 4");
    if (sizes[c] / nseg[c] < 2) return fail(HYDRO_EINVAL, "pencils shorter than 2 planes");
  }
  for (int c = 0; c < 3; ++c) b->nseg[c] = nseg[c];
  b->dirty = true;
  return HYDRO_OK;
}

int hydro_batch_set_tiles(hydro_batch* b, const int tile[3]) {
  if (!b || !tile) return fail(HYDRO_EINVAL, "batch or tile is NULL");
  if (tile[0] != 8) return fail(HYDRO_EINVAL, "8^3 blocks take 8x8 column tiles");
  for (int c = 1; c < 3; ++c)
    if (tile[c] != 8 && tile[c] != 16) return fail(HYDRO_EINVAL, "column tiles must be 8x8 or 16x16");
  for (int c = 0; c < 3; ++c) b->tile[c] = tile[c];
  b->dirty = true;
  return HYDRO_OK;
}

int hydro_batch_set_workgroups(hydro_batch* b, int per_cu) {
  if (!b) return fail(HYDRO_EINVAL, "batch is NULL");
  if (per_cu < 1 || per_cu > 8) return fail(HYDRO_EINVAL, "workgroups per CU must be 1..8");
  b->grid = per_cu * b->cus;
  drop_graph(b);
  return HYDRO_OK;
}

int hydro_batch_use_graph(hydro_batch* b, int enable) {
  if (!b) return fail(HYDRO_EINVAL, "batch is NULL");
  b->use_graph = enable != 0;
  if (!b->use_graph) drop_graph(b);
  return HYDRO_OK;
}

int hydro_batch_step(hydro_batch* b, double cfl, int nsteps) {
  if (!b) return fail(HYDRO_EINVAL, "batch is NULL");
  if (!finite_pos(cfl)) return fail(HYDRO_EINVAL, "cfl must be finite and > 0 (got %g)", cfl);
  if (nsteps < 0) return fail(HYDRO_EINVAL, "nsteps must be >= 0");
  if (b->dirty) {
    int rc = batch_upload(b);
    if (rc) return rc;
  }
  if (b->items.empty() || nsteps == 0) return HYDRO_OK;
  hipStream_t s = (hipStream_t)b->stream;
  int done = 0;
  while (done < nsteps) {
    const bool aligned = (b->step % 6) == 0;
    if (b->use_graph && aligned && nsteps - done >= 6) {
      if (!b->exec) {
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        for (int k = 0; k < 6 && e == hipSuccess; ++k) e = batch_launch(b, cfl, k);
        hipGraph_t gr = nullptr;
        hipError_t e2 = hipStreamEndCapture(s, &gr);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, gr, nullptr, nullptr, 0);
        if (e != hipSuccess) {
          if (gr) (void)hipGraphDestroy(gr);
          b->exec = nullptr;
          return hip_fail(e, "batch graph capture");
        }
        b->graph = gr;
        b->graph_cfl = cfl;
      }
      if (b->graph_cfl != cfl) {
        drop_graph(b);
        continue;
      }
      hipError_t e = hipGraphLaunch(b->exec, s);
      if (e != hipSuccess) return hip_fail(e, "batch graph launch");
      b->step += 6;
      done += 6;
      advance_members(b, 6);
      continue;
    }
    hipError_t e = batch_launch(b, cfl, b->step);
    if (e != hipSuccess) return hip_fail(e, "batch step launch");
    b->step += 1;
    done += 1;
    advance_members(b, 1);
  }
  return HYDRO_OK;
}

int hydro_batch_dts(hydro_batch* b, double* dt_out) {
  if (!b || !dt_out) return fail(HYDRO_EINVAL, "batch or dt_out is NULL");
  hipError_t e = hipStreamSynchronize((hipStream_t)b->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  for (size_t i = 0; i < b->grids.size(); ++i) {
    hydro::WorkHeader h;
    e = hipMemcpy(&h, b->grids[i]->d.work, sizeof h, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy (member header)");
    dt_out[i] = h.dt_last;
  }
  return HYDRO_OK;
}

int hydro_batch_free(hydro_batch* b) {
  if (!b) return HYDRO_OK;
  drop_graph(b);
  for (hydro_grid* g : b->grids) g->batch = nullptr;
  delete b;
  return HYDRO_OK;
}

int hydro_batch_step_static(hydro_grid* const* grids, int n, const int nseg[3], double cfl, int nsteps,
                            void* stream) {
  if (n > (int)hydro::kStaticMaxGrids)
    return fail(HYDRO_ESIZE, "%d grids exceed the static scratch's %zu", n, hydro::kStaticMaxGrids);
  if (!grids || n <= 0) return fail(HYDRO_EINVAL, "a batch needs at least one grid");
  if (!finite_pos(cfl)) return fail(HYDRO_EINVAL, "cfl must be finite and > 0 (got %g)", cfl);
  if (nsteps < 0) return fail(HYDRO_EINVAL, "nsteps must be >= 0");
  int segs[3] = {1, 1, 1};
  const int tiles[3] = {8, 16, 16};
  if (nseg) {
    const int sizes[3] = {8, 16, 32};
    for (int c = 0; c < 3; ++c) {
      if (nseg[c] != 1 && nseg[c] != 2 && nseg[c] != 4)
        return fail(HYDRO_EINVAL, "pencils per column must be 1, 2 or 4");
      if (sizes[c] / nseg[c] < 2) return fail(HYDRO_EINVAL, "pencils shorter than 2 planes");
      segs[c] = nseg[c];
    }
  }
  // duplicates: each call stamps its grids with its own id (linear in n;
  // no host allocation)
  static std::atomic<unsigned long long> calls{0};
  const unsigned long long id = ++calls;
  size_t nitems = 0;
  for (int i = 0; i < n; ++i) {
    if (!grids[i]) return fail(HYDRO_EINVAL, "grid %d is NULL", i);
    if (grids[i]->batch) return fail(HYDRO_EINVAL, "grid %d belongs to a batch", i);
    if (grids[i]->scheme != HYDRO_SCHEME_MH)
      return fail(HYDRO_EINVAL, "grid %d does not use the predictor-corrector scheme", i);
    if (grids[i]->mark == id) return fail(HYDRO_EINVAL, "grid %d appears twice", i);
    grids[i]->mark = id;
    nitems += (size_t)columns_of(grids[i], tiles[size_class(grids[i]->d.nxb)]) * segs[size_class(grids[i]->d.nxb)];
  }
  if (nitems > hydro::kStaticMaxItems)
    return fail(HYDRO_ESIZE, "%zu work items exceed the static scratch's %zu", nitems, hydro::kStaticMaxItems);
  if (nsteps == 0) return HYDRO_OK;
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "device query");
  void* base = nullptr;
  e = hydro::static_scratch(&base);
  if (e != hipSuccess) return hip_fail(e, "static scratch lookup");
  hipStream_t s = (hipStream_t)stream;
  // host copies of the tables stay alive until the next call on this thread
  // (their storage only grows)
  thread_local std::vector<hydro::BatchSim> sims;
  thread_local std::vector<hydro::BatchItem> items;
  thread_local std::vector<unsigned char> active;
  long cls_begin[3], cls_count[3];
  active.assign(n, 1);
  int rc = build_tables(grids, n, active.data(), segs, tiles, s, sims, items, cls_begin, cls_count);
  if (rc) return rc;
  auto* d_sims = (hydro::BatchSim*)base;
  auto* d_items = (hydro::BatchItem*)((char*)base + hydro::kStaticSimsBytes);
  e = hipMemcpyAsync(d_sims, sims.data(), sizeof(hydro::BatchSim) * n, hipMemcpyHostToDevice, s);
  if (e == hipSuccess && !items.empty())
    e = hipMemcpyAsync(d_items, items.data(), sizeof(hydro::BatchItem) * items.size(), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "static table upload");
  for (int k = 0; k < nsteps; ++k) {
    e = class_launches(d_sims, d_items, cls_begin, cls_count, segs, tiles, 2 * cus, cfl, k, s);
    if (e != hipSuccess) return hip_fail(e, "batch step launch");
  }
  for (int i = 0; i < n; ++i) {
    hydro_grid* g = grids[i];
    g->cur ^= (nsteps & 1);
    g->steps += (unsigned long long)nsteps;
    g->sig_valid = true;
  }
  return HYDRO_OK;
}

int hydro_copy_probe(const double* src, double* dst, size_t n, void* stream) {
  if (n == 0) return HYDRO_OK;
  if (!src || !dst) return fail(HYDRO_EINVAL, "copy probe buffers must be non-NULL");
  if (((uintptr_t)src | (uintptr_t)dst) & 15) return fail(HYDRO_EINVAL, "copy probe buffers must be 16-byte aligned");
  const uintptr_t s0 = (uintptr_t)src, d0 = (uintptr_t)dst, b = n * sizeof(double);
  if (s0 < d0 + b && d0 < s0 + b) return fail(HYDRO_EINVAL, "copy probe buffers overlap");
  if (n > (size_t)1 << 40) return fail(HYDRO_EINVAL, "copy probe size too large");
  hipError_t e = hydro::launch_copy(src, dst, (long)n, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "copy kernel launch");
  return HYDRO_OK;
}

const char* hydro_last_error(void) { return g_err; }

}  // extern "C"

// ---- block-structured AMR ---------------------------------------------------

struct hydro_amr {
  hydro_amr_desc d;
  hydro::AmrLaunch L;
  std::vector<unsigned char> refine;       // level-0 flags
  std::vector<unsigned char> refine_deep;  // flags of levels >= 1
  long steps = 0;          // signal slot of the current state: steps % 3
  bool sig_valid = false;  // the slot holds the current state's signal speed
  double* E2 = nullptr;    // device, nroot refinement indicators
  double* E2T = nullptr;   // device, one indicator per block of every level (leaves written)
  std::vector<std::vector<int>> pos;  // host copy of the block positions per level (x, y, z)
  // what rebuilds the leaf steps' column tables (hydro_amr_set_columns)
  struct Cols {
    long nb[3];
    std::vector<int> lookup, plain, rx;
    std::vector<int> face;  // blocks whose views the fine-coarse face fluxes read
    int* d_plain;  // device column tables, room for one column per block
    int* d_rx;
    int* d_zneed;  // device, one entry per block
  };
  std::vector<Cols> cols;
  long tpb = 1, slots = 1;  // column tiles per block; leaf-step workgroup slots of the device
};

namespace {

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct AmrLevelHost {
  long nb[3];
  std::vector<int> pos;  // 4 ints per block
  std::vector<unsigned char> flag;
  std::vector<int> lookup, parent, child_base, refined, leaves, leaf_plain, rx_blocks, reflux, first;
  std::vector<int> roct;  // restriction octants the pass takes (8 r + c)
  size_t o_pos, o_reflux, o_lookup, o_parent, o_child, o_refined, o_leaves, o_plain, o_rx, o_first;  // int offsets
  size_t o_roct;
  size_t o_cplain, o_crx;  // int offsets of the column tables (room for one column per block)
  size_t o_zneed;          // int offset of the halo-plane table (one per block)
  size_t o_G, o_flux;                                                                                 // bytes
};

struct AmrLayout {
  int nlev = 0;
  AmrLevelHost lev[hydro::AMR_MAX_LEVELS];
  long nroot = 0, nfine = 0;
  size_t tab_ints = 0, o_tab = 256, o_E2 = 0, o_E2T = 0, total = 0;
};

// block index at level-l position (x, y, z) after the boundary map; -1 when
// absent, -2 beyond an outflow boundary
long level_block(const AmrLevelHost& L, const int* bc, long x, long y, long z) {
  long p[3] = {x, y, z};
  for (int d = 0; d < 3; ++d) {
    if (bc[d] == HYDRO_BC_PERIODIC) p[d] = ((p[d] % L.nb[d]) + L.nb[d]) % L.nb[d];
    else if (p[d] < 0 || p[d] >= L.nb[d]) return -2;
  }
  return L.lookup[p[0] + L.nb[0] * (p[1] + L.nb[1] * p[2])];
}

// The blocks of `list` (one level) as columns of up to `cap` blocks stacked
// in z at consecutive positions (no wrap), bottom first, 4 ints per column
// (-1 for unused entries); every block of the list is in exactly one.
std::vector<int> amr_columns(const long nb[3], const std::vector<int>& lookup, const std::vector<int>& pos,
                             const std::vector<int>& list, int cap) {
  std::vector<unsigned char> in(pos.size() / 4, 0);
  for (int b : list) in[b] = 1;
  auto at = [&](long x, long y, long z) -> int {
    if (z < 0 || z >= nb[2]) return -1;
    const int b = lookup[x + nb[0] * (y + nb[1] * z)];
    return (b >= 0 && in[b]) ? b : -1;
  };
  std::vector<int> out;
  for (int b : list) {
    const long x = pos[4 * b], y = pos[4 * b + 1], z = pos[4 * b + 2];
    if (at(x, y, z - 1) >= 0) continue;  // not the bottom of its run
    long zz = z;
    int cur = b;
    while (cur >= 0) {
      int col[4] = {-1, -1, -1, -1};
      for (int m = 0; m < cap && cur >= 0; ++m) {
        col[m] = cur;
        cur = at(x, y, ++zz);
      }
      out.insert(out.end(), col, col + 4);
    }
  }
  return out;
}

// Blocks of each level whose leaf views the fine-coarse face fluxes read
// (every halo plane): the leaves next to a refined block of their level,
// and that block's children on the face toward them (the face flux
// kernel's parts 0 and 1..4).
std::vector<std::vector<int>> amr_face_blocks(const AmrLayout& A);

// The whole halo planes each block's fill writes (bit 0: planes -2, -1;
// bit 1: planes n, n+1): below the bottom block of each column and above
// its top block, the only ones a column's pencil reads, and every plane
// for the blocks in `face`.
std::vector<int> amr_zneed(size_t nblk, const std::vector<int>& cp, const std::vector<int>& cr,
                           const std::vector<int>& face) {
  std::vector<int> z(nblk, 0);
  for (const std::vector<int>* c : {&cp, &cr})
    for (size_t i = 0; i + 3 < c->size(); i += 4) {
      int top = (*c)[i];
      for (int m = 1; m < 4; ++m)
        if ((*c)[i + m] >= 0) top = (*c)[i + m];
      z[(*c)[i]] |= 1;
      z[top] |= 2;
    }
  for (int b : face) z[b] = 3;
  return z;
}

// Longest column of a column table (blocks).
int amr_kmax(const std::vector<int>& cols) {
  int k = 0;
  for (size_t i = 0; i + 3 < cols.size(); i += 4)
    k = std::max(k, 1 + (cols[i + 1] >= 0) + (cols[i + 2] >= 0) + (cols[i + 3] >= 0));
  return k;
}

// Column length for a leaf list: `cap` when it is 1, 2 or 4, else (0) the
// one whose tiles, dealt in order to `slots` workgroup slots (each tile of
// a column of k blocks costs k*N + 3 planes: the pencil and its z halo),
// finish first; ties go to shorter columns (more workgroups).
std::vector<int> amr_best_columns(const long nb[3], const std::vector<int>& lookup, const std::vector<int>& pos,
                                  const std::vector<int>& list, int N, long tpb, long slots, int cap0) {
  std::vector<int> best;
  long best_t = -1;
  for (int cap : {1, 2, 4}) {
    if (cap0 && cap != cap0) continue;
    std::vector<int> c = amr_columns(nb, lookup, pos, list, cap);
    std::priority_queue<long, std::vector<long>, std::greater<long>> q;
    for (long i = 0; i < slots; ++i) q.push(0);
    long t = 0;
    for (size_t i = 0; i < c.size(); i += 4) {
      const long k = 1 + (c[i + 1] >= 0) + (c[i + 2] >= 0) + (c[i + 3] >= 0);
      for (long r = 0; r < tpb; ++r) {
        const long f = q.top() + k * N + 3;
        q.pop();
        q.push(f);
        t = std::max(t, f);
      }
    }
    if (best_t < 0 || t < best_t) {
      best_t = t;
      best = std::move(c);
    }
  }
  return best;
}

int amr_layout(const hydro_amr_desc* d, AmrLayout& A) {
  if (!d) return fail(HYDRO_EINVAL, "descriptor is NULL");
  if (d->nxb != 8 && d->nxb != 16 && d->nxb != 32) return fail(HYDRO_EINVAL, "nxb must be 8, 16 or 32");
  if (d->nguard != HYDRO_NGUARD) return fail(HYDRO_EINVAL, "nguard must be %d", HYDRO_NGUARD);
  for (int a = 0; a < 3; ++a) {
    if (d->nblk[a] < 1) return fail(HYDRO_EINVAL, "nblk[%d] must be >= 1", a);
    if (!(std::isfinite(d->lo[a]) && std::isfinite(d->hi[a]) && d->hi[a] > d->lo[a]))
      return fail(HYDRO_EINVAL, "domain axis %d needs finite lo < hi", a);
    if (d->bc[a] != HYDRO_BC_PERIODIC && d->bc[a] != HYDRO_BC_OUTFLOW) return fail(HYDRO_EINVAL, "bad bc[%d]", a);
  }
  if (!(std::isfinite(d->gamma) && d->gamma > 1.0)) return fail(HYDRO_EINVAL, "gamma must be finite and > 1");
  if (!d->refine) return fail(HYDRO_EINVAL, "refine flags are NULL");
  if (d->nrefine_deep && !d->refine_deep) return fail(HYDRO_EINVAL, "refine_deep is NULL");
  const int N = d->nxb;
  A.nroot = (long)d->nblk[0] * d->nblk[1] * d->nblk[2];
  if (A.nroot > (1L << 24)) return fail(HYDRO_EINVAL, "too many root blocks");
  // levels: positions, flags, children
  size_t used_deep = 0;
  for (int l = 0;; ++l) {
    if (l == hydro::AMR_MAX_LEVELS) return fail(HYDRO_EINVAL, "more than %d levels", hydro::AMR_MAX_LEVELS);
    AmrLevelHost& L = A.lev[l];
    for (int ax = 0; ax < 3; ++ax) L.nb[ax] = (long)d->nblk[ax] << l;
    if (l == 0) {
      L.pos.resize(4 * A.nroot);
      for (long b = 0; b < A.nroot; ++b) {
        L.pos[4 * b] = (int)(b % d->nblk[0]);
        L.pos[4 * b + 1] = (int)((b / d->nblk[0]) % d->nblk[1]);
        L.pos[4 * b + 2] = (int)(b / ((long)d->nblk[0] * d->nblk[1]));
        L.pos[4 * b + 3] = 0;
      }
      L.parent.assign(A.nroot, -1);
      L.flag.assign(d->refine, d->refine + A.nroot);
    } else {
      const AmrLevelHost& P = A.lev[l - 1];
      L.pos.clear();
      L.parent.clear();
      for (int r : P.refined)
        for (int c = 0; c < 8; ++c) {
          L.pos.insert(L.pos.end(), {2 * P.pos[4 * r] + (c & 1), 2 * P.pos[4 * r + 1] + ((c >> 1) & 1),
                                     2 * P.pos[4 * r + 2] + ((c >> 2) & 1), 0});
          L.parent.push_back(r);
        }
      const long nblk = (long)L.parent.size();
      if (used_deep < d->nrefine_deep) {
        if (d->nrefine_deep - used_deep < (size_t)nblk)
          return fail(HYDRO_EINVAL, "refine_deep ends inside level %d (%zu of %ld flags left)", l,
                      d->nrefine_deep - used_deep, nblk);
        L.flag.assign(d->refine_deep + used_deep, d->refine_deep + used_deep + nblk);
        used_deep += (size_t)nblk;
      } else {
        L.flag.assign(nblk, 0);
      }
    }
    const long nblk = (long)L.flag.size();
    const long ncells = L.nb[0] * L.nb[1] * L.nb[2];
    if (ncells > (1L << 28)) return fail(HYDRO_EINVAL, "level %d is too fine for its lookup table", l);
    L.lookup.assign(ncells, -1);
    for (long b = 0; b < nblk; ++b)
      L.lookup[L.pos[4 * b] + L.nb[0] * (L.pos[4 * b + 1] + L.nb[1] * (long)L.pos[4 * b + 2])] = (int)b;
    L.child_base.assign(nblk, -1);
    L.refined.clear();
    L.leaves.clear();
    for (long b = 0; b < nblk; ++b) {
      if (L.flag[b]) {
        L.child_base[b] = (int)(8 * L.refined.size());
        L.refined.push_back((int)b);
      } else {
        L.leaves.push_back((int)b);
      }
    }
    if (l > 0) A.nfine += nblk;
    A.nlev = l + 1;
    if (L.refined.empty()) break;
  }
  if (used_deep != d->nrefine_deep)
    return fail(HYDRO_EINVAL, "refine_deep has %zu flags, the levels use %zu", d->nrefine_deep, used_deep);
  // nesting: every refined block of a level >= 1 has its 26 neighbours at its level
  for (int l = 1; l < A.nlev; ++l) {
    const AmrLevelHost& L = A.lev[l];
    for (int r : L.refined)
      for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx)
            if (level_block(L, d->bc, L.pos[4 * r] + dx, L.pos[4 * r + 1] + dy, L.pos[4 * r + 2] + dz) == -1)
              return fail(HYDRO_EINVAL, "refined block %d of level %d lacks a neighbour at its level", r, l);
  }
  // reflux entries: leaves next to a refined block of their level, grouped per leaf
  for (int l = 0; l < A.nlev; ++l) {
    AmrLevelHost& L = A.lev[l];
    L.reflux.clear();
    L.first.assign(1, 0);
    L.leaf_plain.clear();
    L.rx_blocks.clear();
    for (int b : L.leaves) {
      for (int dd = 0; dd < 3; ++dd)
        for (int side = 0; side < 2; ++side) {
          long p[3] = {L.pos[4 * b], L.pos[4 * b + 1], L.pos[4 * b + 2]};
          p[dd] += side ? 1 : -1;
          const long nbr = level_block(L, d->bc, p[0], p[1], p[2]);
          if (nbr < 0 || !L.flag[nbr]) continue;
          L.reflux.insert(L.reflux.end(), {b, dd, side, (int)nbr});
        }
      if ((int)L.reflux.size() / 4 > L.first.back()) {
        L.first.push_back((int)L.reflux.size() / 4);
        L.rx_blocks.push_back(b);
      } else {
        L.leaf_plain.push_back(b);
      }
    }
  }
  // octants of the refined blocks left to the restriction pass: those whose
  // child is refined or takes refluxing (a plain leaf's step writes the
  // mean of its new state into its parent octant itself)
  for (int l = 0; l + 1 < A.nlev; ++l) {
    AmrLevelHost& L = A.lev[l];
    const AmrLevelHost& F = A.lev[l + 1];
    std::vector<unsigned char> rx(F.flag.size(), 0);
    for (int b : F.rx_blocks) rx[b] = 1;
    L.roct.clear();
    for (int r : L.refined)
      for (int c = 0; c < 8; ++c) {
        const int ch = L.child_base[r] + c;
        if (F.flag[ch] || rx[ch]) L.roct.push_back(8 * r + c);
      }
  }
  // table (ints): int4 arrays first (16-byte aligned), then the int arrays
  size_t t = 0;
  auto take = [&](size_t nints) {
    const size_t o = t;
    t += (nints + 3) & ~(size_t)3;
    return o;
  };
  for (int l = 0; l < A.nlev; ++l) {
    AmrLevelHost& L = A.lev[l];
    L.o_pos = take(L.pos.size());
    L.o_reflux = take(L.reflux.size());
    L.o_cplain = take(4 * L.leaf_plain.size());
    L.o_crx = take(4 * L.rx_blocks.size());
  }
  for (int l = 0; l < A.nlev; ++l) {
    A.lev[l].o_zneed = take(A.lev[l].flag.size());
    A.lev[l].o_roct = take(A.lev[l].roct.size());
  }
  for (int l = 0; l < A.nlev; ++l) {
    AmrLevelHost& L = A.lev[l];
    L.o_lookup = take(L.lookup.size());
    L.o_parent = take(L.parent.size());
    L.o_child = take(L.child_base.size());
    L.o_refined = take(L.refined.size());
    L.o_leaves = take(L.leaves.size());
    L.o_plain = take(L.leaf_plain.size());
    L.o_rx = take(L.rx_blocks.size());
    L.o_first = take(L.first.size());
  }
  A.tab_ints = t;
  size_t o = A.o_tab + al256(sizeof(int) * t);
  for (int l = 0; l < A.nlev; ++l) {
    AmrLevelHost& L = A.lev[l];
    const size_t nblk = L.flag.size();
    L.o_G = o;
    o += al256(sizeof(double) * hydro::amr_view_doubles(N) * nblk);
    L.o_flux = o;
    o += al256(sizeof(double) * 30 * (size_t)N * N * nblk);
  }
  A.o_E2 = o;
  o += al256(sizeof(double) * (size_t)A.nroot);
  A.o_E2T = o;
  size_t nall = 0;
  for (int l = 0; l < A.nlev; ++l) nall += A.lev[l].flag.size();
  A.total = o + al256(sizeof(double) * nall);
  return HYDRO_OK;
}

std::vector<std::vector<int>> amr_face_blocks(const AmrLayout& A) {
  std::vector<std::vector<int>> out(A.nlev);
  for (int l = 0; l < A.nlev; ++l) {
    const AmrLevelHost& L = A.lev[l];
    for (size_t e = 0; e + 3 < L.reflux.size(); e += 4) {
      const int b = L.reflux[e], d = L.reflux[e + 1], side = L.reflux[e + 2], r = L.reflux[e + 3];
      out[l].push_back(b);
      if (l + 1 >= A.nlev) continue;  // (a refined block always has a level below it)
      const int t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
      for (int c = 0; c < 4; ++c) {
        int co[3];
        co[d] = side ? 0 : 1;
        co[t0] = c & 1;
        co[t1] = c >> 1;
        out[l + 1].push_back(L.child_base[r] + co[0] + 2 * co[1] + 4 * co[2]);
      }
    }
  }
  return out;
}

}  // namespace

extern "C" {

size_t hydro_amr_fine_blocks(const hydro_amr_desc* d) {
  AmrLayout A;
  if (amr_layout(d, A)) return 0;
  return (size_t)A.nfine;
}

int hydro_amr_levels(const hydro_amr_desc* d, long nblocks[8]) {
  if (!nblocks) return fail(HYDRO_EINVAL, "nblocks is NULL");
  AmrLayout A;
  int rc = amr_layout(d, A);
  if (rc) return rc;
  for (int l = 0; l < 8; ++l) nblocks[l] = l < A.nlev ? (long)A.lev[l].flag.size() : 0;
  return A.nlev;
}

size_t hydro_amr_work_bytes(const hydro_amr_desc* d) {
  AmrLayout A;
  if (amr_layout(d, A)) return 0;
  return A.total;
}

int hydro_amr_create(const hydro_amr_desc* d, hydro_amr** out) {
  if (!out) return fail(HYDRO_EINVAL, "out is NULL");
  *out = nullptr;
  AmrLayout A;
  int rc = amr_layout(d, A);
  if (rc) return rc;
  if (!d->Ur || (A.nfine && !d->Uf)) return fail(HYDRO_EINVAL, "state buffers must be non-NULL");
  if (!d->work || ((uintptr_t)d->work & 255)) return fail(HYDRO_EINVAL, "workspace must be non-NULL and 256-byte aligned");
  if (d->work_bytes < A.total) return fail(HYDRO_ESIZE, "AMR workspace has %zu bytes, needs %zu", d->work_bytes, A.total);
  rc = check_device();
  if (rc) return rc;
  hydro_amr* a = new (std::nothrow) hydro_amr;
  if (!a) return fail(HYDRO_EINVAL, "out of host memory");
  a->d = *d;
  a->refine.assign(d->refine, d->refine + A.nroot);
  a->d.refine = a->refine.data();
  a->refine_deep.assign(d->refine_deep, d->refine_deep + d->nrefine_deep);
  a->d.refine_deep = a->refine_deep.data();
  hydro::AmrLaunch& L = a->L;
  const int N = d->nxb;
  int dev = 0, cus = 0;
  hipError_t qe = hipGetDevice(&dev);
  if (qe == hipSuccess) qe = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (qe != hipSuccess) {
    delete a;
    return hip_fail(qe, "device query");
  }
  // leaf-step workgroups resident per CU: two of 256 threads (16x16 tiles), four of 128 (8x8)
  const long tpb = N == 32 ? 4 : 1, slots = (long)cus * (N == 8 ? 4 : 2);
  a->tpb = tpb;
  a->slots = slots;
  char* w = (char*)d->work;
  int* tab = (int*)(w + A.o_tab);
  std::vector<int> host(A.tab_ints, 0);
  L.nlev = A.nlev;
  size_t fine_off = 0;
  const std::vector<std::vector<int>> face = amr_face_blocks(A);
  for (int l = 0; l < A.nlev; ++l) {
    const AmrLevelHost& H = A.lev[l];
    hydro::AmrLevel& V = L.lev[l];
    for (int ax = 0; ax < 3; ++ax) {
      V.g.nb[ax] = (int)H.nb[ax];
      V.g.bc[ax] = d->bc[ax];
      V.g.inv_dx[ax] = ((double)d->nblk[ax] * N) / (d->hi[ax] - d->lo[ax]) * (double)(1L << l);
    }
    V.g.gamma = d->gamma;
    V.g.small_p = d->small_p;
    const long nblk = (long)H.flag.size();
    V.U = l == 0 ? d->Ur : d->Uf + fine_off * 5 * (size_t)N * N * N;
    if (l > 0) fine_off += (size_t)nblk;
    V.G = (double*)(w + H.o_G);
    V.flux = (double*)(w + H.o_flux);
    auto put = [&](size_t o, const std::vector<int>& v) { std::copy(v.begin(), v.end(), host.begin() + o); };
    put(H.o_pos, H.pos);
    put(H.o_reflux, H.reflux);
    put(H.o_lookup, H.lookup);
    put(H.o_parent, H.parent);
    put(H.o_child, H.child_base);
    put(H.o_refined, H.refined);
    put(H.o_leaves, H.leaves);
    put(H.o_plain, H.leaf_plain);
    put(H.o_rx, H.rx_blocks);
    put(H.o_first, H.first);
    const std::vector<int> cplain = amr_best_columns(H.nb, H.lookup, H.pos, H.leaf_plain, N, tpb, slots, 0);
    const std::vector<int> crx = amr_best_columns(H.nb, H.lookup, H.pos, H.rx_blocks, N, tpb, slots, 0);
    put(H.o_cplain, cplain);
    put(H.o_crx, crx);
    put(H.o_zneed, amr_zneed((size_t)nblk, cplain, crx, face[l]));
    a->cols.push_back(hydro_amr::Cols{{H.nb[0], H.nb[1], H.nb[2]}, H.lookup, H.leaf_plain, H.rx_blocks, face[l],
                                      tab + H.o_cplain, tab + H.o_crx, tab + H.o_zneed});
    V.zneed = tab + H.o_zneed;
    put(H.o_roct, H.roct);
    V.roct = tab + H.o_roct;
    V.nroct = (long)H.roct.size();
    V.cols_plain = (const int4*)(tab + H.o_cplain);
    V.cols_rx = (const int4*)(tab + H.o_crx);
    V.ncols_plain = (long)cplain.size() / 4;
    V.ncols_rx = (long)crx.size() / 4;
    V.kmax_plain = amr_kmax(cplain);
    V.kmax_rx = amr_kmax(crx);
    V.pos = (const int4*)(tab + H.o_pos);
    V.reflux = (const int4*)(tab + H.o_reflux);
    V.lookup = tab + H.o_lookup;
    V.parent = tab + H.o_parent;
    V.child_base = tab + H.o_child;
    V.refined = tab + H.o_refined;
    V.leaves = tab + H.o_leaves;
    V.leaf_plain = tab + H.o_plain;
    V.rx_blocks = tab + H.o_rx;
    V.reflux_first = tab + H.o_first;
    V.nblk = nblk;
    V.nrefined = (long)H.refined.size();
    V.nleaves = (long)H.leaves.size();
    V.nleaf_plain = (long)H.leaf_plain.size();
    V.nreflux = (long)H.reflux.size() / 4;
    V.ngroups = (long)H.first.size() - 1;
  }
  a->E2 = (double*)(w + A.o_E2);
  a->E2T = (double*)(w + A.o_E2T);
  for (int l = 0; l < A.nlev; ++l) a->pos.push_back(A.lev[l].pos);
  L.ws = (hydro::WorkHeader*)w;
  L.dt = 0.0;
  L.cfl = 0.0;
  L.slot = 0;
  hipStream_t s = (hipStream_t)d->stream;
  hydro::amr_segments(N, L, L.segs);
  hipError_t e = hipMemsetAsync(w, 0, 256, s);
  if (e == hipSuccess && !host.empty())
    e = hipMemcpyAsync(tab, host.data(), sizeof(int) * host.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);   // the host table is temporary
  if (e != hipSuccess) {
    delete a;
    return hip_fail(e, "AMR table upload");
  }
  *out = a;
  return HYDRO_OK;
}

}  // extern "C"

namespace {

int amr_ensure_signal(hydro_amr* a) {
  if (a->sig_valid) return HYDRO_OK;
  hipError_t e = hydro::launch_amr_signal(a->d.nxb, a->L, (int)(a->steps % 3), (hipStream_t)a->d.stream);
  if (e != hipSuccess) return hip_fail(e, "AMR signal launch");
  a->sig_valid = true;
  return HYDRO_OK;
}

int amr_launch(hydro_amr* a, double dt, double cfl) {
  a->L.dt = dt;
  a->L.cfl = cfl;
  a->L.slot = (int)(a->steps % 3);
  hipError_t e = hydro::launch_amr_step(a->d.nxb, a->L, (hipStream_t)a->d.stream);
  if (e != hipSuccess) return hip_fail(e, "AMR step launch");
  ++a->steps;
  a->sig_valid = true;  // the step reduced the new state's signal speed
  return HYDRO_OK;
}

int amr_read_header(hydro_amr* a, hydro::WorkHeader* h) {
  hipStream_t s = (hipStream_t)a->d.stream;
  hipError_t e = hipMemcpyAsync(h, a->d.work, sizeof *h, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "AMR header read");
  return HYDRO_OK;
}

}  // namespace

extern "C" {

int hydro_amr_step(hydro_amr* a, double dt) {
  if (!a) return fail(HYDRO_EINVAL, "handle is NULL");
  if (!finite_pos(dt)) return fail(HYDRO_EINVAL, "dt must be finite and > 0 (got %g)", dt);
  return amr_launch(a, dt, 0.0);
}

int hydro_amr_step_cfl(hydro_amr* a, double cfl) {
  if (!a) return fail(HYDRO_EINVAL, "handle is NULL");
  if (!finite_pos(cfl)) return fail(HYDRO_EINVAL, "cfl must be finite and > 0");
  int rc = amr_ensure_signal(a);
  if (rc) return rc;
  return amr_launch(a, 0.0, cfl);
}

int hydro_amr_dt(hydro_amr* a, double cfl, double* dt_out) {
  if (!a || !dt_out) return fail(HYDRO_EINVAL, "handle or dt_out is NULL");
  if (!finite_pos(cfl)) return fail(HYDRO_EINVAL, "cfl must be finite and > 0");
  int rc = amr_ensure_signal(a);
  if (rc) return rc;
  hydro::WorkHeader h;
  rc = amr_read_header(a, &h);
  if (rc) return rc;
  double sig;
  memcpy(&sig, &h.sig[a->steps % 3], sizeof sig);
  const bool ok = std::isfinite(sig) && sig > 0.0;
  if (ok) *dt_out = cfl / sig;
  if (h.cnt[2] != 0)
    return fail(HYDRO_ENONPHYS, "%llu nonphysical cells produced since creation", h.cnt[2]);
  if (!ok) return fail(HYDRO_EINVAL, "maximum signal speed %g is not positive and finite", sig);
  return HYDRO_OK;
}

int hydro_amr_last_dt(hydro_amr* a, double* dt_out) {
  if (!a || !dt_out) return fail(HYDRO_EINVAL, "handle or dt_out is NULL");
  if (a->steps == 0) return fail(HYDRO_EINVAL, "no step has been taken");
  hydro::WorkHeader h;
  int rc = amr_read_header(a, &h);
  if (rc) return rc;
  *dt_out = h.dt_last;
  return HYDRO_OK;
}

int hydro_amr_state_changed(hydro_amr* a) {
  if (!a) return fail(HYDRO_EINVAL, "handle is NULL");
  a->sig_valid = false;
  return HYDRO_OK;
}

int hydro_amr_estimate(hydro_amr* a, double eps, double refine_cutoff, double derefine_cutoff, double* E2_out,
                       unsigned char* flags_out) {
  if (!a || !flags_out) return fail(HYDRO_EINVAL, "handle or flags_out is NULL");
  if (!(std::isfinite(eps) && eps >= 0.0)) return fail(HYDRO_EINVAL, "eps must be finite and >= 0");
  if (!(std::isfinite(refine_cutoff) && std::isfinite(derefine_cutoff) && derefine_cutoff >= 0.0 &&
        derefine_cutoff <= refine_cutoff))
    return fail(HYDRO_EINVAL, "need finite cutoffs with 0 <= derefine_cutoff <= refine_cutoff");
  hipStream_t s = (hipStream_t)a->d.stream;
  hipError_t e = hydro::launch_amr_indicator(a->d.nxb, a->L, eps, a->E2, s);
  if (e != hipSuccess) return hip_fail(e, "AMR indicator launch");
  std::vector<double> E2((size_t)a->L.lev[0].nblk);
  e = hipMemcpyAsync(E2.data(), a->E2, sizeof(double) * E2.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "AMR indicator read");
  const double rc2 = refine_cutoff * refine_cutoff, dc2 = derefine_cutoff * derefine_cutoff;
  for (long b = 0; b < a->L.lev[0].nblk; ++b) {
    unsigned char f = a->refine[b] ? 1 : 0;
    if (E2[b] > rc2) f = 1;
    else if (f && E2[b] < dc2) f = 0;
    flags_out[b] = f;
    if (E2_out) E2_out[b] = E2[b];
  }
  return HYDRO_OK;
}

}  // extern "C"

namespace {

using Pos = std::array<int, 3>;

// Refinement state as sets of refined block positions per level.
struct TreeFlags {
  std::vector<std::set<Pos>> R;
  int nb0[3];
  int bc[3];

  bool is_block(int l, const Pos& p) const {
    return l == 0 || R[l - 1].count(Pos{p[0] / 2, p[1] / 2, p[2] / 2}) > 0;
  }
  bool wrap(int l, Pos& q) const {
    for (int d = 0; d < 3; ++d) {
      const int n = nb0[d] << l;
      if (bc[d] == HYDRO_BC_PERIODIC) q[d] = ((q[d] % n) + n) % n;
      else if (q[d] < 0 || q[d] >= n) return false;
    }
    return true;
  }
  void ensure_block(int l, const Pos& p) {
    if (is_block(l, p)) return;
    const Pos par{p[0] / 2, p[1] / 2, p[2] / 2};
    ensure_block(l - 1, par);
    R[l - 1].insert(par);
  }
  // every refined block of a level >= 1 gets its 26 same-level neighbours:
  // refine (coarsest level first, positions in increasing order) until stable
  void restore_nesting() {
    bool changed = true;
    while (changed) {
      changed = false;
      for (size_t l = 1; l < R.size(); ++l) {
        const std::vector<Pos> snap(R[l].begin(), R[l].end());
        for (const Pos& p : snap)
          if (!is_block((int)l, p)) {
            R[l].erase(p);
            changed = true;
          }
      }
      for (size_t l = 1; l < R.size(); ++l) {
        const std::vector<Pos> snap(R[l].begin(), R[l].end());
        for (const Pos& p : snap)
          for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
              for (int dx = -1; dx <= 1; ++dx) {
                Pos q{p[0] + dx, p[1] + dy, p[2] + dz};
                if (wrap((int)l, q) && !is_block((int)l, q)) {
                  ensure_block((int)l, q);
                  changed = true;
                }
              }
      }
    }
  }
  // flags in descriptor order: level 0 in block order, then each deeper
  // level's blocks (children of the previous level's refined blocks)
  std::vector<unsigned char> flags(long nroot) const {
    std::vector<unsigned char> out;
    std::vector<Pos> cur;
    for (long b = 0; b < nroot; ++b)
      cur.push_back(Pos{(int)(b % nb0[0]), (int)((b / nb0[0]) % nb0[1]), (int)(b / ((long)nb0[0] * nb0[1]))});
    for (size_t l = 0;; ++l) {
      std::vector<Pos> next;
      bool any = false;
      for (const Pos& p : cur) {
        const bool f = l < R.size() && R[l].count(p) > 0;
        out.push_back(f ? 1 : 0);
        if (f) {
          any = true;
          for (int c = 0; c < 8; ++c)
            next.push_back(Pos{2 * p[0] + (c & 1), 2 * p[1] + ((c >> 1) & 1), 2 * p[2] + ((c >> 2) & 1)});
        }
      }
      if (!any) break;
      cur.swap(next);
    }
    return out;
  }
};

}  // namespace

extern "C" {

int hydro_amr_estimate_tree(hydro_amr* a, double eps, double refine_cutoff, double derefine_cutoff, int max_levels,
                            double* E2_out, unsigned char* flags_out, size_t cap, size_t* nflags_out) {
  if (!a || !nflags_out) return fail(HYDRO_EINVAL, "handle or nflags_out is NULL");
  if (!(std::isfinite(eps) && eps >= 0.0)) return fail(HYDRO_EINVAL, "eps must be finite and >= 0");
  if (!(std::isfinite(refine_cutoff) && std::isfinite(derefine_cutoff) && derefine_cutoff >= 0.0 &&
        derefine_cutoff <= refine_cutoff))
    return fail(HYDRO_EINVAL, "need finite cutoffs with 0 <= derefine_cutoff <= refine_cutoff");
  if (max_levels < 1 || max_levels > hydro::AMR_MAX_LEVELS)
    return fail(HYDRO_EINVAL, "max_levels must be in 1..%d", hydro::AMR_MAX_LEVELS);
  const hydro::AmrLaunch& L = a->L;
  hipStream_t s = (hipStream_t)a->d.stream;
  size_t nall = 0;
  double* lev_ptr[hydro::AMR_MAX_LEVELS];
  for (int l = 0; l < L.nlev; ++l) {
    lev_ptr[l] = a->E2T + nall;
    nall += (size_t)L.lev[l].nblk;
  }
  hipError_t e = hipMemsetAsync(a->E2T, 0, sizeof(double) * nall, s);   // refined blocks read as 0
  if (e == hipSuccess) e = hydro::launch_amr_leaf_indicator(a->d.nxb, L, eps, lev_ptr, s);
  if (e != hipSuccess) return hip_fail(e, "AMR indicator launch");
  std::vector<double> E2(nall);
  e = hipMemcpyAsync(E2.data(), a->E2T, sizeof(double) * nall, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "AMR indicator read");
  if (E2_out) std::copy(E2.begin(), E2.end(), E2_out);
  // the rule
  TreeFlags T;
  for (int d = 0; d < 3; ++d) {
    T.nb0[d] = a->d.nblk[d];
    T.bc[d] = a->d.bc[d];
  }
  T.R.resize(std::max(L.nlev, max_levels));
  // current flags of every level, from the descriptor's flags
  std::vector<std::vector<unsigned char>> flag(L.nlev);
  flag[0].assign(a->refine.begin(), a->refine.end());
  size_t used = 0;
  for (int l = 1; l < L.nlev; ++l) {
    const size_t nb = (size_t)L.lev[l].nblk;
    if (used + nb <= a->refine_deep.size())
      flag[l].assign(a->refine_deep.begin() + used, a->refine_deep.begin() + used + nb);
    else
      flag[l].assign(nb, 0);
    used += nb;
  }
  auto pos_of = [&](int l, long b) { return Pos{a->pos[l][4 * b], a->pos[l][4 * b + 1], a->pos[l][4 * b + 2]}; };
  size_t off = 0;
  std::vector<size_t> level_off(L.nlev);
  for (int l = 0; l < L.nlev; ++l) {
    level_off[l] = off;
    off += (size_t)L.lev[l].nblk;
    for (long b = 0; b < L.lev[l].nblk; ++b)
      if (flag[l][b]) T.R[l].insert(pos_of(l, b));
  }
  const double rc2 = refine_cutoff * refine_cutoff, dc2 = derefine_cutoff * derefine_cutoff;
  for (int l = 0; l < L.nlev; ++l)
    for (long b = 0; b < L.lev[l].nblk; ++b)
      if (!flag[l][b] && E2[level_off[l] + b] > rc2 && l + 1 < max_levels) T.R[l].insert(pos_of(l, b));
  for (int l = 0; l + 1 < L.nlev; ++l) {
    long base = 0;  // children of the refined blocks of level l are contiguous, in block order
    for (long r = 0; r < L.lev[l].nblk; ++r) {
      if (!flag[l][r]) continue;
      bool all = true;
      for (long k = base; k < base + 8; ++k) all = all && !flag[l + 1][k] && E2[level_off[l + 1] + k] < dc2;
      if (all) T.R[l].erase(pos_of(l, r));
      base += 8;
    }
  }
  T.restore_nesting();
  const std::vector<unsigned char> out = T.flags(L.lev[0].nblk);
  *nflags_out = out.size();
  if (!flags_out || cap < out.size())
    return fail(HYDRO_ESIZE, "the new flags need %zu entries (capacity %zu)", out.size(), cap);
  std::copy(out.begin(), out.end(), flags_out);
  return HYDRO_OK;
}

int hydro_amr_transfer(hydro_amr* from, hydro_amr* to) {
  if (!from || !to || from == to) return fail(HYDRO_EINVAL, "need two distinct handles");
  const hydro_amr_desc &x = from->d, &y = to->d;
  bool same = x.nxb == y.nxb && x.gamma == y.gamma;
  for (int ax = 0; ax < 3; ++ax)
    same = same && x.nblk[ax] == y.nblk[ax] && x.bc[ax] == y.bc[ax] && x.lo[ax] == y.lo[ax] && x.hi[ax] == y.hi[ax];
  if (!same) return fail(HYDRO_EINVAL, "the two meshes must share their root grid");
  if (y.Uf == x.Uf && to->L.nlev > 1 && from->L.nlev > 1)
    return fail(HYDRO_EINVAL, "the new mesh needs a fine state buffer of its own");
  hipError_t e = hipStreamSynchronize((hipStream_t)x.stream);  // the old mesh's last step has finished
  if (e != hipSuccess) return hip_fail(e, "AMR transfer: waiting for the old mesh");
  hipStream_t s = (hipStream_t)y.stream;
  const size_t N3 = (size_t)x.nxb * x.nxb * x.nxb;
  if (y.Ur != x.Ur) {
    e = hipMemcpyAsync(y.Ur, x.Ur, sizeof(double) * 5 * N3 * (size_t)from->L.lev[0].nblk, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "AMR transfer: root state copy");
  }
  e = hydro::launch_amr_transfer(y.nxb, from->L, to->L, s);
  if (e != hipSuccess) return hip_fail(e, "AMR transfer launch");
  to->sig_valid = false;
  return HYDRO_OK;
}

int hydro_amr_counters(hydro_amr* a, long long out[3]) {
  if (!a || !out) return fail(HYDRO_EINVAL, "handle or out is NULL");
  hipStream_t s = (hipStream_t)a->d.stream;
  hydro::WorkHeader h;
  hipError_t e = hipMemcpyAsync(&h, a->d.work, sizeof h, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "AMR header read");
  for (int c = 0; c < 3; ++c) out[c] = (long long)h.cnt[c];
  return HYDRO_OK;
}

int hydro_amr_set_columns(hydro_amr* a, int cap) {
  if (!a) return fail(HYDRO_EINVAL, "AMR handle is NULL");
  if (cap != 0 && cap != 1 && cap != 2 && cap != 4) return fail(HYDRO_EINVAL, "column length must be 0, 1, 2 or 4");
  hipStream_t s = (hipStream_t)a->d.stream;
  std::vector<int> host;
  for (size_t l = 0; l < a->cols.size(); ++l) {
    const hydro_amr::Cols& C = a->cols[l];
    const std::vector<int> cp = amr_best_columns(C.nb, C.lookup, a->pos[l], C.plain, a->d.nxb, a->tpb, a->slots, cap);
    const std::vector<int> cr = amr_best_columns(C.nb, C.lookup, a->pos[l], C.rx, a->d.nxb, a->tpb, a->slots, cap);
    const std::vector<int> zn = amr_zneed(a->pos[l].size() / 4, cp, cr, C.face);
    hipError_t e = hipSuccess;
    if (!cp.empty()) e = hipMemcpyAsync(C.d_plain, cp.data(), sizeof(int) * cp.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !cr.empty())
      e = hipMemcpyAsync(C.d_rx, cr.data(), sizeof(int) * cr.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(C.d_zneed, zn.data(), sizeof(int) * zn.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);   // the host tables are temporary
    if (e != hipSuccess) return hip_fail(e, "AMR column table upload");
    a->L.lev[l].ncols_plain = (long)cp.size() / 4;
    a->L.lev[l].ncols_rx = (long)cr.size() / 4;
    a->L.lev[l].kmax_plain = amr_kmax(cp);
    a->L.lev[l].kmax_rx = amr_kmax(cr);
  }
  hydro::amr_segments(a->d.nxb, a->L, a->L.segs);
  return HYDRO_OK;
}

int hydro_amr_free(hydro_amr* a) {
  delete a;
  return HYDRO_OK;
}

}  // extern "C"
