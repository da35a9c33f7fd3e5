// C-ABI host side of libhydro: descriptor validation, handles, launches.
// The operation and the conventions are documented in include/hydro.h.
#include "../../include/hydro.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>

#include "hydro_internal.h"

struct hydro_grid {
  hydro_grid_desc d;
  hydro::GridGeom geom;
  int cur;                  // 0: state in d.U, 1: in d.U_alt
  unsigned long long steps; // steps taken; signal slot of the current state = steps % 3
  bool sig_valid;           // slot holds the current state's maximum signal speed
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

int ensure_signal(hydro_grid* g) {
  if (g->sig_valid) return HYDRO_OK;
  hipError_t e = hydro::launch_signal(g->d.nxb, g->geom, cur_state(g), ws_of(g), slot_of(g), stream_of(g));
  if (e != hipSuccess) return hip_fail(e, "signal-speed kernel launch");
  g->sig_valid = true;
  return HYDRO_OK;
}

int do_step(hydro_grid* g, double dt, double cfl) {
  hydro::StepArgs a;
  a.Uin = cur_state(g);
  a.Uout = other_state(g);
  a.ws = ws_of(g);
  a.dt = dt;
  a.cfl = cfl;
  a.slot = slot_of(g);
  hipError_t e = hydro::launch_step(g->d.nxb, g->geom, a, stream_of(g));
  if (e != hipSuccess) return hip_fail(e, "step kernel launch");
  g->cur ^= 1;
  g->steps += 1;
  g->sig_valid = true;
  return HYDRO_OK;
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
  for (const double* st : {g->d.U, g->d.U_alt}) {
    const uintptr_t s0 = (uintptr_t)st, s1 = s0 + sb;
    if (o0 < s1 && s0 < o1) return fail(HYDRO_EINVAL, "guarded output overlaps a state buffer");
  }
  hipError_t e = hydro::launch_fill_guards(g->d.nxb, g->geom, cur_state(g), guarded, stream_of(g));
  if (e != hipSuccess) return hip_fail(e, "guard-fill kernel launch");
  return HYDRO_OK;
}

int hydro_step(hydro_grid* g, double dt) {
  if (!g) return fail(HYDRO_EINVAL, "handle is NULL");
  if (!finite_pos(dt)) return fail(HYDRO_EINVAL, "dt must be finite and > 0 (got %g)", dt);
  return do_step(g, dt, 0.0);
}

int hydro_step_cfl(hydro_grid* g, double cfl) {
  if (!g) return fail(HYDRO_EINVAL, "handle is NULL");
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
  if (!(std::isfinite(s) && s > 0.0 && std::isfinite(dt) && dt > 0.0))
    return fail(HYDRO_EINVAL, "maximum signal speed %g is not positive and finite", s);
  *dt_out = dt;
  if (h.cnt[2] != 0)
    return fail(HYDRO_ENONPHYS, "%llu nonphysical cells produced since init", h.cnt[2]);
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
  delete g;
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
