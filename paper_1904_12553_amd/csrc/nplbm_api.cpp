// nplbm_api.cpp -- the single-domain part of the C ABI (include/nplbm.h).
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "host_internal.h"
#include "nplbm.h"
#include "nplbm_internal.h"

using namespace nplbm;

struct nplbm_domain {
  nplbm_params p;
  std::vector<double> sigma, rho, mu, mob, tau;  // owned copies
  Derived d;
  Layout L;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  unsigned char *base = nullptr;
  bool own_mem = false;
  DomDesc desc;          // host copy of the device descriptor
  DomDesc *desc_dev = nullptr;
  StripDesc *strips_dev = nullptr;
  int nstrips = 0;
  StepGeom geom{64, 60, 1};  // strip geometry of the step kernel
  bool d3 = false;           // 3-D (D3Q15) domain
  int ty = 8;                // tile rows of the 3-D step kernel
  int64_t t = 0;
  bool initialised = false;
  // graphs of 2^j consecutive steps (j = 0..kGraphLevels-1) starting at an
  // even (index 0) or odd (index 1) time step
  hipGraphExec_t graph[2][7] = {{nullptr}};
};

namespace {

// step runs are replayed as graphs of 64, 32, ..., 1 steps
constexpr int kGraphLevels = 7;

double *dptr(nplbm_domain *d, size_t off) { return reinterpret_cast<double *>(d->base + off); }

size_t nnodes(const nplbm_domain *d) { return (size_t)d->p.nx * d->p.ny * dom_nz(&d->p); }

hipError_t launch_any_step(nplbm_domain *d, const StepArgs &a) {
  if (d->d3)
    return launch_step3(d->p.N, d->p.precision, d->ty, a, d->nstrips, d->p.nx, d->p.ny, d->p.nz,
                        d->stream);
  return launch_step(d->p.N, d->p.precision, step_scheme(&d->p), d->geom.bw, a, d->nstrips,
                     d->stream);
}

// resident 3-D step workgroups on the device (0 if unknown)
int resident_step3_blocks(int N, int precision, int ty) {
  int dev = 0, cus = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    cus = prop.multiProcessorCount;
  const int per = step3_blocks_per_cu(N, precision, ty);
  return cus > 0 && per > 0 ? cus * per : 0;
}

int launch_one_step(nplbm_domain *d) {
  StepArgs a;
  std::memset(&a, 0, sizeof a);
  a.strips = d->strips_dev;
  a.doms = d->desc_dev;
  a.substep = (int)(d->t & 1);
  hipError_t e = launch_any_step(d, a);
  if (e != hipSuccess) return hip_fail(e, "step launch");
  d->t += 1;
  return NPLBM_OK;
}

// Capture (once) the graph of 2^level steps starting at a time of parity
// `par`: the launches alternate the ping-pong buffers from that parity.
int capture_graph(nplbm_domain *d, int par, int level) {
  if (d->graph[par][level]) return NPLBM_OK;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(d->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  StepArgs a;
  std::memset(&a, 0, sizeof a);
  a.strips = d->strips_dev;
  a.doms = d->desc_dev;
  hipError_t le = hipSuccess;
  for (int s = 0; s < (1 << level) && le == hipSuccess; ++s) {
    a.substep = (par + s) & 1;
    le = launch_any_step(d, a);
  }
  e = hipStreamEndCapture(d->stream, &g);
  if (le != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(le, "step launch during capture");
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&d->graph[par][level], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    d->graph[par][level] = nullptr;
    return hip_fail(e, "hipGraphInstantiate");
  }
  return NPLBM_OK;
}

// The graphs a run starting at an even time uses, and the one-step graph
// of odd start: captured together at the first step call, so that later
// runs of any length replay existing graphs.
int capture_all(nplbm_domain *d) {
  for (int level = 0; level < kGraphLevels; ++level) {
    int rc = capture_graph(d, 0, level);
    if (rc) return rc;
  }
  return capture_graph(d, 1, 0);
}

int readback(nplbm_domain *d, bool want_up) {
  const int par = (int)(d->t & 1);
  if (d->d3) {
    hipError_t e = launch_macro3(d->desc_dev, d->desc, d->p.precision, par, dptr(d, d->L.phi),
                                 dptr(d, d->L.rho), dptr(d, d->L.C), dptr(d, d->L.c),
                                 want_up ? dptr(d, d->L.u) : nullptr,
                                 want_up ? dptr(d, d->L.p) : nullptr, d->stream);
    if (e != hipSuccess) return hip_fail(e, "macro launch");
    return NPLBM_OK;
  }
  hipError_t e = launch_macro(d->desc_dev, d->desc, d->p.precision, par, dptr(d, d->L.phi),
                              dptr(d, d->L.rho), dptr(d, d->L.C), dptr(d, d->L.c),
                              want_up ? dptr(d, d->L.u) : nullptr,
                              want_up ? dptr(d, d->L.p) : nullptr,
                              d->L.q ? dptr(d, d->L.q) : nullptr, d->stream);
  if (e != hipSuccess) return hip_fail(e, "macro launch");
  return NPLBM_OK;
}

int copy_out(nplbm_domain *d, void *dst, size_t off, size_t bytes) {
  hipError_t e = hipMemcpyAsync(dst, d->base + off, bytes, hipMemcpyDeviceToHost, d->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync D2H");
  e = hipStreamSynchronize(d->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return NPLBM_OK;
}

bool check_domain(const nplbm_domain *d) { return d != nullptr && d->base != nullptr; }

}  // namespace

extern "C" {

const char *nplbm_last_error(void) { return last_error(); }

int nplbm_validate(const nplbm_params *p, double *lambda_out, double *beta2_out, double *K_out) {
  clear_error();
  Derived d;
  int rc = derive(p, d);
  if (rc) return rc;
  const int M = p->N - 1;
  if (lambda_out)
    for (int i = 0; i < M * M; ++i) lambda_out[i] = d.lam[i];
  if (beta2_out) *beta2_out = d.beta2;
  if (K_out) *K_out = d.K;
  return NPLBM_OK;
}

size_t nplbm_footprint(const nplbm_params *p) {
  Derived d;
  if (derive(p, d)) return 0;
  return plan_layout(p).total;
}

int nplbm_create(const nplbm_params *p, void *stream, void *device_mem, size_t device_bytes,
                 nplbm_domain **out) {
  clear_error();
  if (!out) return fail(NPLBM_EINVAL, "out is NULL");
  *out = nullptr;
  nplbm_domain *d = new nplbm_domain();
  int rc = derive(p, d->d);
  if (rc) {
    delete d;
    return rc;
  }
  const int N = p->N;
  d->sigma.assign(p->sigma, p->sigma + N * N);
  d->rho.assign(p->rho, p->rho + N);
  d->mu.assign(p->mu, p->mu + N);
  d->mob.assign(p->mobility, p->mobility + N - 1);
  d->tau.assign(p->tau_phi, p->tau_phi + N - 1);
  d->p = *p;
  d->p.sigma = d->sigma.data();
  d->p.rho = d->rho.data();
  d->p.mu = d->mu.data();
  d->p.mobility = d->mob.data();
  d->p.tau_phi = d->tau.data();
  d->L = plan_layout(&d->p);
  hipError_t e = hipGetDevice(&d->device);
  if (e != hipSuccess) {
    delete d;
    return hip_fail(e, "hipGetDevice");
  }
  // set-up of the static scratch of nplbm_diagnostics_noalloc on this device
  // (its address is looked up once per device, here, outside any capture)
  double *scr = nullptr;
  e = static_diag_scratch(&scr);
  if (e != hipSuccess) {
    delete d;
    return hip_fail(e, "static scratch address");
  }
  d->stream = static_cast<hipStream_t>(stream);
  if (device_mem) {
    if (device_bytes < d->L.total) {
      size_t need = d->L.total;
      delete d;
      return fail(NPLBM_ENOMEM, "device buffer of %zu bytes, %zu needed", device_bytes, need);
    }
    if (reinterpret_cast<uintptr_t>(device_mem) & 255) {
      delete d;
      return fail(NPLBM_EINVAL, "device_mem must be 256-byte aligned");
    }
    d->base = static_cast<unsigned char *>(device_mem);
  } else {
    void *m = nullptr;
    e = hipMalloc(&m, d->L.total);
    if (e != hipSuccess) {
      size_t need = d->L.total;
      delete d;
      return fail(NPLBM_ENOMEM, "hipMalloc(%zu): %s", need, hipGetErrorString(e));
    }
    d->base = static_cast<unsigned char *>(m);
    d->own_mem = true;
  }
  // descriptor
  DomDesc &D = d->desc;
  std::memset(&D, 0, sizeof D);
  for (int b = 0; b < 2; ++b) {
    D.h[b] = d->base + d->L.h[b];
    D.g[b] = d->base + d->L.g[b];
  }
  D.prev[0] = d->base + d->L.prev[0];
  D.prev[1] = d->base + d->L.prev[1];
  for (int G = 0; G < 3; ++G) {
    D.ps[G] = d->L.ps[G];
    D.rs[G] = d->L.rs[G];
  }
  D.nx = p->nx;
  D.ny = p->ny;
  D.nz = dom_nz(p);
  if (is3d(p)) {
    D.phi3 = d->base + d->L.phi3;
    D.rsf = (N - 1) * d->L.pitch;
  }
  D.pitch = d->L.pitch;
  D.wall = is3d(p) ? p->wall_z : p->wall_y;
  D.N = N;
  D.parity0 = 0;
  D.steps_left = INT_MAX;
  D.scheme = step_scheme(p);
  D.cd = d->d.cd;
  D.cf = d->d.cf;
  d->desc_dev = reinterpret_cast<DomDesc *>(d->base + d->L.desc);
  std::vector<StripDesc> strips;
  d->d3 = is3d(p);
  if (d->d3) {
    d->ty = step3_ty(N, p->precision);
    int target = resident_step3_blocks(N, p->precision, d->ty);
    if (const char *env = std::getenv("NPLBM_TARGET_BLOCKS")) target = std::atoi(env);
    build_tiles3(p->nx, p->ny, p->nz, 0, d->ty, target, strips);
  } else {
    d->geom = step_geom(p->N, p->precision, step_scheme(p));
    build_strips(p->nx, p->ny, 0, d->geom, strips, single_domain_target(p));
  }
  xcd_order(strips);
  if ((int)strips.size() > d->L.nstrips) {
    nplbm_destroy(d);
    return fail(NPLBM_EINVAL, "strip table overflow");
  }
  d->nstrips = (int)strips.size();
  d->strips_dev = reinterpret_cast<StripDesc *>(d->base + d->L.strips);
  e = hipMemcpyAsync(d->desc_dev, &D, sizeof D, hipMemcpyHostToDevice, d->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d->strips_dev, strips.data(), sizeof(StripDesc) * strips.size(),
                       hipMemcpyHostToDevice, d->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(d->stream);
  if (e != hipSuccess) {
    int r = hip_fail(e, "descriptor upload");
    nplbm_destroy(d);
    return r;
  }
  *out = d;
  return NPLBM_OK;
}

int nplbm_set_fields(nplbm_domain *d, const double *c, const double *u) {
  clear_error();
  if (!check_domain(d) || !c) return fail(NPLBM_EINVAL, "NULL domain or c");
  const int N = d->p.N;
  const size_t n = nnodes(d);
  const int nu = d->d3 ? 3 : 2;
  for (size_t id = 0; id < n; ++id) {
    double s = 0.0;
    for (int k = 0; k < N; ++k) {
      const double v = c[(size_t)k * n + id];
      if (!std::isfinite(v)) return fail(NPLBM_EINVAL, "c is not finite at node %zu", id);
      s += v;
    }
    if (std::fabs(s - 1.0) > 1e-9)
      return fail(NPLBM_EINVAL, "sum_k c_k = %.17g at node %zu (must be 1)", s, id);
  }
  if (u)
    for (size_t id = 0; id < nu * n; ++id)
      if (!std::isfinite(u[id])) return fail(NPLBM_EINVAL, "u is not finite");
  hipError_t e = hipMemcpyAsync(dptr(d, d->L.c), c, (size_t)N * n * 8, hipMemcpyHostToDevice,
                                d->stream);
  if (e == hipSuccess && u)
    e = hipMemcpyAsync(dptr(d, d->L.u), u, nu * n * 8, hipMemcpyHostToDevice, d->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync H2D");
  e = (d->d3 ? launch_init3 : launch_init)(d->desc_dev, d->desc, d->p.precision, d->d.P1,
                                           d->d.PN, d->d.P0, dptr(d, d->L.c),
                                           u ? dptr(d, d->L.u) : nullptr, dptr(d, d->L.phi),
                                           dptr(d, d->L.C), d->stream);
  if (e != hipSuccess) return hip_fail(e, "init launch");
  e = hipStreamSynchronize(d->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  d->t = 0;
  d->initialised = true;
  return NPLBM_OK;
}

int nplbm_step(nplbm_domain *d, int64_t nsteps) {
  clear_error();
  if (!check_domain(d)) return fail(NPLBM_EINVAL, "NULL domain");
  if (nsteps < 0) return fail(NPLBM_EINVAL, "nsteps < 0");
  if (!d->initialised) return fail(NPLBM_ESTATE, "nplbm_set_fields was not called");
  // runs are replayed as HIP graphs of 2^j steps (the largest that fits the
  // steps left, at most 64); the null stream cannot be captured, so there
  // (and with NPLBM_NO_GRAPH set) every step is launched on its own
  const bool use_graph = d->stream && std::getenv("NPLBM_NO_GRAPH") == nullptr;
  if (use_graph && nsteps > 0) {
    int rc = capture_all(d);
    if (rc) return rc;
  }
  while (nsteps > 0) {
    if (!use_graph) {
      int rc = launch_one_step(d);
      if (rc) return rc;
      nsteps -= 1;
      continue;
    }
    int level = kGraphLevels - 1;
    while ((int64_t)1 << level > nsteps) --level;
    const int par = (int)(d->t & 1);
    if (par) level = 0;  // an odd start takes one step to reach even parity
    int rc = capture_graph(d, par, level);
    if (rc) return rc;
    hipError_t e = hipGraphLaunch(d->graph[par][level], d->stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    d->t += (int64_t)1 << level;
    nsteps -= (int64_t)1 << level;
  }
  return NPLBM_OK;
}

int nplbm_get_c(nplbm_domain *d, double *c) {
  clear_error();
  if (!check_domain(d) || !c) return fail(NPLBM_EINVAL, "NULL argument");
  if (!d->initialised) return fail(NPLBM_ESTATE, "nplbm_set_fields was not called");
  int rc = readback(d, false);
  if (rc) return rc;
  return copy_out(d, c, d->L.c, (size_t)d->p.N * nnodes(d) * 8);
}

int nplbm_get_u(nplbm_domain *d, double *u) {
  clear_error();
  if (!check_domain(d) || !u) return fail(NPLBM_EINVAL, "NULL argument");
  if (!d->initialised) return fail(NPLBM_ESTATE, "nplbm_set_fields was not called");
  int rc = readback(d, true);
  if (rc) return rc;
  return copy_out(d, u, d->L.u, (size_t)(d->d3 ? 3 : 2) * nnodes(d) * 8);
}

int nplbm_get_p(nplbm_domain *d, double *p) {
  clear_error();
  if (!check_domain(d) || !p) return fail(NPLBM_EINVAL, "NULL argument");
  if (!d->initialised) return fail(NPLBM_ESTATE, "nplbm_set_fields was not called");
  int rc = readback(d, true);
  if (rc) return rc;
  return copy_out(d, p, d->L.p, nnodes(d) * 8);
}

int nplbm_diagnostics(nplbm_domain *d, double *mass_out, double *max_sum_dev,
                      int64_t *nonfinite) {
  clear_error();
  if (!check_domain(d)) return fail(NPLBM_EINVAL, "NULL domain");
  if (!d->initialised) return fail(NPLBM_ESTATE, "nplbm_set_fields was not called");
  int rc = readback(d, false);
  if (rc) return rc;
  const int N = d->p.N;
  const int64_t n = (int64_t)nnodes(d);
  hipError_t e = launch_diag(dptr(d, d->L.c), N, n, dptr(d, d->L.partials), d->L.nblk,
                             dptr(d, d->L.out), d->stream);
  if (e != hipSuccess) return hip_fail(e, "diag launch");
  double out[kMaxN + 2];
  rc = copy_out(d, out, d->L.out, (size_t)(N + 2) * 8);
  if (rc) return rc;
  if (mass_out)
    for (int k = 0; k < N; ++k) mass_out[k] = out[k];
  if (max_sum_dev) *max_sum_dev = out[N];
  if (nonfinite) *nonfinite = (int64_t)out[N + 1];
  return NPLBM_OK;
}

int nplbm_diagnostics_noalloc(nplbm_domain *d, double *out_dev) {
  clear_error();
  if (!check_domain(d) || !out_dev) return fail(NPLBM_EINVAL, "NULL argument");
  if (!d->initialised) return fail(NPLBM_ESTATE, "nplbm_set_fields was not called");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != d->device)
    return fail(NPLBM_EINVAL, "the domain lives on device %d, device %d is current", d->device,
                dev);
  const int N = d->p.N;
  const int nblk = d->L.nblk;
  if ((int64_t)nblk * (N + 2) > kStaticDiagPartials)
    return fail(NPLBM_EINVAL, "reduction of %d blocks x %d values exceeds the static scratch "
                "(%d doubles)", nblk, N + 2, kStaticDiagPartials);
  double *scr = nullptr;
  e = static_diag_scratch(&scr);
  if (e != hipSuccess) return hip_fail(e, "static scratch address");
  int rc = readback(d, false);
  if (rc) return rc;
  e = launch_diag(dptr(d, d->L.c), N, (int64_t)nnodes(d), scr, nblk, out_dev, d->stream);
  if (e != hipSuccess) return hip_fail(e, "diag launch");
  return NPLBM_OK;
}

int nplbm_laplace(nplbm_domain *d, double xc, double yc, double r_in, double r_out, double *dp) {
  clear_error();
  if (!check_domain(d) || !dp) return fail(NPLBM_EINVAL, "NULL argument");
  if (!d->initialised) return fail(NPLBM_ESTATE, "nplbm_set_fields was not called");
  if (!(r_in >= 0.0) || !(r_out >= r_in)) return fail(NPLBM_EINVAL, "need 0 <= r_in <= r_out");
  if (d->d3) return fail(NPLBM_EINVAL, "nplbm_laplace measures 2-D domains (see nplbm_laplace3)");
  int rc = readback(d, true);
  if (rc) return rc;
  hipError_t e = launch_laplace(dptr(d, d->L.p), d->p.nx, d->p.ny, 1, xc, yc, 0.0, r_in, r_out,
                                dptr(d, d->L.partials), d->L.nblk, dptr(d, d->L.out), d->stream);
  if (e != hipSuccess) return hip_fail(e, "laplace launch");
  return copy_out(d, dp, d->L.out, 8);
}

int nplbm_laplace3(nplbm_domain *d, double xc, double yc, double zc, double r_in, double r_out,
                   double *dp) {
  clear_error();
  if (!check_domain(d) || !dp) return fail(NPLBM_EINVAL, "NULL argument");
  if (!d->initialised) return fail(NPLBM_ESTATE, "nplbm_set_fields was not called");
  if (!(r_in >= 0.0) || !(r_out >= r_in)) return fail(NPLBM_EINVAL, "need 0 <= r_in <= r_out");
  if (!d->d3) return fail(NPLBM_EINVAL, "nplbm_laplace3 measures 3-D domains (see nplbm_laplace)");
  int rc = readback(d, true);
  if (rc) return rc;
  hipError_t e = launch_laplace(dptr(d, d->L.p), d->p.nx, d->p.ny, d->p.nz, xc, yc, zc, r_in,
                                r_out, dptr(d, d->L.partials), d->L.nblk, dptr(d, d->L.out),
                                d->stream);
  if (e != hipSuccess) return hip_fail(e, "laplace launch");
  return copy_out(d, dp, d->L.out, 8);
}

int64_t nplbm_time(const nplbm_domain *d) { return d ? d->t : -1; }

int nplbm_sync(nplbm_domain *d) {
  clear_error();
  if (!check_domain(d)) return fail(NPLBM_EINVAL, "NULL domain");
  hipError_t e = hipStreamSynchronize(d->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return NPLBM_OK;
}

void nplbm_destroy(nplbm_domain *d) {
  if (!d) return;
  if (d->stream) (void)hipStreamSynchronize(d->stream);
  else (void)hipDeviceSynchronize();
  for (auto &row : d->graph)
    for (hipGraphExec_t &g : row)
      if (g) (void)hipGraphExecDestroy(g);
  if (d->own_mem && d->base) (void)hipFree(d->base);
  delete d;
}

size_t nplbm_state_bytes(const nplbm_domain *d) {
  if (!d) return 0;
  const size_t s = d->p.precision == 64 ? 8 : 4;
  const int M = d->p.N - 1;
  (void)s;
  (void)M;
  return d->L.gbytes[0] + d->L.gbytes[1] + d->L.gbytes[2];
}

int nplbm_get_state(nplbm_domain *d, void *host, int64_t *time_out) {
  clear_error();
  if (!check_domain(d) || !host) return fail(NPLBM_EINVAL, "NULL argument");
  const size_t s = d->p.precision == 64 ? 8 : 4;
  const int M = d->p.N - 1;
  const int par = (int)(d->t & 1);
  const size_t hb = d->L.gbytes[0], gb = d->L.gbytes[1], pb = d->L.gbytes[2];
  (void)s;
  (void)M;
  unsigned char *o = static_cast<unsigned char *>(host);
  hipError_t e = hipMemcpyAsync(o, d->base + d->L.h[par], hb, hipMemcpyDeviceToHost, d->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(o + hb, d->base + d->L.g[par], gb, hipMemcpyDeviceToHost, d->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(o + hb + gb, d->base + d->L.prev[par], pb, hipMemcpyDeviceToHost,
                       d->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(d->stream);
  if (e != hipSuccess) return hip_fail(e, "state copy");
  if (time_out) *time_out = d->t;
  return NPLBM_OK;
}

int nplbm_set_state(nplbm_domain *d, const void *host, int64_t time) {
  clear_error();
  if (!check_domain(d) || !host || time < 0) return fail(NPLBM_EINVAL, "bad argument");
  const size_t s = d->p.precision == 64 ? 8 : 4;
  const int M = d->p.N - 1;
  const int par = (int)(time & 1);
  const size_t hb = d->L.gbytes[0], gb = d->L.gbytes[1], pb = d->L.gbytes[2];
  (void)s;
  (void)M;
  const unsigned char *o = static_cast<const unsigned char *>(host);
  hipError_t e = hipMemcpyAsync(d->base + d->L.h[par], o, hb, hipMemcpyHostToDevice, d->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d->base + d->L.g[par], o + hb, gb, hipMemcpyHostToDevice, d->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d->base + d->L.prev[par], o + hb + gb, pb, hipMemcpyHostToDevice,
                       d->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(d->stream);
  if (e != hipSuccess) return hip_fail(e, "state copy");
  d->t = time;
  d->initialised = true;
  return NPLBM_OK;
}

int nplbm_device_copy(void *dst, const void *src, size_t nbytes, void *stream) {
  clear_error();
  if (!dst || !src) return fail(NPLBM_EINVAL, "NULL pointer");
  hipError_t e = launch_copy(dst, src, nbytes, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "copy launch");
  return NPLBM_OK;
}

}  // extern "C"
