// nplbm_server.cpp -- continuous batching of many small domains on one GPU
// (the serving part of the C ABI in include/nplbm.h).
//
// Every resident domain keeps its distributions in its own device
// allocation for its whole life.  One pump = admit what fits, then one
// quantum of Q steps in which every resident domain of a given (N,
// precision) group is advanced by the same step kernel launch, driven by a
// packed strip table over all the group's domains.  The Q launches of a
// quantum are captured once per resident set into a HIP graph and replayed;
// per-domain progress (which ping-pong buffer is current, how many of the
// Q sub-steps it still needs) lives in a small device array updated before
// each replay, so a domain that finishes mid-quantum simply stops.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "host_internal.h"
#include "nplbm.h"
#include "nplbm_internal.h"

using namespace nplbm;

namespace {

// side streams of the quantum graph (groups beyond this share them)
constexpr int kSideStreams = 4;

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Req {
  uint64_t ticket = 0;
  nplbm_params p{};
  std::vector<double> sigma, rho, mu, mob, tau;
  std::vector<double> c, u;
  bool has_u = false;
  int64_t nsteps = 0;
  int64_t done_steps = 0;
  // 0 queued, 1 resident, 2 done, 3 failed; written and read only under the
  // server's mutex, after everything it publishes (results, times) is written
  int state = 0;
  int err = 0;      // failed request: the error code and message
  std::string msg;
  double t_submit = 0, t_admit = 0, t_done = 0;
  // resident
  Derived d;
  Layout L;
  size_t bytes = 0;
  unsigned char *base = nullptr;
  int slot = -1;
  DomDesc desc{};
  // results
  std::vector<double> c_out, u_out, p_out;
};

}  // namespace

struct nplbm_server {
  size_t budget = 0, used = 0;
  int max_slots = 0, quantum = 1;
  hipStream_t stream = nullptr;
  std::mutex mu;
  uint64_t next_ticket = 1;
  std::deque<Req *> queue;
  std::map<uint64_t, Req *> reqs;
  std::vector<Req *> slots;  // resident requests by slot (nullptr = free)
  DomDesc *descs_dev = nullptr;
  StripDesc *strips_dev = nullptr;
  size_t strips_cap = 0;
  struct Group {
    int N, precision, scheme;
    size_t off, count;
  };
  std::vector<Group> groups;
  // side streams and events of the quantum graph: each group's chain of
  // launches is captured on its own stream, so the groups run side by side
  std::vector<hipStream_t> side;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  hipGraphExec_t graph = nullptr;
  bool dirty = true;
  double node_updates = 0, busy = 0;
  int64_t completed = 0;
  // completion latencies (submit to done) of every finished request, and
  // the first submission / last completion times (under the mutex)
  std::vector<double> lat;
  double t_first = -1.0, t_last = 0.0;
};

namespace {

void release(nplbm_server *s, Req *r) {
  if (r->base) (void)hipFree(r->base);
  r->base = nullptr;
  s->used -= r->bytes;
  if (r->slot >= 0) s->slots[r->slot] = nullptr;
  r->slot = -1;
}

int admit(nplbm_server *s, Req *r) {
  void *m = nullptr;
  hipError_t e = hipMalloc(&m, r->bytes);
  if (e != hipSuccess)
    return fail(NPLBM_ENOMEM, "hipMalloc(%zu): %s", r->bytes, hipGetErrorString(e));
  r->base = static_cast<unsigned char *>(m);
  s->used += r->bytes;
  int slot = -1;
  for (int i = 0; i < s->max_slots; ++i)
    if (!s->slots[i]) {
      slot = i;
      break;
    }
  r->slot = slot;
  s->slots[slot] = r;
  DomDesc &D = r->desc;
  std::memset(&D, 0, sizeof D);
  for (int b = 0; b < 2; ++b) {
    D.h[b] = r->base + r->L.h[b];
    D.g[b] = r->base + r->L.g[b];
  }
  D.prev[0] = r->base + r->L.prev[0];
  D.prev[1] = r->base + r->L.prev[1];
  for (int G = 0; G < 3; ++G) {
    D.ps[G] = r->L.ps[G];
    D.rs[G] = r->L.rs[G];
  }
  D.nx = r->p.nx;
  D.ny = r->p.ny;
  D.nz = 1;
  D.pitch = r->L.pitch;
  D.wall = r->p.wall_y;
  D.N = r->p.N;
  D.parity0 = 0;
  D.steps_left = INT_MAX;
  D.scheme = step_scheme(&r->p);
  D.cd = r->d.cd;
  D.cf = r->d.cf;
  const size_t n = (size_t)r->p.nx * r->p.ny;
  double *cdev = reinterpret_cast<double *>(r->base + r->L.c);
  double *udev = reinterpret_cast<double *>(r->base + r->L.u);
  e = hipMemcpyAsync(s->descs_dev + slot, &D, sizeof D, hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(cdev, r->c.data(), r->c.size() * 8, hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess && r->has_u)
    e = hipMemcpyAsync(udev, r->u.data(), 2 * n * 8, hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess)
    e = launch_init(s->descs_dev + slot, D, r->p.precision, r->d.P1, r->d.PN, r->d.P0, cdev,
                    r->has_u ? udev : nullptr,
                    reinterpret_cast<double *>(r->base + r->L.phi),
                    reinterpret_cast<double *>(r->base + r->L.C), s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) {
    release(s, r);
    return hip_fail(e, "admission");
  }
  std::vector<double>().swap(r->c);
  std::vector<double>().swap(r->u);
  r->t_admit = now_s();
  r->done_steps = 0;
  s->dirty = true;
  return NPLBM_OK;
}

// Rebuild the packed strip tables (one per (N, precision, step-kernel
// scheme) group) and recapture the quantum graph.
int rebuild(nplbm_server *s) {
  if (s->graph) {
    (void)hipGraphExecDestroy(s->graph);
    s->graph = nullptr;
  }
  s->groups.clear();
  std::vector<StripDesc> all;
  for (int sch : {kSchemeCentral, kSchemeMixed, kSchemeRemark1})
    for (int prec : {32, 64})
      for (int N = 2; N <= kMaxN; ++N) {
        std::vector<StripDesc> g;
        for (int slot = 0; slot < s->max_slots; ++slot) {
          Req *r = s->slots[slot];
          if (!r || r->p.N != N || r->p.precision != prec || step_scheme(&r->p) != sch) continue;
          build_strips(r->p.nx, r->p.ny, slot, step_geom(N, prec, sch), g);
        }
        if (g.empty()) continue;
        xcd_order(g);
        s->groups.push_back({N, prec, sch, all.size(), g.size()});
        all.insert(all.end(), g.begin(), g.end());
      }
  // the resident set is marked clean only once its graph exists: a failed
  // rebuild leaves it dirty, so the next pump tries again
  if (all.empty()) {
    s->dirty = false;
    return NPLBM_OK;
  }
  if (all.size() > s->strips_cap) {
    if (s->strips_dev) (void)hipFree(s->strips_dev);
    s->strips_dev = nullptr;
    size_t cap = std::max(all.size() * 2, (size_t)1024);
    hipError_t e = hipMalloc(&s->strips_dev, cap * sizeof(StripDesc));
    if (e != hipSuccess) {
      s->strips_cap = 0;
      return hip_fail(e, "strip table allocation");
    }
    s->strips_cap = cap;
  }
  hipError_t e = hipMemcpyAsync(s->strips_dev, all.data(), all.size() * sizeof(StripDesc),
                                hipMemcpyHostToDevice, s->stream);
  if (e != hipSuccess) return hip_fail(e, "strip table upload");
  // Groups touch disjoint domains and strip tables, so their chains of
  // launches are independent: with more than one group, each chain is
  // captured on a side stream forked from and joined back to the server's
  // stream, and the graph runs the groups concurrently (a small group no
  // longer leaves the GPU half idle for a whole launch).
  const int ngr = (int)s->groups.size();
  const int nside = ngr > 1 ? std::min(ngr, kSideStreams) : 0;
  while ((int)s->side.size() < nside) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) {
      if (st) (void)hipStreamDestroy(st);
      return hip_fail(e, "side stream creation");
    }
    s->side.push_back(st);
    s->join.push_back(ev);
  }
  if (nside && !s->fork) {
    e = hipEventCreateWithFlags(&s->fork, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "event creation");
  }
  hipGraph_t g = nullptr;
  e = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  hipError_t le = hipSuccess;
  if (nside) {
    le = hipEventRecord(s->fork, s->stream);
    for (int j = 0; j < nside && le == hipSuccess; ++j)
      le = hipStreamWaitEvent(s->side[j], s->fork, 0);
  }
  for (int q = 0; q < s->quantum && le == hipSuccess; ++q)
    for (int gi = 0; gi < ngr; ++gi) {
      const auto &gr = s->groups[gi];
      StepArgs a;
      std::memset(&a, 0, sizeof a);
      a.strips = s->strips_dev + gr.off;
      a.doms = s->descs_dev;
      a.substep = q;
      le = launch_step(gr.N, gr.precision, gr.scheme,
                       step_geom(gr.N, gr.precision, gr.scheme).bw, a, (int)gr.count,
                       nside ? s->side[gi % nside] : s->stream);
      if (le != hipSuccess) break;
    }
  for (int j = 0; j < nside && le == hipSuccess; ++j) {
    le = hipEventRecord(s->join[j], s->side[j]);
    if (le == hipSuccess) le = hipStreamWaitEvent(s->stream, s->join[j], 0);
  }
  e = hipStreamEndCapture(s->stream, &g);
  if (le != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return hip_fail(le, "step launch during capture");
  }
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&s->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    s->graph = nullptr;
    return hip_fail(e, "hipGraphInstantiate");
  }
  s->dirty = false;
  return NPLBM_OK;
}

// Publish the outcome of a request (under the mutex): done, with its
// latency recorded, or failed, with the error the admission or read-back
// raised.
void finish(nplbm_server *s, Req *r, int rc) {
  std::lock_guard<std::mutex> lk(s->mu);
  if (rc) {
    r->err = rc;
    r->msg = last_error();
    r->state = 3;
    return;
  }
  s->lat.push_back(r->t_done - r->t_submit);
  s->t_last = std::max(s->t_last, r->t_done);
  r->state = 2;
}

int retire(nplbm_server *s, Req *r) {
  const size_t n = (size_t)r->p.nx * r->p.ny;
  const int par = (int)(r->done_steps & 1);
  DomDesc D = r->desc;
  r->c_out.resize((size_t)r->p.N * n);
  r->u_out.resize(2 * n);
  r->p_out.resize(n);
  auto dp = [&](size_t off) { return reinterpret_cast<double *>(r->base + off); };
  hipError_t e = launch_macro(s->descs_dev + r->slot, D, r->p.precision, par, dp(r->L.phi),
                              dp(r->L.rho), dp(r->L.C), dp(r->L.c), dp(r->L.u), dp(r->L.p),
                              r->L.q ? dp(r->L.q) : nullptr, s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(r->c_out.data(), dp(r->L.c), r->c_out.size() * 8, hipMemcpyDeviceToHost,
                       s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(r->u_out.data(), dp(r->L.u), r->u_out.size() * 8, hipMemcpyDeviceToHost,
                       s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(r->p_out.data(), dp(r->L.p), r->p_out.size() * 8, hipMemcpyDeviceToHost,
                       s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  release(s, r);
  s->dirty = true;
  if (e != hipSuccess) return hip_fail(e, "retire");
  r->t_done = now_s();
  s->completed += 1;
  return NPLBM_OK;
}

}  // namespace

extern "C" {

int nplbm_server_create(size_t hbm_budget, int32_t max_slots, int32_t quantum, void *stream,
                        nplbm_server **out) {
  clear_error();
  if (!out) return fail(NPLBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_slots < 1 || max_slots > 4096 || quantum < 1 || quantum > 100000 || hbm_budget == 0)
    return fail(NPLBM_EINVAL, "bad server limits");
  if (!stream) return fail(NPLBM_EINVAL, "the server needs a non-null stream (graph capture)");
  nplbm_server *s = new nplbm_server();
  s->budget = hbm_budget;
  s->max_slots = max_slots;
  s->quantum = quantum;
  s->stream = static_cast<hipStream_t>(stream);
  s->slots.assign(max_slots, nullptr);
  hipError_t e = hipMalloc(&s->descs_dev, sizeof(DomDesc) * (size_t)max_slots);
  if (e != hipSuccess) {
    delete s;
    return fail(NPLBM_ENOMEM, "descriptor table allocation: %s", hipGetErrorString(e));
  }
  *out = s;
  return NPLBM_OK;
}

int nplbm_submit(nplbm_server *s, const nplbm_params *p, const double *c, const double *u,
                 int64_t nsteps, uint64_t *ticket) {
  clear_error();
  if (!s || !p || !c || !ticket) return fail(NPLBM_EINVAL, "NULL argument");
  if (nsteps < 0) return fail(NPLBM_EINVAL, "nsteps < 0");
  if (is3d(p)) return fail(NPLBM_EINVAL, "the server takes 2-D domains (nz 0 or 1)");
  Req *r = new Req();
  int rc = derive(p, r->d);
  if (rc) {
    delete r;
    return rc;
  }
  const int N = p->N;
  r->sigma.assign(p->sigma, p->sigma + N * N);
  r->rho.assign(p->rho, p->rho + N);
  r->mu.assign(p->mu, p->mu + N);
  r->mob.assign(p->mobility, p->mobility + N - 1);
  r->tau.assign(p->tau_phi, p->tau_phi + N - 1);
  r->p = *p;
  r->p.sigma = r->sigma.data();
  r->p.rho = r->rho.data();
  r->p.mu = r->mu.data();
  r->p.mobility = r->mob.data();
  r->p.tau_phi = r->tau.data();
  r->L = plan_layout(&r->p);
  r->bytes = r->L.total;
  if (r->bytes > s->budget) {
    size_t b = r->bytes;
    delete r;
    return fail(NPLBM_ETOOBIG, "request needs %zu bytes, budget is %zu", b, s->budget);
  }
  const size_t n = (size_t)p->nx * p->ny;
  for (size_t id = 0; id < n; ++id) {
    double sum = 0.0;
    for (int k = 0; k < N; ++k) sum += c[(size_t)k * n + id];
    if (!(std::fabs(sum - 1.0) <= 1e-9)) {
      delete r;
      return fail(NPLBM_EINVAL, "sum_k c_k != 1 at node %zu", id);
    }
  }
  r->c.assign(c, c + (size_t)N * n);
  if (u) {
    r->u.assign(u, u + 2 * n);
    r->has_u = true;
  }
  r->nsteps = nsteps;
  r->t_submit = now_s();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->t_first < 0.0) s->t_first = r->t_submit;
  r->ticket = s->next_ticket++;
  s->reqs[r->ticket] = r;
  s->queue.push_back(r);
  *ticket = r->ticket;
  return NPLBM_OK;
}

int nplbm_server_pump(nplbm_server *s, int32_t *active_out) {
  clear_error();
  if (!s) return fail(NPLBM_EINVAL, "NULL server");
  const double t0 = now_s();
  // admission: first fit in arrival order
  std::vector<Req *> cand;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    cand.assign(s->queue.begin(), s->queue.end());
  }
  int nres = 0;
  for (Req *r : s->slots) nres += r != nullptr;
  for (Req *r : cand) {
    if (nres >= s->max_slots) break;
    if (s->used + r->bytes > s->budget) continue;
    int rc = admit(s, r);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->queue.erase(std::find(s->queue.begin(), s->queue.end(), r));
      if (!rc) r->state = 1;
    }
    if (!rc && r->nsteps == 0) rc = retire(s, r);
    else if (!rc) ++nres;
    if (rc || r->nsteps == 0) finish(s, r, rc);
  }
  if (s->dirty) {
    int rc = rebuild(s);
    if (rc) return rc;
  }
  if (nres > 0 && !s->graph) return fail(NPLBM_ESTATE, "resident requests but no quantum graph");
  if (s->graph) {
    // per-domain progress for this quantum
    double nodes = 0;
    // host copies stay alive until the stream is synchronised below
    std::vector<int32_t> dyn(2 * (size_t)s->max_slots);
    for (int slot = 0; slot < s->max_slots; ++slot) {
      Req *r = s->slots[slot];
      if (!r) continue;
      dyn[2 * slot] = (int32_t)(r->done_steps & 1);
      dyn[2 * slot + 1] = (int32_t)std::min<int64_t>(r->nsteps - r->done_steps, INT_MAX);
      hipError_t e = hipMemcpyAsync(&s->descs_dev[slot].parity0, &dyn[2 * slot],
                                    2 * sizeof(int32_t), hipMemcpyHostToDevice, s->stream);
      if (e != hipSuccess) return hip_fail(e, "progress upload");
      const int64_t adv = std::min<int64_t>(s->quantum, r->nsteps - r->done_steps);
      nodes += (double)adv * r->p.nx * r->p.ny;
    }
    hipError_t e = hipGraphLaunch(s->graph, s->stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "quantum");
    s->node_updates += nodes;
    for (int slot = 0; slot < s->max_slots; ++slot) {
      Req *r = s->slots[slot];
      if (!r) continue;
      r->done_steps += std::min<int64_t>(s->quantum, r->nsteps - r->done_steps);
      if (r->done_steps >= r->nsteps) finish(s, r, retire(s, r));
    }
  }
  if (active_out) {
    int a = 0;
    for (Req *r : s->slots) a += r != nullptr;
    *active_out = a;
  }
  s->busy += now_s() - t0;
  return NPLBM_OK;
}

int nplbm_poll(nplbm_server *s, uint64_t ticket, int32_t *state) {
  clear_error();
  if (!s || !state) return fail(NPLBM_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(NPLBM_ENOTFOUND, "unknown ticket");
  *state = it->second->state;
  return NPLBM_OK;
}

int nplbm_result(nplbm_server *s, uint64_t ticket, double *c, double *u, double *p,
                 double *admit_s, double *done_s) {
  clear_error();
  if (!s) return fail(NPLBM_EINVAL, "NULL server");
  Req *r = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(NPLBM_ENOTFOUND, "unknown ticket");
    r = it->second;
    if (r->state == 3) {
      // a failed request is reaped here: its error is returned once
      s->reqs.erase(it);
      const int err = r->err ? r->err : NPLBM_EDEVICE;
      const std::string msg = r->msg;
      delete r;
      return fail(err, "request %llu failed: %s", (unsigned long long)ticket, msg.c_str());
    }
    if (r->state != 2) return fail(NPLBM_ESTATE, "request not finished (state %d)", r->state);
    s->reqs.erase(it);
  }
  if (c) std::memcpy(c, r->c_out.data(), r->c_out.size() * 8);
  if (u) std::memcpy(u, r->u_out.data(), r->u_out.size() * 8);
  if (p) std::memcpy(p, r->p_out.data(), r->p_out.size() * 8);
  if (admit_s) *admit_s = r->t_admit - r->t_submit;
  if (done_s) *done_s = r->t_done - r->t_submit;
  delete r;
  return NPLBM_OK;
}

int nplbm_server_stats(nplbm_server *s, double *p50_s, double *p99_s, double *mlups,
                       double *node_updates, double *busy_s, int64_t *completed) {
  clear_error();
  if (!s) return fail(NPLBM_EINVAL, "NULL server");
  std::vector<double> lat;
  double span = 0.0;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    lat = s->lat;
    span = s->t_first >= 0.0 ? s->t_last - s->t_first : 0.0;
  }
  // percentiles by linear interpolation between order statistics (rank
  // q (n - 1) of the sorted latencies)
  std::sort(lat.begin(), lat.end());
  auto pct = [&](double q) {
    if (lat.empty()) return 0.0;
    const double pos = q * (double)(lat.size() - 1);
    const size_t i = (size_t)pos;
    const double f = pos - (double)i;
    return i + 1 < lat.size() ? lat[i] + f * (lat[i + 1] - lat[i]) : lat[i];
  };
  if (p50_s) *p50_s = pct(0.50);
  if (p99_s) *p99_s = pct(0.99);
  if (mlups) *mlups = span > 0.0 ? s->node_updates / span / 1e6 : 0.0;
  if (node_updates) *node_updates = s->node_updates;
  if (busy_s) *busy_s = s->busy;
  if (completed) *completed = s->completed;
  return NPLBM_OK;
}

void nplbm_server_destroy(nplbm_server *s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  for (Req *r : s->slots)
    if (r) release(s, r);
  for (auto &kv : s->reqs) delete kv.second;
  if (s->graph) (void)hipGraphExecDestroy(s->graph);
  if (s->strips_dev) (void)hipFree(s->strips_dev);
  if (s->descs_dev) (void)hipFree(s->descs_dev);
  for (hipStream_t st : s->side) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : s->join) (void)hipEventDestroy(ev);
  if (s->fork) (void)hipEventDestroy(s->fork);
  delete s;
}

}  // extern "C"
