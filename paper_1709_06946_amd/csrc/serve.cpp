// Serving runtime: continuous admission of independent Brownian-dynamics
// simulations onto one GPU.
//
// Requests (N, box, tolerance, grid, steps, seed, initial positions, forces)
// wait in a FIFO queue.  A request is admitted as soon as a worker slot is
// free and its device footprint (pse_footprint_bytes: grids, tables, cell
// lists, Krylov bases, particle arrays) fits in the remaining budget; it then
// owns a library handle on its own stream, keeps its state resident, and
// runs all its steps: the first synchronously, the others as replays of one
// captured graph of the whole step (one host launch per step).  Several
// admitted requests execute at once, so their kernels overlap on the
// device; requests arriving meanwhile are admitted as slots and memory free
// up.  At most one request with a large grid (kHeavyGrid) runs at a time;
// small ones run beside it.  Each step's
// completion time is recorded for latency percentiles.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <shared_mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pse.h"
#include "pse_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

// A request whose grid has this many points per side or more keeps the whole
// device busy in every stage (at 256^3 a line pass alone has 2^15 and more
// workgroups): overlapping it with others only shares the same bandwidth
// and caches, so it runs alone; smaller requests, whose launches leave most
// of the device idle, run several at a time.
constexpr int kHeavyGrid = 256;

struct Req {
  int64_t id;
  pse_request r;
  std::vector<double> x0, fl, x_out;
  std::vector<double> lat_ms;     // per-step latency
  size_t bytes = 0;
  bool heavy = false;             // grid of kHeavyGrid^3 points or more
  int status = 0;                 // 0 queued, 1 running, 2 done, <0 failed
  int rc = 0;
  std::string err;
  double t_submit = 0, t_admit = 0, t_done = 0;
};

}  // namespace

struct pse_server {
  size_t budget;
  int max_active;
  std::mutex mu;
  std::condition_variable cv_admit;   // wakes workers
  std::condition_variable cv_done;    // wakes waiters
  std::deque<std::shared_ptr<Req>> queue;
  std::map<int64_t, std::shared_ptr<Req>> all;
  size_t used = 0;
  int active = 0;
  bool heavy_active = false;          // a heavy request is running (alone)
  bool stopping = false;
  int64_t next_id = 1;
  int device = 0;
  Clock::time_point t0;
  std::vector<std::thread> workers;
  // totals
  int64_t completed = 0, failed = 0;
  double particle_steps = 0;
  size_t peak_used = 0;
  int peak_active = 0;

  double now() const {
    return std::chrono::duration<double>(Clock::now() - t0).count();
  }
};

namespace {

void run_request(pse_server *s, Req &q) {
  pse_params p{};
  p.n = q.r.n;
  p.box = q.r.box;
  p.radius = q.r.radius;
  p.viscosity = q.r.viscosity;
  p.kT = q.r.kT;
  p.tol = q.r.tol;
  p.grid = q.r.grid;
  p.precision = q.r.precision;
  p.gmres_tol = q.r.gmres_tol;
  p.lanczos_tol = q.r.lanczos_tol;
  pse_handle *h = nullptr;
  int rc = pse_create(&p, &h);
  if (rc != PSE_OK) {
    q.rc = rc;
    q.err = pse_last_error(nullptr);
    return;
  }
  const size_t n = (size_t)q.r.n;
  double *dx = nullptr, *dfl = nullptr;
  try {
    pse::dev_alloc((void **)&dx, 3 * n * sizeof(double));
    if (q.r.FL) pse::dev_alloc((void **)&dfl, 6 * n * sizeof(double));
  } catch (const pse::Error &e) {
    q.rc = PSE_ERR_NOMEM;
    q.err = "device allocation of request state failed: " + e.msg;
    pse::dev_free(dx);
    pse_destroy(h);
    return;
  }
  hipError_t ce = pse::dev_copy(dx, q.x0.data(), 3 * n * sizeof(double),
                                hipMemcpyHostToDevice);
  if (ce == hipSuccess && dfl)
    ce = pse::dev_copy(dfl, q.fl.data(), 6 * n * sizeof(double), hipMemcpyHostToDevice);
  if (ce != hipSuccess) {
    q.rc = PSE_ERR_HIP;
    q.err = std::string("copy of request inputs: ") + hipGetErrorString(ce);
    pse::dev_free(dx);
    pse::dev_free(dfl);
    pse_destroy(h);
    return;
  }
  double tprev = s->now();
  // Step 0 runs synchronously and gives the Krylov iteration counts; the
  // remaining steps are one captured graph (the whole step, device-checked
  // solves with those counts plus a margin, noise counter on the device)
  // replayed once per step, so a step costs one launch on the host.
  pse_stats st0{};
  rc = q.r.steps > 0 ? pse_constrained_step(h, dx, dfl, q.r.dt, q.r.seed, 0, nullptr, &st0)
                     : PSE_OK;
  if (q.r.steps > 0) {
    const double t = s->now();
    q.lat_ms.push_back(1e3 * (t - tprev));
    tprev = t;
  }
  if (rc < 0) {
    q.rc = rc;
    q.err = pse_last_error(h);
  } else if (rc > 0) {
    q.rc = rc;
  }
  pse_step_graph *graph = nullptr;
  pse_stats *pst = nullptr;
  if (q.rc >= 0 && q.r.steps > 1) {
    pse_derived d{};
    pse_get_derived(h, &d);
    const int passes = std::max(1, st0.refine_passes);
    // margins over the first step's counts (they barely move between steps)
    const int lz = std::min(d.lanczos_maxit, st0.lanczos_iters + 1);
    const int gm = std::min(d.gmres_restart, st0.gmres_iters / passes + 3);
    {
      std::unique_lock<std::shared_mutex> lk(pse::capture_gate());
      if (hipHostMalloc((void **)&pst, sizeof(pse_stats)) != hipSuccess) pst = nullptr;
    }
    if (pst && pse_set_krylov(h, 1, std::max(lz, 1), std::max(gm, 1), passes, 1) == PSE_OK &&
        pse_step_graph_create(h, dx, dfl, q.r.dt, q.r.seed, 1, pst, &graph) != PSE_OK)
      graph = nullptr;
    if (!graph) (void)pse_set_krylov(h, 0, 1, 1, 1, 0);   // synchronous steps instead
  }
  for (int k = 1; k < q.r.steps && q.rc >= 0; ++k) {
    if (graph) {
      rc = pse_step_graph_launch(graph);
      if (rc == PSE_OK) rc = pse_synchronize(h);
      if (rc == PSE_OK && (pst->status != 0 || !pst->converged))
        rc = pst->status != 0 ? PSE_ERR_NONFINITE : PSE_WARN_NOT_CONVERGED;
    } else {
      pse_stats st{};
      rc = pse_constrained_step(h, dx, dfl, q.r.dt, q.r.seed, (uint64_t)k, nullptr, &st);
    }
    const double t = s->now();
    q.lat_ms.push_back(1e3 * (t - tprev));
    tprev = t;
    if (rc < 0) {
      q.rc = rc;
      q.err = rc == PSE_ERR_NONFINITE && graph ? "device status: non-finite position or "
                                                 "pair list overflow"
                                               : pse_last_error(h);
      break;
    }
    if (rc > 0) q.rc = rc;
  }
  if (graph) pse_step_graph_destroy(graph);
  if (pst) {
    std::unique_lock<std::shared_mutex> lk(pse::capture_gate());
    (void)hipHostFree(pst);
  }
  q.x_out.resize(3 * n);
  ce = pse::dev_copy(q.x_out.data(), dx, 3 * n * sizeof(double), hipMemcpyDeviceToHost);
  if (ce != hipSuccess && q.rc >= 0) {
    q.rc = PSE_ERR_HIP;
    q.err = std::string("copy of request results: ") + hipGetErrorString(ce);
  }
  pse::dev_free(dx);
  pse::dev_free(dfl);
  pse_destroy(h);
}

void worker(pse_server *s) {
  (void)hipSetDevice(s->device);
  // requests are created, copied and freed here while other workers'
  // handles capture their operator graphs: relaxed capture interaction for
  // this thread (it ends with the server)
  hipStreamCaptureMode mode = hipStreamCaptureModeRelaxed;
  (void)hipThreadExchangeStreamCaptureMode(&mode);
  for (;;) {
    std::shared_ptr<Req> q;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_admit.wait(lk, [&] {
        if (s->stopping && s->queue.empty()) return true;
        if (s->queue.empty()) return false;
        if (s->active == 0) return true;
        // FIFO; one heavy request at a time (two would only share the
        // same HBM), and small requests join whatever runs, within the
        // budget and the limit on requests in flight
        if (s->queue.front()->heavy && s->heavy_active) return false;
        return s->used + s->queue.front()->bytes <= s->budget;
      });
      if (s->queue.empty()) return;   // stopping
      q = s->queue.front();
      s->queue.pop_front();
      s->used += q->bytes;
      s->active += 1;
      if (q->heavy) s->heavy_active = true;
      s->peak_used = std::max(s->peak_used, s->used);
      s->peak_active = std::max(s->peak_active, s->active);
      q->status = 1;
      q->t_admit = s->now();
    }
    run_request(s, *q);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->used -= q->bytes;
      s->active -= 1;
      if (q->heavy) s->heavy_active = false;
      q->t_done = s->now();
      q->status = q->rc < 0 ? q->rc : 2;
      if (q->rc < 0) {
        s->failed += 1;
      } else {
        s->completed += 1;
        s->particle_steps += (double)q->r.n * q->r.steps;
      }
    }
    s->cv_admit.notify_all();
    s->cv_done.notify_all();
  }
}

}  // namespace

extern "C" {

int pse_server_create(size_t budget_bytes, int max_active, pse_server **out) {
  if (!out || max_active < 1 || max_active > 64) return PSE_ERR_INVALID;
  *out = nullptr;
  pse_server *s = new (std::nothrow) pse_server();
  if (!s) return PSE_ERR_NOMEM;
  if (budget_bytes == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      delete s;
      return PSE_ERR_HIP;
    }
    budget_bytes = (size_t)(0.9 * (double)fr);
  }
  (void)hipGetDevice(&s->device);
  s->budget = budget_bytes;
  s->max_active = max_active;
  s->t0 = Clock::now();
  for (int i = 0; i < max_active; ++i) s->workers.emplace_back(worker, s);
  *out = s;
  return PSE_OK;
}

int pse_server_submit(pse_server *s, const pse_request *r, int64_t *id) {
  if (!s || !r || !id || r->n <= 0 || !r->x0 || r->steps < 0 || !(r->dt > 0))
    return PSE_ERR_INVALID;
  pse_params p{};
  p.n = r->n;
  p.box = r->box;
  p.radius = r->radius;
  p.viscosity = r->viscosity;
  p.kT = r->kT;
  p.tol = r->tol;
  p.grid = r->grid;
  p.precision = r->precision;
  p.gmres_tol = r->gmres_tol;
  p.lanczos_tol = r->lanczos_tol;
  size_t bytes = 0;
  int rc = pse_footprint_bytes(&p, &bytes);
  if (rc != PSE_OK) return rc;
  pse_derived d{};
  rc = pse_derive(&p, &d);
  if (rc != PSE_OK) return rc;
  bytes += (size_t)r->n * 9 * sizeof(double);   // request positions and forces
  if (bytes > s->budget) return PSE_ERR_NOMEM;
  auto q = std::make_shared<Req>();
  q->r = *r;
  q->x0.assign(r->x0, r->x0 + 3 * r->n);
  if (r->FL) q->fl.assign(r->FL, r->FL + 6 * r->n);
  q->r.x0 = nullptr;
  q->r.FL = r->FL ? q->fl.data() : nullptr;
  q->bytes = bytes;
  q->heavy = d.grid >= kHeavyGrid;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return PSE_ERR_INVALID;
    q->id = s->next_id++;
    q->t_submit = s->now();
    s->queue.push_back(q);
    s->all[q->id] = q;
    *id = q->id;
  }
  s->cv_admit.notify_all();
  return PSE_OK;
}

int pse_server_wait(pse_server *s, int64_t id, pse_request_info *info) {
  if (!s) return PSE_ERR_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->all.find(id);
  if (it == s->all.end()) return PSE_ERR_INVALID;
  auto q = it->second;
  s->cv_done.wait(lk, [&] { return q->status == 2 || q->status < 0; });
  if (info) {
    info->id = q->id;
    info->status = q->status == 2 ? (q->rc > 0 ? q->rc : PSE_OK) : q->status;
    info->steps_done = (int32_t)q->lat_ms.size();
    info->bytes = q->bytes;
    info->t_submit = q->t_submit;
    info->t_admit = q->t_admit;
    info->t_done = q->t_done;
  }
  return q->status < 0 ? q->status : PSE_OK;
}

int pse_server_result(pse_server *s, int64_t id, double *x_out, double *step_ms) {
  if (!s) return PSE_ERR_INVALID;
  std::shared_ptr<Req> q;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(id);
    if (it == s->all.end()) return PSE_ERR_INVALID;
    q = it->second;
    if (q->status != 2 && q->status >= 0) return PSE_ERR_INVALID;
  }
  if (x_out && !q->x_out.empty()) std::memcpy(x_out, q->x_out.data(), q->x_out.size() * 8);
  if (step_ms && !q->lat_ms.empty()) std::memcpy(step_ms, q->lat_ms.data(), q->lat_ms.size() * 8);
  return PSE_OK;
}

const char *pse_server_error(pse_server *s, int64_t id) {
  if (!s) return "";
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(id);
  if (it == s->all.end() || it->second->status >= 0) return "";
  return it->second->err.c_str();
}

int pse_server_release(pse_server *s, int64_t id) {
  if (!s) return PSE_ERR_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->all.find(id);
  if (it == s->all.end()) return PSE_ERR_INVALID;
  if (it->second->status == 0 || it->second->status == 1) return PSE_ERR_INVALID;
  s->all.erase(it);
  return PSE_OK;
}

int pse_server_stats(pse_server *s, pse_server_info *out) {
  if (!s || !out) return PSE_ERR_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  out->budget = s->budget;
  out->used = s->used;
  out->peak_used = s->peak_used;
  out->active = s->active;
  out->peak_active = s->peak_active;
  out->queued = (int32_t)s->queue.size();
  out->completed = s->completed;
  out->failed = s->failed;
  out->particle_steps = s->particle_steps;
  out->elapsed = s->now();
  return PSE_OK;
}

int pse_server_destroy(pse_server *s) {
  if (!s) return PSE_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
  }
  s->cv_admit.notify_all();
  for (auto &t : s->workers) t.join();
  delete s;
  return PSE_OK;
}

}  // extern "C"
