// Serving loop: continuous batching of Helmholtz solve requests.
//
// A scheduler thread owns every admitted request.  Requests are admitted in
// arrival order when their device footprint fits the HBM budget and a slot
// is free; admission queues the request's assembly, right-hand sides and
// strip factorisation on the request's own stream and does not wait for
// them.  Every tick the scheduler (1) moves requests whose factorisation has
// completed into the iterating set, (2) advances every iterating solve of
// every request by one MPGMRES iteration with the batched engine (one sweep
// launch, one SpMV launch and one set of Gram-Schmidt launches for the whole
// mix), and (3) finalises converged solves and retires finished requests,
// releasing their memory for the queue.  Results are identical to those of
// the same request run alone: every solve is an independent Krylov process
// and the batched kernels treat each task independently.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <thread>

#include "engine.h"
#include "hh_internal.h"
#include "krylov.h"

using namespace hh;

namespace {

// Krylov iterations charged at admission; a solve that runs longer charges
// each growth of its bases when it happens (Engine::set_grow_hook), and a
// growth that would exceed the budget stops that solve alone (HH_EBUDGET).
constexpr int kReserveIterations = 32;

size_t esz(int prec) { return prec == HH_FP64 ? sizeof(c128) : sizeof(c64); }

// Device bytes a request holds while running: operator, strip image, pivots,
// transmission stencils, the LU work buffer (released after factorisation but
// charged throughout), right-hand sides, and per solve the Krylov bases for
// min(maxit, kReserveIterations) iterations plus sweep scratch.  Growth past
// those iterations is charged when it happens.
size_t request_footprint(const hh_request& r) {
  const long long n = r.n, len = n * n, N = r.nstrips;
  const int nd = ((r.dirs & HH_DIR_X) ? 1 : 0) + ((r.dirs & HH_DIR_Y) ? 1 : 0);
  const long long m = (n - 1) / N;
  const size_t es = esz(r.precision);
  int kl_max = 0;
  long long img = 0, band = 0, piv = 0, ns_max = 0;
  for (long long s = 0; s < N; ++s) {
    const long long a = std::max(0LL, s * m - 1), b = std::min(n - 1, (s + 1) * m + 1);
    kl_max = std::max(kl_max, (int)(b - a + 2));
  }
  const int S = 2 * kl_max + 1 <= 64 ? 1 : 2;
  const int KP = blocked_kp(kl_max);
  const int P = sweep_segments(map_dim(KP), (int)n, es);
  for (long long s = 0; s < N; ++s) {
    const long long a = std::max(0LL, s * m - 1), b = std::min(n - 1, (s + 1) * m + 1);
    const long long w = b - a + 1, ns = n * w, kl = w + 1;
    img += strip_image_elems(ns, S, KP, (int)kl, P, sweep_wide_fits(r.precision, P, kl_max, (int)n));
    band += ns * (3 * kl + 1);
    piv += ns + HH_PAD;
    ns_max = std::max(ns_max, ns);
  }
  size_t bytes = (size_t)4 * len * sizeof(c128);
  bytes += (size_t)nd * ((img + band) * es + piv * sizeof(int) + 14 * n * N * es);
  bytes += (size_t)r.nsrc * len * sizeof(c128);  // b
  const int it = std::min(r.maxit, kReserveIterations);
  const size_t per_solve = (size_t)len * (1 + (it + 1) * nd) * sizeof(c128) +
                           (size_t)len * it * nd * es + (size_t)nd * (ns_max + N * n) * es +
                           (size_t)64 * 1024;
  return bytes + (size_t)r.nsrc * per_solve;
}

struct Request {
  uint64_t ticket = 0;
  hh_request req{};
  std::vector<double> c;
  size_t footprint = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int stage = 0;  // 0 queued, 1 factoring, 2 iterating, 3 done
  int status = HH_PENDING;
  hh_problem* pb = nullptr;
  c128* b = nullptr;
  hipEvent_t ready = nullptr;
  std::vector<std::unique_ptr<Solve>> solves;
  hh_result res{};
};

}  // namespace

struct hh_server {
  size_t budget = 0, used = 0;
  int max_active = 1;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> queue;
  std::vector<Request*> active;
  std::map<uint64_t, Request*> finished;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread th;
  hipStream_t st = nullptr;
  std::unique_ptr<Engine> engine;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  int device = 0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void loop();
  void admit(Request* r);
  void fail(Request* r, int code);
  void retire(Request* r);
};

void hh_server::fail(Request* r, int code) {
  r->status = code;
  r->stage = 3;
}

void hh_server::admit(Request* r) {
  const hh_request& q = r->req;
  r->pb = problem_create(q.omega, (int)r->c.size(), r->c.data(), q.n);
  hipStream_t ps = r->pb->st[0];
  const long long len = (long long)q.n * q.n;
  r->b = (c128*)dev_alloc((size_t)q.nsrc * len * sizeof(c128));
  launch_load_vector(q.n, q.nsrc, (const c128*)q.f, r->b, ps);
  factor_setup(r->pb, q.dirs, q.nstrips, q.precision);
  r->pb->fs.eager_batch_maps = true;  // the server's sweeps take plan 0
  factor_launch(r->pb, ps);
  HH_HIP(hipEventCreateWithFlags(&r->ready, hipEventDisableTiming));
  HH_HIP(hipEventRecord(r->ready, ps));
  r->stage = 1;
}

void hh_server::retire(Request* r) {
  int imax = 0;
  double rmax = 0;
  int status = r->status == HH_PENDING ? HH_OK : r->status;
  for (auto& s : r->solves)
    if (s->fail && (status == HH_OK || status == HH_ENOCONV)) status = s->fail;
  for (auto& s : r->solves) {
    imax = std::max(imax, s->k);
    rmax = std::max(rmax, s->res_true);
    if (!s->converged && status == HH_OK) status = HH_ENOCONV;
    Engine::release(s.get());
  }
  r->solves.clear();
  if (r->ready) (void)hipEventDestroy(r->ready);
  r->ready = nullptr;
  dev_free(r->b);
  r->b = nullptr;
  problem_destroy(r->pb);
  r->pb = nullptr;
  r->t_done = now();
  r->res.status = status;
  r->res.iterations_max = imax;
  r->res.res_true_max = rmax;
  r->res.t_submit = r->t_submit;
  r->res.t_admit = r->t_admit;
  r->res.t_done = r->t_done;
  r->stage = 3;
}

void hh_server::loop() {
  HH_HIP(hipSetDevice(device));
  for (;;) {
    std::vector<Request*> admitted;
    {
      std::unique_lock<std::mutex> lk(mu);
      const bool busy = !active.empty();
      if (!busy) cv.wait(lk, [&] { return stop || !queue.empty(); });
      if (stop && queue.empty() && active.empty()) break;
      while (!queue.empty() && (int)active.size() < max_active &&
             used + queue.front()->footprint <= budget) {
        Request* r = queue.front();
        queue.pop_front();
        used += r->footprint;
        r->t_admit = now();
        active.push_back(r);
        admitted.push_back(r);
      }
    }
    for (Request* r : admitted) {
      try {
        admit(r);
      } catch (...) {
        fail(r, HH_EDEVICE);
      }
    }
    // factorisations that completed join the iterating set
    std::vector<Solve*> joining;
    for (Request* r : active) {
      if (r->stage != 1) continue;
      if (hipEventQuery(r->ready) != hipSuccess) continue;
      int rc = factor_finish(r->pb);
      if (rc != HH_OK) {
        fail(r, rc);
        continue;
      }
      const long long len = (long long)r->req.n * r->req.n;
      for (int v = 0; v < r->req.nsrc; ++v) {
        auto s = std::make_unique<Solve>();
        s->pb = r->pb;
        s->b = r->b + v * len;
        s->x = (c128*)r->req.x + v * len;
        s->len = len;
        s->tol = r->req.tol;
        s->maxit = r->req.maxit;
        s->owner = r;
        s->charged_its = std::min(r->req.maxit, kReserveIterations);
        joining.push_back(s.get());
        r->solves.push_back(std::move(s));
      }
      r->stage = 2;
    }
    try {
      if (!joining.empty()) engine->begin(joining);
      std::vector<Solve*> running;
      for (Request* r : active)
        if (r->stage == 2)
          for (auto& s : r->solves)
            if (!s->done) running.push_back(s.get());
      if (!running.empty()) engine->step(running);
      std::vector<Solve*> ending;
      for (Request* r : active)
        if (r->stage == 2)
          for (auto& s : r->solves)
            if (s->done && !s->finalized) ending.push_back(s.get());
      if (!ending.empty()) engine->finish(ending);  // x = Z y and the FP64 residual
    } catch (...) {
      for (Request* r : active)
        if (r->stage == 2) fail(r, HH_EDEVICE);
    }
    // retire requests whose solves are all done
    std::vector<Request*> done_now;
    for (Request* r : active) {
      if (r->stage == 3) {
        done_now.push_back(r);
        continue;
      }
      if (r->stage != 2) continue;
      bool all = true;
      for (auto& s : r->solves) all &= s->finalized;
      if (all) done_now.push_back(r);
    }
    if (!done_now.empty()) {
      for (Request* r : done_now) retire(r);
      std::lock_guard<std::mutex> lk(mu);
      for (Request* r : done_now) {
        used -= r->footprint;
        active.erase(std::find(active.begin(), active.end(), r));
        finished[r->ticket] = r;
      }
      cv.notify_all();
    } else if (!admitted.empty() || !joining.empty()) {
      // progress was made; loop again immediately
    } else {
      bool iterating = false;
      for (Request* r : active) iterating |= r->stage == 2;
      if (!iterating) std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
  }
}

extern "C" {

int hh_server_create(size_t hbm_budget, int max_active, hh_server** out) {
  if (!out) return HH_EINVAL;
  *out = nullptr;
  if (max_active < 1 || hbm_budget == 0) {
    set_error("need a positive HBM budget and max_active >= 1");
    return HH_EINVAL;
  }
  try {
    auto* s = new hh_server();
    s->budget = hbm_budget;
    s->max_active = max_active;
    HH_HIP(hipGetDevice(&s->device));
    HH_HIP(hipStreamCreate(&s->st));
    s->engine = std::make_unique<Engine>(s->st);
    // one workgroup per chain whatever the mix: a plan chosen by the number
    // of chains in flight would make a result depend on what else runs
    s->engine->set_wide(false);
    s->engine->set_grow_hook([s](Solve* sv, long long delta) {
      std::lock_guard<std::mutex> lk(s->mu);
      if (delta > 0 && s->used + (size_t)delta > s->budget) return false;
      s->used = (size_t)((long long)s->used + delta);
      static_cast<Request*>(sv->owner)->footprint =
          (size_t)((long long)static_cast<Request*>(sv->owner)->footprint + delta);
      return true;
    });
    s->th = std::thread([s] {
      try {
        s->loop();
      } catch (...) {
      }
    });
    *out = s;
    return HH_OK;
  } catch (...) {
    return HH_EDEVICE;
  }
}

int hh_submit(hh_server* srv, const hh_request* req, uint64_t* ticket) {
  if (!srv || !req || !ticket) {
    set_error("invalid arguments");
    return HH_EINVAL;
  }
  const hh_request& q = *req;
  if (q.n < 3 || q.nsrc < 1 || !q.f || !q.x || q.nlayers < 1 || !q.c_layers || !(q.omega > 0) ||
      !std::isfinite(q.omega) || !(q.tol > 0) || q.maxit < 1 || q.dirs < 1 || q.dirs > 3 ||
      (q.precision != HH_FP64 && q.precision != HH_FP32) || q.nstrips < 1 ||
      (q.n - 1) % q.nstrips != 0 || (q.nstrips > 1 && (q.n - 1) / q.nstrips < 2) ||
      (q.n - 1) / q.nstrips + 4 > 63) {  // band half-width of an interior strip
    set_error("invalid request fields");
    return HH_EINVAL;
  }
  for (int l = 0; l < q.nlayers; ++l)
    if (!(q.c_layers[l] > 0) || !std::isfinite(q.c_layers[l])) {
      set_error("invalid layer speed");
      return HH_EINVAL;
    }
  auto* r = new Request();
  r->req = q;
  r->c.assign(q.c_layers, q.c_layers + q.nlayers);
  r->req.c_layers = nullptr;
  r->footprint = request_footprint(q);
  if (r->footprint > srv->budget) {
    set_error("request needs %zu bytes, budget is %zu", r->footprint, srv->budget);
    delete r;
    return HH_EBUDGET;
  }
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    r->ticket = srv->next_ticket++;
    r->t_submit = srv->now();
    srv->queue.push_back(r);
  }
  srv->cv.notify_all();
  *ticket = r->ticket;
  return HH_OK;
}

int hh_poll(hh_server* srv, uint64_t ticket, hh_result* res) {
  if (!srv || !res) return HH_EINVAL;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->finished.find(ticket);
  if (it == srv->finished.end()) {
    for (Request* r : srv->queue)
      if (r->ticket == ticket) return HH_PENDING;
    for (Request* r : srv->active)
      if (r->ticket == ticket) return HH_PENDING;
    set_error("unknown ticket %llu", (unsigned long long)ticket);
    return HH_EINVAL;
  }
  *res = it->second->res;
  delete it->second;
  srv->finished.erase(it);
  return HH_OK;
}

double hh_server_clock(const hh_server* srv) { return srv ? srv->now() : 0.0; }

int hh_server_destroy(hh_server* srv) {
  if (!srv) return HH_OK;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv.notify_all();
  if (srv->th.joinable()) srv->th.join();
  for (auto& kv : srv->finished) delete kv.second;
  srv->engine.reset();
  (void)hipStreamDestroy(srv->st);
  delete srv;
  return HH_OK;
}

}  // extern "C"
