// Served execution with continuous batching.
//
// Requests wait in arrival order, in one of two queues by route.  2D
// requests whose steps can run in lockstep (adaptive, cyclic-reduction
// solves) go to the lockstep thread: it admits them as soon as their
// footprint fits the budget, sets each up on its own stream and adds it to
// a lockstep engine (one per band width), and runs rounds of multi-instance
// launches over every admitted request; a request joins at its first step
// and leaves when its steps are done.  The other requests (3D, and 2D ones
// that do not qualify) go to a pool of worker threads, each owning a
// non-blocking HIP stream, which admits the oldest one whenever a worker is
// idle and its footprint (the exact allocation ctd_init will make) fits,
// then sets the instance up and steps it on its stream.  Requests arriving
// while others run thus start as soon as memory (and, for the pool, a
// worker) is free, and the kernels of all running requests overlap on the
// device.  Finished requests keep their modes on the device until fetched.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ctd_internal.h"

namespace {

thread_local std::string g_server_error = "no error";
using Clock = std::chrono::steady_clock;

struct Request {
  int64_t ticket = 0;
  ctd_problem P{};
  int32_t m0 = 0, nsteps = 0;
  std::vector<double> init[3];
  std::vector<double> amp;
  uint64_t footprint = 0;
  int32_t state = CTD_REQ_QUEUED, error = 0, steps_done = 0, modes = 0;
  double t_submit = 0, t_start = 0, t_done = 0;
  ctd_solver* solver = nullptr;
  bool busy = false;   // a fetch holds the request (claimed under the lock)
  bool lockstep = false;   // routed to the lockstep thread
  std::string err;
};

// Route of a request: the lockstep engine takes 2D adaptive requests with
// cyclic-reduction solves (the directional solver of 2D under the automatic
// choice) and no full-solve fallback.
bool lockstep_route(const ctd_problem& p) {
  return p.dim == 2 && p.schedule == CTD_SCHED_ADAPTIVE && p.solve_method != CTD_SOLVE_FD && !p.actd;
}

}  // namespace

struct ctd_server {
  uint64_t budget = 0, in_use = 0;
  int device = 0;
  Clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work;   // workers: queue, memory or stop changed
  std::condition_variable cv_done;   // waiters: a request finished
  std::deque<Request*> queue;       // worker-pool route
  std::deque<Request*> queue_ls;    // lockstep route
  hipStream_t ls_stream = nullptr;
  std::thread ls_thread;
  bool use_lockstep = true;
  std::map<int64_t, std::unique_ptr<Request>> reqs;
  std::vector<hipStream_t> streams;
  std::vector<std::thread> workers;
  int64_t next_ticket = 1, submitted = 0, completed = 0, failed = 0, running = 0, steps_total = 0;
  double busy_ms = 0, busy_since = 0;
  bool stop = false;
  std::string err = "no error";
  double now_ms() const {
    return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
  }
};

namespace {

// Mark a request finished (under the lock).
void finish_locked(ctd_server* S, Request* r, int rc, const std::string& msg) {
  r->t_done = S->now_ms();
  if (rc) {
    r->state = CTD_REQ_FAILED;
    r->error = rc;
    r->err = msg;
    S->in_use -= r->footprint;
    ++S->failed;
  } else {
    r->state = CTD_REQ_DONE;
    ++S->completed;
  }
  if (--S->running == 0) S->busy_ms += r->t_done - S->busy_since;
}

void worker_main(ctd_server* S, int w) {
  (void)hipSetDevice(S->device);
  hipStream_t st = S->streams[w];
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] {
        return S->stop ||
               (!S->queue.empty() && S->in_use + S->queue.front()->footprint <= S->budget);
      });
      if (S->stop) return;
      r = S->queue.front();
      S->queue.pop_front();
      S->in_use += r->footprint;
      r->state = CTD_REQ_RUNNING;
      r->t_start = S->now_ms();
      if (S->running++ == 0) S->busy_since = r->t_start;
    }
    const double* ip[3] = {r->init[0].data(), r->init[1].data(), r->init[2].data()};
    std::string msg;
    int rc = ctd_init(&r->P, r->m0, ip, r->amp.empty() ? nullptr : r->amp.data(), st, &r->solver);
    if (rc) msg = ctd_last_error(nullptr);
    for (int k = 0; rc == CTD_OK && k < r->nsteps; ++k) {
      ctd_step_info info{};
      rc = ctd_step(r->solver, 1, &info);
      if (rc) {
        msg = ctd_last_error(r->solver);
        break;
      }
      std::lock_guard<std::mutex> lk(S->mu);
      r->steps_done = k + 1;
      r->modes = info.modes;
      ++S->steps_total;
      if (S->stop) { rc = CTD_ESTATE; msg = "server stopped"; }
    }
    if (rc) {
      ctd_destroy(r->solver);
      r->solver = nullptr;
    }
    for (auto& v : r->init) std::vector<double>().swap(v);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      finish_locked(S, r, rc, msg);
    }
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
}

void lockstep_main(ctd_server* S) {
  (void)hipSetDevice(S->device);
  hipStream_t st = S->ls_stream;
  std::map<int, std::unique_ptr<ctd::Lockstep>> engines;   // by band half-width
  std::map<std::pair<int, int>, Request*> running;          // (band, slot) -> request
  std::vector<std::pair<int, ctd_step_info>> steps;
  std::vector<int> finished;
  std::vector<std::pair<int, int>> failed;
  for (;;) {
    std::vector<Request*> admit;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      auto can_admit = [&] {
        return !S->queue_ls.empty() && S->in_use + S->queue_ls.front()->footprint <= S->budget;
      };
      S->cv_work.wait(lk, [&] { return S->stop || can_admit() || !running.empty(); });
      if (S->stop) break;
      while (can_admit()) {
        Request* r = S->queue_ls.front();
        S->queue_ls.pop_front();
        S->in_use += r->footprint;
        r->state = CTD_REQ_RUNNING;
        r->t_start = S->now_ms();
        if (S->running++ == 0) S->busy_since = r->t_start;
        admit.push_back(r);
      }
    }
    // set-up of the admitted requests (their own stream: the engine's)
    for (Request* r : admit) {
      const double* ip[3] = {r->init[0].data(), r->init[1].data(), r->init[2].data()};
      std::string msg;
      int rc = ctd_init(&r->P, r->m0, ip, r->amp.empty() ? nullptr : r->amp.data(), st, &r->solver);
      if (rc) msg = ctd_last_error(nullptr);
      for (auto& v : r->init) std::vector<double>().swap(v);
      int slot = -1, band = 0;
      if (rc == CTD_OK && r->nsteps > 0) {
        band = 2 * r->P.patch_s + 1;
        auto& e = engines[band];
        if (!e) e.reset(new ctd::Lockstep(st));
        rc = e->add(r->solver, r->nsteps, &slot, msg);
      }
      if (rc == CTD_OK && r->nsteps > 0) {
        running[{band, slot}] = r;
        continue;
      }
      if (rc && r->solver) {
        ctd_destroy(r->solver);
        r->solver = nullptr;
      }
      {
        std::lock_guard<std::mutex> lk(S->mu);
        finish_locked(S, r, rc, msg);
      }
      S->cv_done.notify_all();
      S->cv_work.notify_all();
    }
    // one round of every engine with requests in it
    for (auto& kv : engines) {
      if (kv.second->empty()) continue;
      steps.clear();
      finished.clear();
      failed.clear();
      std::string msg;
      const int rc = kv.second->round(steps, finished, msg, &failed);
      std::lock_guard<std::mutex> lk(S->mu);
      for (auto& f : failed) {
        Request* r = running[{kv.first, f.first}];
        running.erase({kv.first, f.first});
        const std::string m = ctd_last_error(r->solver);
        ctd_destroy(r->solver);
        r->solver = nullptr;
        finish_locked(S, r, f.second, m);
      }
      for (auto& si : steps) {
        Request* r = running[{kv.first, si.first}];
        ++r->steps_done;
        r->modes = si.second.modes;
        ++S->steps_total;
      }
      for (int slot : finished) {
        Request* r = running[{kv.first, slot}];
        running.erase({kv.first, slot});
        finish_locked(S, r, CTD_OK, "");
      }
      if (rc) {
        // a failed round leaves the engine's instances in an unknown state:
        // every request in it fails
        for (auto it = running.begin(); it != running.end();) {
          if (it->first.first != kv.first) { ++it; continue; }
          Request* r = it->second;
          ctd_destroy(r->solver);
          r->solver = nullptr;
          finish_locked(S, r, rc, msg);
          it = running.erase(it);
        }
        kv.second.reset(new ctd::Lockstep(st));
      }
    }
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
  // stopped: requests still running fail
  std::lock_guard<std::mutex> lk(S->mu);
  for (auto& kv : running) finish_locked(S, kv.second, CTD_ESTATE, "server stopped");
}

Request* find(ctd_server* S, int64_t ticket) {
  auto it = S->reqs.find(ticket);
  return it == S->reqs.end() ? nullptr : it->second.get();
}

}  // namespace

extern "C" {

int ctd_server_create(uint64_t budget_bytes, int32_t workers, ctd_server** out) {
  if (!out) { g_server_error = "out is NULL"; return CTD_EINVAL; }
  *out = nullptr;
  if (workers < 1 || workers > 64) { g_server_error = "workers must be in [1, 64]"; return CTD_EINVAL; }
  if (ctd::configure_kernels() != hipSuccess) { g_server_error = "no HIP device"; return CTD_EDEVICE; }
  auto* S = new (std::nothrow) ctd_server();
  if (!S) return CTD_ENOMEM;
  S->t0 = Clock::now();
  (void)hipGetDevice(&S->device);
  if (budget_bytes == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) { delete S; g_server_error = "hipMemGetInfo failed"; return CTD_EDEVICE; }
    budget_bytes = (uint64_t)(0.8 * (double)fr);
  }
  S->budget = budget_bytes;
  S->streams.assign(workers, nullptr);
  for (int w = 0; w < workers; ++w)
    if (hipStreamCreateWithFlags(&S->streams[w], hipStreamNonBlocking) != hipSuccess) {
      for (int v = 0; v < w; ++v) (void)hipStreamDestroy(S->streams[v]);
      delete S;
      g_server_error = "stream creation failed";
      return CTD_EDEVICE;
    }
  if (hipStreamCreateWithFlags(&S->ls_stream, hipStreamNonBlocking) != hipSuccess) {
    for (hipStream_t st : S->streams) (void)hipStreamDestroy(st);
    delete S;
    g_server_error = "stream creation failed";
    return CTD_EDEVICE;
  }
  for (int w = 0; w < workers; ++w) S->workers.emplace_back(worker_main, S, w);
  S->ls_thread = std::thread(lockstep_main, S);
  *out = S;
  return CTD_OK;
}

int ctd_server_submit(ctd_server* S, const ctd_problem* p, int32_t m0, const double* const* init,
                      const double* amp, int32_t nsteps, int64_t* ticket) {
  if (!S || !p || !init || !ticket || m0 < 1 || nsteps < 0) return CTD_EINVAL;
  uint64_t fp = 0;
  int rc = ctd_footprint_bytes(p, m0, &fp);
  if (rc) {
    std::lock_guard<std::mutex> lk(S->mu);
    S->err = "invalid problem";
    return rc;
  }
  auto r = std::make_unique<Request>();
  r->P = *p;
  r->m0 = m0;
  r->nsteps = nsteps;
  r->footprint = fp;
  for (int d = 0; d < p->dim; ++d) {
    if (!init[d]) return CTD_EINVAL;
    r->init[d].assign(init[d], init[d] + (size_t)p->nodes[d] * m0);
  }
  if (amp) r->amp.assign(amp, amp + m0);
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->stop) return CTD_ESTATE;
  if (fp > S->budget) {
    S->err = "request footprint exceeds the server budget";
    return CTD_ENOMEM;
  }
  r->ticket = S->next_ticket++;
  r->t_submit = S->now_ms();
  *ticket = r->ticket;
  r->lockstep = S->use_lockstep && lockstep_route(r->P);
  (r->lockstep ? S->queue_ls : S->queue).push_back(r.get());
  S->reqs[r->ticket] = std::move(r);
  ++S->submitted;
  S->cv_work.notify_all();
  return CTD_OK;
}

int ctd_server_status(ctd_server* S, int64_t ticket, ctd_request_status* st) {
  if (!S || !st) return CTD_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  Request* r = find(S, ticket);
  if (!r) { S->err = "unknown ticket"; return CTD_EINVAL; }
  st->state = r->state;
  st->steps_done = r->steps_done;
  st->modes = r->modes;
  st->error = r->error;
  st->t_submit_ms = r->t_submit;
  st->t_start_ms = r->t_start;
  st->t_done_ms = r->t_done;
  st->footprint = r->footprint;
  if (r->state == CTD_REQ_FAILED) S->err = r->err;
  return CTD_OK;
}

int ctd_server_wait(ctd_server* S, int64_t ticket, double timeout_ms) {
  if (!S) return CTD_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  Request* r = find(S, ticket);
  if (!r) { S->err = "unknown ticket"; return CTD_EINVAL; }
  auto done = [&] { return r->state == CTD_REQ_DONE || r->state == CTD_REQ_FAILED; };
  if (timeout_ms < 0) {
    S->cv_done.wait(lk, done);
  } else if (!S->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), done)) {
    return CTD_EAGAIN;
  }
  if (r->state == CTD_REQ_FAILED) { S->err = r->err; return r->error; }
  return CTD_OK;
}

int ctd_server_fetch(ctd_server* S, int64_t ticket, int32_t* m, double* amp, double* const* out,
                     int32_t cap, int32_t release) {
  if (!S || !m) return CTD_EINVAL;
  Request* r = nullptr;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    r = find(S, ticket);
    if (!r) { S->err = "unknown ticket"; return CTD_EINVAL; }
    if (r->state == CTD_REQ_FAILED) {
      // its device memory went back at failure; release forgets the ticket
      S->err = r->err;
      const int code = r->error;
      if (release && !r->busy) S->reqs.erase(ticket);
      return code;
    }
    if (r->state != CTD_REQ_DONE) { S->err = "request not done"; return CTD_EAGAIN; }
    if (r->busy) { S->err = "request is being fetched by another thread"; return CTD_EAGAIN; }
    // claimed: no worker touches a DONE request and no other fetch may now
    r->busy = true;
  }
  int rc = ctd_get_modes(r->solver, m, amp, out, cap);
  if (rc || !release) {
    std::lock_guard<std::mutex> lk(S->mu);
    if (rc) S->err = ctd_last_error(r->solver);
    r->busy = false;
    return rc;
  }
  // the worker stream may already run another request: free on the null
  // stream (the worker streams are non-blocking, so this waits for nothing
  // of theirs; the request's own work finished before it was marked done)
  ctd::solver_bind_stream(r->solver, nullptr);
  ctd_destroy(r->solver);
  r->solver = nullptr;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->in_use -= r->footprint;
    S->reqs.erase(ticket);
  }
  S->cv_work.notify_all();
  return CTD_OK;
}

int ctd_server_get_stats(ctd_server* S, ctd_server_stats* st) {
  if (!S || !st) return CTD_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  st->submitted = S->submitted;
  st->completed = S->completed;
  st->failed = S->failed;
  st->queued = (int64_t)(S->queue.size() + S->queue_ls.size());
  st->running = S->running;
  st->bytes_in_use = S->in_use;
  st->budget = S->budget;
  st->steps_done = S->steps_total;
  st->busy_ms = S->busy_ms + (S->running ? S->now_ms() - S->busy_since : 0.0);
  return CTD_OK;
}

const char* ctd_server_last_error(const ctd_server* S) {
  return S ? S->err.c_str() : g_server_error.c_str();
}

void ctd_server_destroy(ctd_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  for (auto& t : S->workers) t.join();
  if (S->ls_thread.joinable()) S->ls_thread.join();
  for (auto& kv : S->reqs)
    if (kv.second->solver) ctd_destroy(kv.second->solver);
  for (hipStream_t st : S->streams) (void)hipStreamDestroy(st);
  if (S->ls_stream) (void)hipStreamDestroy(S->ls_stream);
  delete S;
}

int ctd_server_set_lockstep(ctd_server* S, int32_t on) {
  if (!S) return CTD_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  S->use_lockstep = on != 0;
  return CTD_OK;
}

}  // extern "C"
