// Batched execution of many independent CTD instances.
//
// Two executors.  Lockstep (the default when every instance is a 2D one
// with cyclic-reduction solves of one band width): the instances advance
// together in rounds of multi-instance launches, one launch per phase of a
// sweep for all of them and one read-back of all their scalars per round
// (solver.hip, lockstep_steps).  Worker streams (otherwise, or on request):
// a pool of worker threads, each owning a non-blocking HIP stream, takes
// instances longest-first from a shared counter and steps each one on its
// own stream, so the kernels of several instances are in flight at once.
// Either way an instance's arithmetic is that of a single ctd_solver, so its
// result does not depend on the batch around it.
#include <algorithm>
#include <atomic>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "ctd_internal.h"

struct ctd_batch {
  std::vector<ctd_solver*> inst;
  std::vector<double> cost;      // relative cost of one step (longest first)
  hipStream_t home = nullptr;    // stream the instances were set up on
  int workers = 8;
  int mode = CTD_BATCH_AUTO;
  std::string err = "no error";
};

namespace {
thread_local std::string g_batch_error = "no error";

// Relative cost of a step: the per-sweep work of the dominant phase times the
// mode cap (modes x sweeps scale alike for every instance).
double step_cost(const ctd_problem& p) {
  const double M = std::max(1, p.max_modes);
  if (p.dim == 3) {
    double nq = 0;
    for (int d = 0; d < 3; ++d) nq += 5.0 * (double)p.nodes[d];
    return M * (nq * M * M * M / 6.0 + 3e4);
  }
  const double n0 = (double)p.nodes[0], n1 = (double)p.nodes[1];
  return M * (n0 * n1 + 40.0 * (n0 + n1) * M + 3e4);
}
}  // namespace

extern "C" {

int ctd_batch_create(int32_t count, const ctd_problem* problems, const int32_t* m0,
                     const double* const* const* inits, const double* const* amps,
                     void* hip_stream, ctd_batch** out) {
  if (!out) { g_batch_error = "out is NULL"; return CTD_EINVAL; }
  *out = nullptr;
  if (count < 1 || !problems || !m0 || !inits) { g_batch_error = "empty batch"; return CTD_EINVAL; }
  ctd_batch* b = new (std::nothrow) ctd_batch();
  if (!b) return CTD_ENOMEM;
  b->home = (hipStream_t)hip_stream;
  for (int i = 0; i < count; ++i) {
    ctd_solver* s = nullptr;
    int rc = ctd_init(&problems[i], m0[i], inits[i], amps ? amps[i] : nullptr, hip_stream, &s);
    if (rc) {
      g_batch_error = "instance " + std::to_string(i) + ": " + ctd_last_error(nullptr);
      for (auto* p : b->inst) ctd_destroy(p);
      delete b;
      return rc;
    }
    b->inst.push_back(s);
    b->cost.push_back(step_cost(problems[i]));
  }
  *out = b;
  return CTD_OK;
}

int ctd_batch_set_workers(ctd_batch* b, int32_t workers) {
  if (!b || workers < 1 || workers > 64) return CTD_EINVAL;
  b->workers = workers;
  return CTD_OK;
}

namespace {
// every instance 2D, adaptive, cyclic-reduction solves, and one band width
bool lockstep_batch(const ctd_batch* b) {
  for (auto* s : b->inst)
    if (!ctd::lockstep_eligible(s) || ctd::band_halfwidth(s) != ctd::band_halfwidth(b->inst[0])) return false;
  return true;
}
}  // namespace

int ctd_batch_set_mode(ctd_batch* b, int32_t mode) {
  if (!b || (mode != CTD_BATCH_AUTO && mode != CTD_BATCH_LOCKSTEP && mode != CTD_BATCH_STREAMS))
    return CTD_EINVAL;
  if (mode == CTD_BATCH_LOCKSTEP && !lockstep_batch(b)) {
    b->err = "lockstep needs 2D instances with cyclic-reduction solves of one band width";
    return CTD_EUNSUPPORTED;
  }
  b->mode = mode;
  return CTD_OK;
}

int ctd_batch_step(ctd_batch* b, int32_t nsteps, ctd_step_info* info) {
  if (!b || nsteps < 0) return CTD_EINVAL;
  const int count = (int)b->inst.size();
  if (nsteps == 0 || count == 0) return CTD_OK;
  if (b->mode != CTD_BATCH_STREAMS && lockstep_batch(b)) {
    const int rc = ctd::lockstep_steps(b->inst, nsteps, info, b->home, b->err);
    for (auto* s : b->inst) ctd::solver_bind_stream(s, b->home);
    return rc;
  }
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return b->cost[x] > b->cost[y]; });
  const int W = std::min(b->workers, count);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) { b->err = "no device"; return CTD_EDEVICE; }
  std::vector<hipStream_t> streams(W, nullptr);
  for (int w = 0; w < W; ++w)
    if (hipStreamCreateWithFlags(&streams[w], hipStreamNonBlocking) != hipSuccess) {
      for (int v = 0; v < w; ++v) (void)hipStreamDestroy(streams[v]);
      b->err = "stream creation failed";
      return CTD_EDEVICE;
    }
  std::atomic<int> next{0};
  std::atomic<int> first_rc{CTD_OK};
  std::vector<std::string> errs(W);
  auto run = [&](int w) {
    (void)hipSetDevice(dev);
    for (;;) {
      if (first_rc.load() != CTD_OK) break;
      const int k = next.fetch_add(1);
      if (k >= count) break;
      const int i = order[k];
      ctd_solver* s = b->inst[i];
      ctd::solver_bind_stream(s, streams[w]);
      const int rc = ctd_step(s, nsteps, info ? info + (size_t)i * nsteps : nullptr);
      if (rc) {
        errs[w] = "instance " + std::to_string(i) + ": " + ctd_last_error(s);
        int expect = CTD_OK;
        first_rc.compare_exchange_strong(expect, rc);
      }
      ctd::solver_bind_stream(s, b->home);
    }
  };
  std::vector<std::thread> pool;
  for (int w = 1; w < W; ++w) pool.emplace_back(run, w);
  run(0);
  for (auto& t : pool) t.join();
  for (int w = 0; w < W; ++w) (void)hipStreamDestroy(streams[w]);
  const int rc = first_rc.load();
  if (rc != CTD_OK)
    for (const auto& e : errs)
      if (!e.empty()) { b->err = e; break; }
  return rc;
}

int ctd_batch_get_modes(ctd_batch* b, int32_t i, int32_t* m, double* amp,
                        double* const* out, int32_t cap) {
  if (!b || i < 0 || i >= (int)b->inst.size()) return CTD_EINVAL;
  return ctd_get_modes(b->inst[i], m, amp, out, cap);
}

int ctd_batch_reconstruct(ctd_batch* b, int32_t i, void* out, int32_t dtype, int32_t on_device,
                          const int64_t* strides) {
  if (!b || i < 0 || i >= (int)b->inst.size()) return CTD_EINVAL;
  return ctd_reconstruct(b->inst[i], out, dtype, on_device, strides);
}

const char* ctd_batch_last_error(const ctd_batch* b) {
  return b ? b->err.c_str() : g_batch_error.c_str();
}

void ctd_batch_destroy(ctd_batch* b) {
  if (!b) return;
  for (auto* s : b->inst) ctd_destroy(s);
  delete b;
}

}  // extern "C"
