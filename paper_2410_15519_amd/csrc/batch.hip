// Batched execution of many independent CTD instances on one stream.
#include <string>
#include <vector>

#include "ctd_internal.h"

struct ctd_batch {
  std::vector<ctd_solver*> inst;
  std::string err = "no error";
};

namespace {
thread_local std::string g_batch_error = "no error";
}

extern "C" {

int ctd_batch_create(int32_t count, const ctd_problem* problems, const int32_t* m0,
                     const double* const* const* inits, const double* const* amps,
                     void* hip_stream, ctd_batch** out) {
  if (!out) { g_batch_error = "out is NULL"; return CTD_EINVAL; }
  *out = nullptr;
  if (count < 1 || !problems || !m0 || !inits) { g_batch_error = "empty batch"; return CTD_EINVAL; }
  ctd_batch* b = new (std::nothrow) ctd_batch();
  if (!b) return CTD_ENOMEM;
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
  }
  *out = b;
  return CTD_OK;
}

int ctd_batch_step(ctd_batch* b, int32_t nsteps, ctd_step_info* info) {
  if (!b || nsteps < 0) return CTD_EINVAL;
  for (size_t i = 0; i < b->inst.size(); ++i) {
    int rc = ctd_step(b->inst[i], nsteps, info ? info + i * nsteps : nullptr);
    if (rc) {
      b->err = "instance " + std::to_string(i) + ": " + ctd_last_error(b->inst[i]);
      return rc;
    }
  }
  return CTD_OK;
}

int ctd_batch_get_modes(ctd_batch* b, int32_t i, int32_t* m, double* amp,
                        double* const* out, int32_t cap) {
  if (!b || i < 0 || i >= (int)b->inst.size()) return CTD_EINVAL;
  return ctd_get_modes(b->inst[i], m, amp, out, cap);
}

int ctd_batch_reconstruct(ctd_batch* b, int32_t i, void* out, int32_t dtype, int32_t on_device) {
  if (!b || i < 0 || i >= (int)b->inst.size()) return CTD_EINVAL;
  return ctd_reconstruct(b->inst[i], out, dtype, on_device);
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
