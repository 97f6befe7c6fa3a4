// Allocation-free variant of the batched banded solve (ctd_kernel_band_solve)
// for callers that cannot allocate device memory: its workspace (the
// cyclic-reduction block data of systems too large for LDS) is a file-scope
// device array of fixed size instead of a stream-ordered allocation.  The
// array's device address is looked up once per device and kept; host code
// uses only that address.  Every call on a device shares the array, so calls
// that overlap on one device race (see include/ctd.h).
#include <mutex>

#include "ctd_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)CTD_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (set up on first use).
hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" int ctd_kernel_band_solve_noalloc(int32_t n, int32_t bw, const double* Mb,
                                             const double* Kb, const double* alpha,
                                             const double* beta, const double* b, double* x,
                                             int32_t count, void* hip_stream) {
  if (n < bw + 1 || (bw != 3 && bw != 5 && bw != 7) || count < 0) return CTD_EINVAL;
  if (!Mb || !Kb || !alpha || !beta || !b || !x) return CTD_EINVAL;
  if (count == 0) return CTD_OK;
  if (ctd::configure_kernels() != hipSuccess) return CTD_EDEVICE;
  const size_t need = ctd::band_solve_workspace_bytes(n, bw, count);
  if (need > kScratchBytes) return CTD_ENOMEM;
  double* ws = nullptr;
  if (need) {
    void* p = nullptr;
    if (scratch_address(&p) != hipSuccess) return CTD_EDEVICE;
    ws = (double*)p;
  }
  const hipError_t e = ctd::launch_band_solve_batch_ws(n, bw, Mb, Kb, alpha, beta, b, x, count, ws,
                                                       (hipStream_t)hip_stream);
  return e == hipSuccess ? CTD_OK : CTD_EDEVICE;
}
