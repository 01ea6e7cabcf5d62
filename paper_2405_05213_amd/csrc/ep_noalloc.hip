// Allocation-free exp(H): the exponential of ep_expm for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops).  Its work matrices
// live in a library-owned device array, `scratch`, sized for the largest subspace (m = 256);
// each GPU the library runs on holds one copy until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ep.h"
#include "ep_expm.hpp"
#include "ep_kernels.hpp"

namespace {

constexpr int kNoAllocMaxM = 256;
// six m x ld matrices of FP64 at m = 256 (ld = 257): 3,158,016 bytes
constexpr size_t kNoAllocScratchDoubles = 6 * (size_t)kNoAllocMaxM * (kNoAllocMaxM + 1);

static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

// Device address of `scratch` on each device, looked up once per device with that device
// current (the host symbol is not a device address).
constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};

ep_status scratch_of_current_device(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return EP_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return EP_ERR_HIP;
    g_scratch[dev] = static_cast<double*>(p);
  }
  *out = g_scratch[dev];
  return EP_OK;
}

}  // namespace

extern "C" ep_status ep_expm_noalloc(int m, const double* H_dev, double* E_dev, void* hip_stream) {
  if (m < 1 || m > kNoAllocMaxM || H_dev == nullptr || E_dev == nullptr) return EP_ERR_ARG;
  if ((size_t)ep::expm_scratch(m) > kNoAllocScratchDoubles) return EP_ERR_ARG;
  double* scr = nullptr;
  const ep_status s = scratch_of_current_device(&scr);
  if (s != EP_OK) return s;
  // every entry the kernel reads is written first in the same launch: nothing to clear
  ep::launch_expm(m, H_dev, E_dev, scr, static_cast<hipStream_t>(hip_stream));
  if (hipGetLastError() != hipSuccess) return EP_ERR_HIP;
  return EP_OK;
}
