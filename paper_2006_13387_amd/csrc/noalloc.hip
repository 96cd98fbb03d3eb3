// The CG dot product for callers that cannot allocate device memory (code
// under HIP graph capture, serving loops that forbid hipMalloc): the same
// two-stage wavefront reduction as msp_vec_dot, with its workgroup partials
// and its ticket counter in a fixed file-scope device array instead of
// buffers allocated per call, and the result left in device memory.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "common.h"
#include "msp.h"

namespace msp {
// k_vec.hip
void launch_dot(long long, const double*, const double*, double*,
                unsigned int*, double*, hipStream_t);
int dot_max_blocks();
// runtime.cpp
msp_status set_static_error(msp_status st, const std::string& msg);
}  // namespace msp

using namespace msp;

namespace {

// Partials of the dot launcher's largest grid, then one 8-byte slot whose
// low word is the workgroup ticket counter.
constexpr int kScratchParts = 1024;
constexpr int kScratchWords = kScratchParts + 1;
constexpr int kMaxDevices = 64;

// The array's name is a host-side stand-in in host code: kernels get the
// per-device address from hipGetSymbolAddress below, never the name.
static __device__ __align__(256) double scratch[kScratchWords];

std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

__global__ void k_clear_ticket(unsigned int* ticket) { *ticket = 0u; }

// Device address of this device's copy of the scratch array, looked up once
// per device with that device current.
hipError_t scratch_of_current_device(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<double*>(g_scratch_ptr[dev]);
  return hipSuccess;
}

}  // namespace

extern "C" msp_status msp_vec_dot_noalloc(int64_t n, const double* x,
                                          const double* y, double* out,
                                          hipStream_t s) {
  if (!x || !y || !out || n < 0)
    return set_static_error(MSP_E_INVALID, "msp_vec_dot_noalloc: bad argument");
  if (n > MSP_NOALLOC_DOT_MAX_N)
    return set_static_error(MSP_E_INVALID,
                            "msp_vec_dot_noalloc: n exceeds MSP_NOALLOC_DOT_MAX_N");
  if (dot_max_blocks() > kScratchParts)
    return set_static_error(MSP_E_INVALID,
                            "msp_vec_dot_noalloc: dot grid exceeds the scratch");
  double* base = nullptr;
  hipError_t e = scratch_of_current_device(&base);
  if (e != hipSuccess)
    return set_static_error(MSP_E_DEVICE, std::string("scratch lookup failed: ") +
                                              hipGetErrorString(e));
  unsigned int* ticket = reinterpret_cast<unsigned int*>(base + kScratchParts);
  // the reduction leaves the counter at zero; clear it anyway (a kernel,
  // not a memset node, so the call can be captured into a graph)
  hipLaunchKernelGGL(k_clear_ticket, dim3(1), dim3(1), 0, s, ticket);
  launch_dot(n, x, y, base, ticket, out, s);
  e = hipGetLastError();
  if (e != hipSuccess)
    return set_static_error(MSP_E_DEVICE, hipGetErrorString(e));
  return MSP_OK;
}
