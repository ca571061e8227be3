// Allocation-free variant of fbsde_forward_backward: the workspace is a
// file-scope device array instead of a caller-supplied buffer.
//
// Each GPU the library runs on holds its own copy of `scratch` (a code-object
// global, allocated when the runtime loads the code object on that device and
// held until the process ends).  Host code never uses the array's name as an
// address: the device address of each GPU's copy is looked up once per
// device with hipGetSymbolAddress (under a lock, with that device current)
// and kept; kernels receive that pointer exactly as they receive a caller's
// workspace in fbsde_forward_backward, whose launch sequence this call
// shares.
//
// Every call on one GPU uses the same array and it keeps the previous call's
// contents.  The launch sequence writes every workspace word it later reads
// within the same call (the scan clears the non-finite flag it shares with
// the reductions; the gradient partials are written in full), so no clearing
// pass is needed.  Calls that overlap in time on one GPU (different streams,
// threads or plans) race on the array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fbsde_internal.h"

namespace {

constexpr size_t kScratchBytes = FBSDE_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_lock;
void* g_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (nullptr on a
// HIP error, reported through *err).
void* scratch_ptr(int dev, hipError_t* err) {
  std::lock_guard<std::mutex> guard(g_lock);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
      *err = e;
      return nullptr;
    }
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

}  // namespace

extern "C" fbsde_status fbsde_forward_backward_noalloc(fbsde_plan* plan, const float* params_dev,
                                                       const double* y0_dev, float* grad_dev,
                                                       double* grad_y0_dev, double* loss_dev, uint64_t seed,
                                                       uint64_t iter, void* stream) {
  if (!plan) return fbsde::api_fail(FBSDE_ERR_INVALID, "plan is NULL");
  size_t need = 0;
  int plan_dev = -1;
  fbsde_status st = fbsde::api_active_workspace(plan, &need, &plan_dev);
  if (st != FBSDE_OK) return st;
  if (need > kScratchBytes)
    return fbsde::api_fail(FBSDE_ERR_UNSUPPORTED,
                               "fbsde_forward_backward_noalloc: the plan's workspace exceeds the "
                               "library's static scratch (FBSDE_NOALLOC_SCRATCH_BYTES); use "
                               "fbsde_forward_backward with a caller workspace");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fbsde::api_fail(FBSDE_ERR_HIP, hipGetErrorString(e));
  if (dev != plan_dev)
    return fbsde::api_fail(FBSDE_ERR_INVALID,
                               "fbsde_forward_backward_noalloc: make the plan's device current");
  if (dev < 0 || dev >= kMaxDevices) return fbsde::api_fail(FBSDE_ERR_UNSUPPORTED, "device index too large");
  void* ws = scratch_ptr(dev, &e);
  if (!ws) return fbsde::api_fail(FBSDE_ERR_HIP, hipGetErrorString(e));
  return fbsde_forward_backward(plan, params_dev, y0_dev, grad_dev, grad_y0_dev, loss_dev, seed, iter, ws,
                                stream);
}
