// pinn_jet_step_noalloc: one residual + loss + loss-gradient step of a network
// that allocates no device memory.  Its workspace is `scratch`, a static
// device array of PINN_NOALLOC_SCRATCH_BYTES that every GPU the library runs
// on holds until the process ends.  The step runs the same kernels, with the
// same default tuning, as pinn_jet_residual + pinn_jet_backward on a plan
// created for exactly N points.
//
// In host code the name `scratch` is a host-side stand-in, not a device
// address.  Host code only ever uses the address hipGetSymbolAddress returns
// for the current device, fetched once per device and kept in g_scratch.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>
#include <string>

#include "pinn_jet.h"
#include "plan_region.hpp"

namespace {

constexpr size_t kScratchBytes = (size_t)PINN_NOALLOC_SCRATCH_BYTES;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices];  // device address of `scratch` on each device

pinn_status fail_msg(pinn_status st, const char *msg) {
  pj_host::set_error(msg);
  return st;
}

// The device address of `scratch` on the current device.
pinn_status scratch_on_current_device(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) return fail_msg(PINN_ERR_DEVICE, "no usable HIP device");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      char buf[256];
      snprintf(buf, sizeof buf, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
      return fail_msg(PINN_ERR_DEVICE, buf);
    }
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return PINN_OK;
}

}  // namespace

extern "C" pinn_status pinn_jet_step_noalloc(const pinn_net *net, const pinn_pde *pde, int32_t prec,
                                             const float *x, int64_t N, float *r, float *loss, float *const *dW,
                                             float *const *db, void *stream) {
  pj_host::set_error("");
  size_t need = 0;
  pinn_status st = pj_host::plan_region_bytes(net, pde, N, prec, &need);
  if (st) return st;
  if (need > kScratchBytes) {
    char buf[256];
    snprintf(buf, sizeof buf, "workspace of %zu bytes for N = %lld exceeds the %zu-byte static scratch", need,
             (long long)N, kScratchBytes);
    return fail_msg(PINN_ERR_CAP, buf);
  }
  void *base = nullptr;
  st = scratch_on_current_device(&base);
  if (st) return st;
  pinn_plan plan = nullptr;
  st = pj_host::plan_create_in_region(net, pde, N, prec, base, kScratchBytes, &plan);
  if (st) return st;
  st = pinn_jet_residual(plan, net, pde, x, N, r, loss, nullptr, nullptr, stream);
  if (st == PINN_OK) st = pinn_jet_backward(plan, net, pde, x, N, nullptr, dW, db, nullptr, nullptr, stream);
  if (st == PINN_OK) {
    (void)pinn_plan_destroy(plan);  // host bookkeeping only: the region is not freed
    return PINN_OK;
  }
  const std::string msg = pinn_last_error();
  (void)pinn_plan_destroy(plan);
  return fail_msg(st, msg.c_str());
}
