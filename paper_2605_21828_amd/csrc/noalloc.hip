// bfmht_apply_noalloc: the synthesis f = Phi~ c of bfmht_apply with its two
// level buffers in a fixed device array that the library holds, for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).
//
// The array `scratch` below is a file-scope device variable: every GPU the
// library runs on holds its own copy (kNoallocBytes) from the first use of the
// library's code on that device until the process ends.  In host code its
// name is only a host-side stand-in, so the entry point resolves the array's
// device address once per device (hipGetSymbolAddress, with that device
// current) and passes that address to the stage kernels as their workspace,
// exactly where bfmht_apply passes the caller's buffer.  No part of the array
// needs to start at zero: every level row a stage reads was written by the
// stage before it in the same call (rows past a block are never read).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/bfmht.h"
#include "bfmht_internal.h"

namespace {

constexpr int64_t kNoallocBytes = BFMHT_NOALLOC_WORKSPACE_BYTES;
static_assert(kNoallocBytes % 256 == 0, "whole 256-byte units");

static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};   // per device: the array's device address, once resolved

// Device address of this device's array; resolved on the first call per device.
bfmht_status scratch_on(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices)
    return bfmht::set_error(BFMHT_EINVAL, "bfmht_apply_noalloc: device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
    void *ptr = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur >= 0 && cur != dev) {
      const hipError_t e2 = hipSetDevice(cur);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess || !ptr)
      return bfmht::set_error(BFMHT_EHIP, std::string("bfmht_apply_noalloc: device address of the fixed workspace: ") +
                                              hipGetErrorString(e));
    g_ptr[dev] = ptr;
  }
  *out = g_ptr[dev];
  return BFMHT_OK;
}

}  // namespace

extern "C" bfmht_status bfmht_apply_noalloc(const bfmht_plan *p, const void *c, int64_t ldc, void *f, int64_t ldf,
                                            int32_t nrhs, void *stream) {
  if (!p) return bfmht::set_error(BFMHT_EINVAL, "plan is NULL");
  if (nrhs < 0) return bfmht::set_error(BFMHT_EINVAL, "nrhs < 0");
  const int64_t need = bfmht_workspace_bytes(p, nrhs);
  if (need > kNoallocBytes)
    return bfmht::set_error(BFMHT_ENOSPACE, "bfmht_apply_noalloc: " + std::to_string(nrhs) +
                                                " right-hand sides need " + std::to_string(need) +
                                                " bytes of level buffers; the fixed device array holds " +
                                                std::to_string(kNoallocBytes));
  int dev = -1;
  hipError_t e = stream ? hipStreamGetDevice(static_cast<hipStream_t>(stream), &dev) : hipGetDevice(&dev);
  if (e != hipSuccess) return bfmht::set_error(BFMHT_EHIP, std::string("bfmht_apply_noalloc: ") + hipGetErrorString(e));
  void *ws = nullptr;
  const bfmht_status st = scratch_on(dev, &ws);
  if (st != BFMHT_OK) return st;
  return bfmht::apply_with_workspace(p, true, c, ldc, f, ldf, nrhs, ws, kNoallocBytes, stream);
}
