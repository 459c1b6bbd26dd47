// The apply without allocation: pinv_apply with its scratch (split-contraction
// partials, refinement vectors, factor-only intermediates) taken from a fixed
// device array instead of the stream-ordered pool, for callers that cannot
// allocate device memory.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <unordered_map>

#include "../../include/pinv.h"
#include "pinv_internal.h"

using namespace pinv;

// Library-internal (pinv_api.hip).
pinv_status apply_items(pinv_context* c, int32_t n, const pinv_apply_item* items,
                        int32_t refine_steps, Scratch& sc, hipStream_t s);
size_t item_scratch_bytes(const pinv_plan* p, int F, int steps);
int pinv_context_device(const pinv_context* c);
pinv_status pinv_fail(pinv_status s, const std::string& msg);

// The scratch region: each GPU that loads the library holds its own copy
// until the process ends.  In host code `scratch` names a host-side stand-in,
// not a device address, so the address on each device is looked up once with
// hipGetSymbolAddress while that device is current, and only that address is
// handed to kernels.
static __device__ __align__(256) char scratch[PINV_NOALLOC_SCRATCH_BYTES];

static std::mutex g_mu;
static std::unordered_map<int, char*> g_base;   // device -> address of its scratch

// The calling thread's current device must be `device`.
static hipError_t scratch_base(int device, char** out) {
  std::lock_guard<std::mutex> g(g_mu);
  auto it = g_base.find(device);
  if (it != g_base.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_base[device] = (char*)ptr;
  *out = (char*)ptr;
  return hipSuccess;
}

extern "C" pinv_status pinv_apply_noalloc(pinv_context* c, const pinv_plan* p, const void* data,
                                          int64_t F, void* image, int32_t refine_steps,
                                          void* stream) {
  if (!c || !p) return pinv_fail(PINV_ERR_INVALID, "NULL context or plan");
  if (refine_steps < 0 || refine_steps > 4)
    return pinv_fail(PINV_ERR_INVALID, "refine_steps in 0..4");
  if (F < 0 || F > (1 << 24)) return pinv_fail(PINV_ERR_INVALID, "F out of range");
  const int device = pinv_context_device(c);
  (void)hipGetLastError();   // an error left pending by earlier calls is not this call's
  const hipError_t de = hipSetDevice(device);
  if (de != hipSuccess) return pinv_fail(PINV_ERR_DEVICE, hipGetErrorString(de));
  const size_t need = item_scratch_bytes(p, (int)F, refine_steps);
  if (need > PINV_NOALLOC_SCRATCH_BYTES)
    return pinv_fail(PINV_ERR_INVALID,
                     "this apply needs " + std::to_string(need) + " bytes of scratch; the "
                     "no-allocation entry point holds " +
                         std::to_string((size_t)PINV_NOALLOC_SCRATCH_BYTES) +
                         " (use pinv_apply, or fewer frames per call)");
  Scratch sc;
  const hipError_t se = scratch_base(device, &sc.base);
  if (se != hipSuccess)
    return pinv_fail(PINV_ERR_DEVICE, std::string("hipGetSymbolAddress: ") + hipGetErrorString(se));
  sc.cap = PINV_NOALLOC_SCRATCH_BYTES;
  pinv_apply_item it{p, data, image, F};
  return apply_items(c, 1, &it, refine_steps, sc, (hipStream_t)stream);
}
