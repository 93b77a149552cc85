// pss_sort_noalloc: the sort of pss_sort with the library's own fixed scratch
// array as its workspace, for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  The array is a file-scope device array of
// PSS_NOALLOC_SCRATCH_BYTES; each GPU the library runs on holds its own copy
// until the process ends.  Its device address is looked up once per device
// when a context is created on that device (pss_create calls scratch_setup
// with the device current); host code uses only that address, never the
// array's name, which on the host is a stand-in and not a device address.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "../../include/pss.h"
#include "pss_internal.hpp"

static __device__ __align__(256) unsigned char scratch[PSS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t kScratchBytes = PSS_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

std::mutex g_mu;
bool g_looked_up[kMaxDevices] = {};
hipError_t g_lookup[kMaxDevices] = {};
void *g_scratch[kMaxDevices] = {};

}  // namespace

namespace pss {

hipError_t scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_looked_up[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_lookup[device] = e;
    g_scratch[device] = e == hipSuccess ? p : nullptr;
    g_looked_up[device] = true;
  }
  return g_lookup[device];
}

}  // namespace pss

extern "C" pss_status pss_sort_noalloc(pss_ctx *ctx, pss_key_t key, pss_val_t val,
                                       const void *keys_in, void *keys_out,
                                       const uint32_t *vals_in, uint32_t *vals_out, uint64_t n,
                                       uint32_t n_blocks, uint32_t n_parts, void *stream) {
  if (!ctx) {
    pss::set_thread_error("null context");
    return PSS_ERR_INVALID;
  }
  if (!pss::valid_enum(key, 5) || !pss::valid_enum(val, 1))
    return pss::ctx_fail(ctx, PSS_ERR_INVALID, "unknown key or value type");
  size_t need = 0;
  const pss_status ws = pss_workspace_bytes(ctx, key, val, n, n_blocks, n_parts, &need);
  if (ws != PSS_OK) return ws;
  if (need > kScratchBytes) {
    char m[200];
    snprintf(m, sizeof m,
             "the sort needs %zu bytes of workspace, above the %zu bytes of the library's "
             "scratch array (pass a workspace to pss_sort instead)",
             need, kScratchBytes);
    return pss::ctx_fail(ctx, PSS_ERR_WORKSPACE, m);
  }
  const int dev = pss::ctx_device(ctx);
  void *w = nullptr;
  hipError_t e = hipErrorInvalidDevice;
  if (dev >= 0 && dev < kMaxDevices) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_looked_up[dev]) {
      e = g_lookup[dev];
      w = g_scratch[dev];
    }
  }
  if (e != hipSuccess || !w) {
    char m[200];
    snprintf(m, sizeof m, "scratch array of device %d unavailable: %s", dev, hipGetErrorString(e));
    return pss::ctx_fail(ctx, PSS_ERR_HIP, m);
  }
  // no timing events inside this call: creating one may allocate
  const bool prof = pss::ctx_set_profiling(ctx, false);
  const pss_status st = pss_sort(ctx, key, val, keys_in, keys_out, vals_in, vals_out, n,
                                 n_blocks, n_parts, w, kScratchBytes, stream);
  pss::ctx_set_profiling(ctx, prof);
  return st;
}
