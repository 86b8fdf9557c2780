// sync_step_noalloc: sync_step for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// allocation).  The step's scratch -- the control block that receives the
// step monitors and one PanelStat per panel -- lives in a fixed array of
// device memory owned by the library instead of a caller workspace.
#include <hip/hip_runtime.h>

#include <mutex>

#include "device.h"
#include "host.h"
#include "nsrgs.h"

namespace nsrgs {

// The library's scratch: one copy per GPU, held until the process ends.
constexpr size_t kNoAllocScratchBytes = (size_t)NSRGS_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

static_assert(kNoAllocScratchBytes > sizeof(DevCtl), "scratch must hold the control block");

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
char *g_scratch_ptr[kMaxDevices];   // device address of `scratch` on each device
}  // namespace

// Device address of this device's copy of `scratch`, looked up once per
// device with that device current.  The array's name is a host-side stand-in
// and must never be passed to a kernel or a copy; only this address is used.
static int scratch_on_current_device(char **out) {
  int dev = 0;
  NSRGS_HIP(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(NSRGS_ERR_UNSUPPORTED, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return dev_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = static_cast<char *>(p);
  }
  *out = g_scratch_ptr[dev];
  return NSRGS_OK;
}

}  // namespace nsrgs

using namespace nsrgs;

extern "C" {

int sync_step_noalloc(const nsrgs_matrix *A, int n, int d, double mu, int ns_steps, const void *X_in,
                      void *X_out, void *stream) {
  char *base = nullptr;
  int st;
  if ((st = check_step_inputs(A, n, d, mu, ns_steps, X_in, X_out))) return st;
  if ((st = scratch_on_current_device(&base))) return st;
  // Nothing in the scratch has to start at zero: every panel writes its
  // monitors before the same call's reduction reads them, and the reduction
  // writes every control field a later call reads.
  const size_t ctl_bytes = align256(sizeof(DevCtl));
  return step_checked_into(A, n, d, mu, ns_steps, X_in, X_out, reinterpret_cast<DevCtl *>(base),
                           base + ctl_bytes, kNoAllocScratchBytes - ctl_bytes, (hipStream_t)stream);
}

}  // extern "C"
