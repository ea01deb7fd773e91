// Entry point for callers that cannot allocate device memory: the Hermitian
// eigensolver of pw_eigh with its workspace in a static device array.
//
// Every GPU the library runs on holds one copy of `scratch` (12.6 MB, for
// matrices up to 512 x 512) until the process ends, and every call on that
// GPU shares it: calls that overlap on one GPU (two streams, two host
// threads) race on it.  The eigensolver writes every part of its workspace
// before reading it, so what an earlier call left there does not matter.
//
// On the host the array's name only stands in for the device symbol: it is
// never passed to a kernel or a copy.  The device address comes from
// hipGetSymbolAddress, once per device, with that device current, at the
// first call on the device, and is kept per device.
#include <mutex>

#include "common.h"

namespace pw {

constexpr int kNoAllocMaxM = 512;
static __device__ __align__(256) unsigned char scratch[eigh_ws_bytes(kNoAllocMaxM)];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`.
static int noalloc_scratch(void **out) {
  int dev = -1;
  PW_HIP(hipGetDevice(&dev));
  PW_CHECK_ARG(dev >= 0 && dev < kMaxDevices, PW_ERR_INVALID, "pw_eigh_noalloc: device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    PW_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    PW_CHECK_ARG(p != nullptr, PW_ERR_HIP, "pw_eigh_noalloc: no device address for the static scratch");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PW_OK;
}

}  // namespace pw

using namespace pw;

extern "C" {

pw_status pw_eigh_noalloc(const void *A, int64_t lda, int32_t m, double *w, void *Z, int64_t ldz,
                          void *stream) {
  PW_CHECK_ARG(A && w && Z && m >= 1 && lda >= m && ldz >= m, PW_ERR_INVALID,
               "pw_eigh_noalloc: bad argument");
  PW_CHECK_ARG(m <= kNoAllocMaxM, PW_ERR_INVALID,
               "pw_eigh_noalloc: m exceeds the static scratch maximum of 512 (use pw_eigh with a workspace)");
  void *work = nullptr;
  int rc = noalloc_scratch(&work);
  if (rc != PW_OK) return rc;
  rc = eigh_impl(A, lda, m, w, Z, ldz, work, static_cast<hipStream_t>(stream));
  if (rc != PW_OK) set_error("pw_eigh_noalloc: launch failed");
  return rc;
}

}  // extern "C"
