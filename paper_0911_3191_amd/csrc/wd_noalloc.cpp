// M_hat^dagger M_hat on canonical FP64 parity spinors for callers that cannot
// allocate device memory (code under graph capture, tight serving loops,
// harnesses that forbid allocation): the same operator as mdagm, with its
// four encoded scratch fields in one file-scope device array instead of a
// caller workspace.
//
// Every GPU the library runs on holds its own copy of `scratch` until the
// process ends.  Its device address is looked up once per device (with that
// device current) and kept; host code only ever passes that address, never
// the array's name, which on the host is a stand-in and not a device pointer.
// Calls on one GPU share the array: calls that overlap in time on one GPU
// (on different streams, or from different host threads) race and must be
// serialised by the caller.  Nothing in the array needs to start at zero:
// every field is written (encoded) before it is read.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "wd_internal.h"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per GPU
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on first use).
hipError_t scratch_ptr(char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[dev] = p;
  }
  *out = static_cast<char*>(g_ptr[dev]);
  return hipSuccess;
}

}  // namespace

using namespace wd;

extern "C" {

wd_status mdagm_noalloc(const wd_gauge* g, double kappa, double* out, const double* in, wd_prec prec,
                        int32_t nrhs, void* stream) {
  set_error("");
  if (!g) return fail(WD_EINVAL, "gauge handle is NULL");
  if (prec < WD_FP64 || prec > WD_HALF_F16) return fail(WD_EINVAL, "unknown precision");
  if (!(g->mask & WD_PREC_MASK(prec)) || !g->link[prec])
    return fail(WD_EINVAL, "gauge handle does not hold the requested precision");
  if (nrhs < 1 || nrhs > 65535) return fail(WD_EINVAL, "nrhs must be in [1, 65535]");
  if (!out || !in) return fail(WD_EINVAL, "out and in must be non-NULL");
  if (reinterpret_cast<uintptr_t>(out) % 256 || reinterpret_cast<uintptr_t>(in) % 256)
    return fail(WD_EINVAL, "out and in must be 256-byte aligned");
  if (!std::isfinite(kappa) || kappa <= 0) return fail(WD_EINVAL, "kappa must be finite and > 0");
  const size_t slot = operator_field_slot(g->geom, prec, nrhs);
  if (4 * slot > kScratchBytes)
    return fail(WD_EINVAL, "lattice and nrhs need " + std::to_string(4 * slot) +
                               " bytes of scratch, above the static maximum of " +
                               std::to_string(kScratchBytes) + " (use mdagm with a workspace)");
  char* ws = nullptr;
  hipError_t e = scratch_ptr(&ws);
  if (e == hipSuccess)
    e = canon_operator(g, 2, kappa, out, in, 0, 0, prec, nrhs, ws, slot, static_cast<hipStream_t>(stream),
                       /*no_tune=*/true);
  if (e != hipSuccess) return fail(WD_EDEVICE, std::string("mdagm_noalloc: ") + hipGetErrorString(e));
  return WD_OK;
}

}  // extern "C"
