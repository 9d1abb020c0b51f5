// Allocation-free variant of tddft_conductivity (declared in include/tddft.h)
// for callers that cannot allocate device memory: code under stream capture,
// tight serving loops. Inputs and outputs are device arrays of the caller; the
// chunk partials and the mean of the transform live in a fixed file-scope
// device array, one copy per GPU, held until the process ends.
#include <cmath>
#include <mutex>
#include <string>

#include "../../include/tddft.h"
#include "internal.h"

using namespace td;

namespace {
constexpr size_t kScratchBytes = (size_t)8 << 20;  // 8 MiB per GPU
constexpr size_t kScratchEntries = kScratchBytes / sizeof(double2);
constexpr int kMaxDevices = 64;
}  // namespace

// Host code never passes this name to a kernel: the device address of each
// GPU's copy comes from hipGetSymbolAddress below.
static __device__ __align__(256) double2 scratch[kScratchEntries];

namespace {

std::mutex g_mu;
double2* g_ptr[kMaxDevices] = {};

// The device address of the current GPU's copy, looked up once per device
// with that device current.
tddft_status scratch_for_current_device(double2** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    set_stateless_error((std::string("conductivity_noalloc: hipGetDevice: ") + hipGetErrorString(e)).c_str());
    return TDDFT_EDEVICE;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    set_stateless_error("conductivity_noalloc: device index beyond the supported 64");
    return TDDFT_EDEVICE;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_stateless_error((std::string("conductivity_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e)).c_str());
      return TDDFT_EDEVICE;
    }
    g_ptr[dev] = static_cast<double2*>(p);
  }
  *out = g_ptr[dev];
  return TDDFT_OK;
}

}  // namespace

extern "C" {

tddft_status tddft_conductivity_noalloc(int32_t n_t, const double* I, double dt, double A0, int32_t n_w,
                                        const double* omega, uint32_t flags, double* sigma, double* eps,
                                        void* stream) {
  if (n_t < 2 || n_w < 1 || !I || !omega || !sigma) {
    set_stateless_error("conductivity_noalloc: bad sizes or null pointer");
    return TDDFT_EINVAL;
  }
  if (!std::isfinite(dt) || dt == 0.0 || !std::isfinite(A0) || A0 == 0.0) {
    set_stateless_error("conductivity_noalloc: dt and A0 must be finite and nonzero");
    return TDDFT_EINVAL;
  }
  if (flags & ~(uint32_t)(TDDFT_SPECTRUM_NO_MASK | TDDFT_SPECTRUM_SUBTRACT_MEAN)) {
    set_stateless_error("conductivity_noalloc: unknown flags");
    return TDDFT_EINVAL;
  }
  if (spectrum_scratch_entries(n_t, n_w) > kScratchEntries) {
    set_stateless_error("conductivity_noalloc: 1 + chunks * n_w exceeds the fixed 8 MiB workspace "
                        "(n_w <= 8191 for series of 16384 samples or more)");
    return TDDFT_EINVAL;
  }
  double2* scr = nullptr;
  tddft_status st = scratch_for_current_device(&scr);
  if (st != TDDFT_OK) return st;
  hipError_t e = launch_spectrum(I, n_t, dt, omega, n_w, 0, -kC / A0, !(flags & TDDFT_SPECTRUM_NO_MASK),
                                 (flags & TDDFT_SPECTRUM_SUBTRACT_MEAN) ? 1 : 0, scr, sigma, eps,
                                 static_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    set_stateless_error((std::string("conductivity_noalloc: launch: ") + hipGetErrorString(e)).c_str());
    return TDDFT_EDEVICE;
  }
  return TDDFT_OK;
}

}  // extern "C"
