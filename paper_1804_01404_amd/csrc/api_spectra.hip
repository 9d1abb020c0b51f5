// C ABI of the spectra and work entry points (declared in include/tddft.h).
//
// These take host arrays like the rest of the library: each call allocates
// device buffers for its inputs, outputs and the chunk partials of the
// transform, runs the kernels of k_spectra.hip on a stream of its own and
// copies the result back before it returns.
#include <cmath>
#include <cstring>
#include <string>

#include "../../include/tddft.h"
#include "internal.h"

using namespace td;

namespace {

thread_local std::string g_err = "no error";

tddft_status sfail(tddft_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

bool all_finite(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// one device allocation for every buffer of a call, freed on scope exit
struct Scratch {
  void* p = nullptr;
  hipStream_t s = nullptr;
  ~Scratch() {
    if (s) (void)hipStreamSynchronize(s);
    if (p) (void)hipFree(p);
    if (s) (void)hipStreamDestroy(s);
  }
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

#define SHIP(expr)                                                                                      \
  do {                                                                                                  \
    hipError_t e_ = (expr);                                                                             \
    if (e_ != hipSuccess) return sfail(TDDFT_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// shared by conductivity (kind 0) and oscillator strength (kind 1)
tddft_status spectrum_host(int kind, int32_t n_t, const double* x, double dt, double scale, int32_t n_w,
                           const double* om, int use_mask, int subtract_mean, double* out, double* eps) {
  if (n_t < 2 || n_w < 1 || !x || !om || !out) return sfail(TDDFT_EINVAL, "spectrum: bad sizes or null pointer");
  if (!std::isfinite(dt) || dt == 0.0 || !std::isfinite(scale))
    return sfail(TDDFT_EINVAL, "spectrum: dt must be finite and nonzero, the kick finite and nonzero");
  if (!all_finite(x, (size_t)n_t) || !all_finite(om, (size_t)n_w))
    return sfail(TDDFT_EINVAL, "spectrum: series or frequencies not finite");
  const size_t nx = align256((size_t)n_t * sizeof(double)), nwb = align256((size_t)n_w * sizeof(double));
  const size_t nout = align256((size_t)n_w * (kind == 0 ? 2 : 1) * sizeof(double));
  const size_t neps = eps ? align256((size_t)n_w * 2 * sizeof(double)) : 0;
  const size_t nscr = align256(spectrum_scratch_entries(n_t, n_w) * sizeof(double2));
  Scratch sc;
  SHIP(hipStreamCreateWithFlags(&sc.s, hipStreamNonBlocking));
  if (hipMalloc(&sc.p, nx + nwb + nout + neps + nscr) != hipSuccess) {
    (void)hipGetLastError();
    sc.p = nullptr;
    return sfail(TDDFT_ENOMEM, "spectrum: device allocation failed");
  }
  char* base = static_cast<char*>(sc.p);
  double* dx = reinterpret_cast<double*>(base);
  double* dw = reinterpret_cast<double*>(base + nx);
  double* dout = reinterpret_cast<double*>(base + nx + nwb);
  double* deps = eps ? reinterpret_cast<double*>(base + nx + nwb + nout) : nullptr;
  double2* dscr = reinterpret_cast<double2*>(base + nx + nwb + nout + neps);
  SHIP(hipMemcpyAsync(dx, x, (size_t)n_t * sizeof(double), hipMemcpyHostToDevice, sc.s));
  SHIP(hipMemcpyAsync(dw, om, (size_t)n_w * sizeof(double), hipMemcpyHostToDevice, sc.s));
  SHIP(launch_spectrum(dx, n_t, dt, dw, n_w, kind, scale, use_mask, subtract_mean, dscr, dout, deps, sc.s));
  SHIP(hipMemcpyAsync(out, dout, (size_t)n_w * (kind == 0 ? 2 : 1) * sizeof(double), hipMemcpyDeviceToHost, sc.s));
  if (eps) SHIP(hipMemcpyAsync(eps, deps, (size_t)n_w * 2 * sizeof(double), hipMemcpyDeviceToHost, sc.s));
  SHIP(hipStreamSynchronize(sc.s));
  return TDDFT_OK;
}

}  // namespace

namespace td {
void set_stateless_error(const char* msg) { g_err = msg; }
const char* stateless_error() { return g_err.c_str(); }
}  // namespace td

extern "C" {

tddft_status tddft_conductivity(int32_t n_t, const double* I, double dt, double A0, int32_t n_w, const double* omega,
                                uint32_t flags, double* sigma, double* eps) {
  if (!std::isfinite(A0) || A0 == 0.0) return sfail(TDDFT_EINVAL, "conductivity: A0 must be finite and nonzero");
  if (flags & ~(uint32_t)(TDDFT_SPECTRUM_NO_MASK | TDDFT_SPECTRUM_SUBTRACT_MEAN))
    return sfail(TDDFT_EINVAL, "conductivity: unknown flags");
  return spectrum_host(0, n_t, I, dt, -kC / A0, n_w, omega, !(flags & TDDFT_SPECTRUM_NO_MASK),
                       (flags & TDDFT_SPECTRUM_SUBTRACT_MEAN) ? 1 : 0, sigma, eps);
}

tddft_status tddft_oscillator_strength(int32_t n_t, const double* d, double dt, double F0, int32_t n_E,
                                       const double* E, double* dfdE) {
  if (!std::isfinite(F0) || F0 == 0.0) return sfail(TDDFT_EINVAL, "oscillator_strength: F0 must be finite and nonzero");
  return spectrum_host(1, n_t, d, dt, 1.0 / F0, n_E, E, 1, 0, dfdE, nullptr);
}

tddft_status tddft_work(int32_t n_t, const double* I, const double* A, double dt, double volume, double* W) {
  if (n_t < 1 || !I || !A || !W) return sfail(TDDFT_EINVAL, "work: bad size or null pointer");
  if (!std::isfinite(dt) || dt == 0.0 || !std::isfinite(volume))
    return sfail(TDDFT_EINVAL, "work: dt must be finite and nonzero, the volume finite");
  if (!all_finite(I, 3 * (size_t)n_t) || !all_finite(A, 3 * (size_t)n_t))
    return sfail(TDDFT_EINVAL, "work: series not finite");
  const size_t nb = align256(3 * (size_t)n_t * sizeof(double));
  Scratch sc;
  SHIP(hipStreamCreateWithFlags(&sc.s, hipStreamNonBlocking));
  if (hipMalloc(&sc.p, 2 * nb + align256((size_t)n_t * sizeof(double))) != hipSuccess) {
    (void)hipGetLastError();
    sc.p = nullptr;
    return sfail(TDDFT_ENOMEM, "work: device allocation failed");
  }
  char* base = static_cast<char*>(sc.p);
  double* dI = reinterpret_cast<double*>(base);
  double* dA = reinterpret_cast<double*>(base + nb);
  double* dW = reinterpret_cast<double*>(base + 2 * nb);
  SHIP(hipMemcpyAsync(dI, I, 3 * (size_t)n_t * sizeof(double), hipMemcpyHostToDevice, sc.s));
  SHIP(hipMemcpyAsync(dA, A, 3 * (size_t)n_t * sizeof(double), hipMemcpyHostToDevice, sc.s));
  SHIP(launch_work(dI, dA, n_t, dt, volume, dW, sc.s));
  SHIP(hipMemcpyAsync(W, dW, (size_t)n_t * sizeof(double), hipMemcpyDeviceToHost, sc.s));
  SHIP(hipStreamSynchronize(sc.s));
  return TDDFT_OK;
}

}  // extern "C"
