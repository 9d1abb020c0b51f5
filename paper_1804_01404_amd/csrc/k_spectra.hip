// Spectra and the work of the field from the time series of one run.
//
// * masked Fourier transform of a real series x(t_n), t_n = n dt:
//     Z(w) = sum_n c_n f(t_n / T) (x_n - xbar) exp(i w t_n),
//   trapezoid weights c_n (dt, halved at both ends), T = t_{N-1}, the cubic
//   mask f(u) = 1 - 3u^2 + 2u^3 (Sec. 3.1) or none, xbar the sample mean or 0.
//   The conductivity is sigma = -(c / A0) Z of the current after a kick A0
//   (Sec. 4.1, Eq. sigma_ft; the mean subtraction is the DC correction of
//   Sec. 4.2), the dielectric function eps = 1 + 4 pi i sigma / w (Sec. 4.1),
//   and the oscillator-strength distribution df/dE = (2E / pi) Im Z / F0 of
//   the dipole after a kick F0 (Sec. 3.1, Eq. distribution).
// * the work of the field on the electrons (Sec. 4.1, the excitation energy
//   for potentials without an energy functional):
//     W_n = volume sum_{m<n} dt (I_m + I_{m+1}) / 2 . E_m,
//     E_m = -(A_{m+1} - A_m) / (c dt).
// Every sum runs in a fixed order: the results do not depend on timing.
#include "internal.h"

namespace td {

// sample mean of x[0..n) (one workgroup; contiguous blocks per thread, then a
// fixed tree over the threads)
__global__ __launch_bounds__(1024) void k_series_mean(const double* __restrict__ x, int n, double* __restrict__ mean) {
  __shared__ double red[1024];
  const int t = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int i0 = t * per, i1 = min(n, i0 + per);
  double s = 0.0;
  for (int i = i0; i < i1; ++i) s += x[i];
  red[t] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) *mean = red[0] / (double)n;
}

// Part of Z(w_j) over the samples of chunk c: one thread per frequency; the
// chunk's weighted samples are staged in LDS 1024 at a time and read by every
// thread in sample order.
__global__ __launch_bounds__(kSpecThreads) void k_spec_partial(const double* __restrict__ x, int n, double dt,
                                                               const double* __restrict__ om, int n_w, int chunk,
                                                               int use_mask, const double* __restrict__ mean,
                                                               double2* __restrict__ part) {
  __shared__ double wx[1024];
  const int j = blockIdx.x * kSpecThreads + threadIdx.x;
  const int c = blockIdx.y;
  const int n0 = c * chunk, n1 = min(n, n0 + chunk);
  const double xbar = mean ? *mean : 0.0;
  const double w = j < n_w ? om[j] : 0.0;
  const double T = (double)(n - 1) * dt;
  double zr = 0.0, zi = 0.0;
  for (int b = n0; b < n1; b += 1024) {
    const int nb = min(1024, n1 - b);
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += kSpecThreads) {
      const int m = b + i;
      const double t = (double)m * dt;
      double f = 1.0;
      if (use_mask) {
        const double u = t / T;
        f = 1.0 - 3.0 * (u * u) + 2.0 * (u * u * u);
      }
      const double cw = (m == 0 || m == n - 1) ? 0.5 * dt : dt;
      wx[i] = cw * f * (x[m] - xbar);
    }
    __syncthreads();
    if (j < n_w) {
      for (int i = 0; i < nb; ++i) {
        double s, co;
        sincos(w * ((double)(b + i) * dt), &s, &co);
        zr += wx[i] * co;
        zi += wx[i] * s;
      }
    }
  }
  if (j < n_w) part[(size_t)c * n_w + j] = make_double2(zr, zi);
}

// Z(w_j) = sum over chunks in order, then the output of the kind:
// kind 0: sigma = scale Z as (re, im), and eps (may be null);
// kind 1: df/dE = (2 E / pi) Im Z * scale with scale = 1 / F0
__global__ void k_spec_final(const double2* __restrict__ part, int n_chunks, int n_w, const double* __restrict__ om,
                             int kind, double scale, double* __restrict__ out, double* __restrict__ eps) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_w) return;
  double zr = 0.0, zi = 0.0;
  for (int c = 0; c < n_chunks; ++c) {
    const double2 p = part[(size_t)c * n_w + j];
    zr += p.x;
    zi += p.y;
  }
  const double w = om[j];
  if (kind == 0) {
    const double sr = scale * zr, si = scale * zi;
    out[2 * j] = sr;
    out[2 * j + 1] = si;
    if (eps) {  // 1 + 4 pi i (sr + i si) / w
      eps[2 * j] = 1.0 - 4.0 * M_PI * si / w;
      eps[2 * j + 1] = 4.0 * M_PI * sr / w;
    }
  } else {
    out[j] = 2.0 * w / M_PI * zi * scale;
  }
}

int spec_chunks(int n_t) { return std::min(kSpecChunksMax, (n_t + 255) / 256); }

hipError_t launch_spectrum(const double* x, int n_t, double dt, const double* om, int n_w, int kind, double scale,
                           int use_mask, int subtract_mean, double2* scratch, double* out, double* eps,
                           hipStream_t s) {
  const int nc = spec_chunks(n_t);
  const int chunk = (n_t + nc - 1) / nc;
  double* mean = reinterpret_cast<double*>(scratch);
  double2* part = scratch + 1;
  if (subtract_mean) hipLaunchKernelGGL(k_series_mean, dim3(1), dim3(1024), 0, s, x, n_t, mean);
  const dim3 grid((unsigned)((n_w + kSpecThreads - 1) / kSpecThreads), (unsigned)nc);
  hipLaunchKernelGGL(k_spec_partial, grid, dim3(kSpecThreads), 0, s, x, n_t, dt, om, n_w, chunk, use_mask,
                     subtract_mean ? mean : (const double*)nullptr, part);
  hipLaunchKernelGGL(k_spec_final, dim3((unsigned)((n_w + 255) / 256)), dim3(256), 0, s, part, nc, n_w, om, kind,
                     scale, out, eps);
  return hipGetLastError();
}

size_t spectrum_scratch_entries(int n_t, int n_w) { return 1 + (size_t)spec_chunks(n_t) * n_w; }

// W_n for n = 0 .. n_t - 1 (one workgroup): thread t forms the increments of a
// contiguous block and their running sum, the block totals are scanned in
// order by one thread, then each block adds its offset.
__global__ __launch_bounds__(1024) void k_work(const double* __restrict__ I, const double* __restrict__ A, int n_t,
                                               double dt, double volume, double* __restrict__ W) {
  __shared__ double tot[1024];
  const int t = threadIdx.x;
  const int n_inc = n_t - 1;
  const int per = (n_inc + 1023) / 1024;
  const int m0 = t * per, m1 = min(n_inc, m0 + per);
  double run = 0.0;
  for (int m = m0; m < m1; ++m) {
    double s = 0.0;
    for (int mu = 0; mu < 3; ++mu) {
      const double E = -(A[3 * (size_t)(m + 1) + mu] - A[3 * (size_t)m + mu]) / (kC * dt);
      s += 0.5 * (I[3 * (size_t)m + mu] + I[3 * (size_t)(m + 1) + mu]) * E;
    }
    run += dt * s;
    W[m + 1] = run;  // running sum within the block; offset added below
  }
  tot[t] = run;
  __syncthreads();
  if (t == 0) {
    double acc = 0.0;
    for (int i = 0; i < 1024; ++i) {
      const double v = tot[i];
      tot[i] = acc;
      acc += v;
    }
    W[0] = 0.0;
  }
  __syncthreads();
  const double off = tot[t];
  for (int m = m0; m < m1; ++m) W[m + 1] = volume * (W[m + 1] + off);
}

hipError_t launch_work(const double* I, const double* A, int n_t, double dt, double volume, double* W, hipStream_t s) {
  hipLaunchKernelGGL(k_work, dim3(1), dim3(1024), 0, s, I, A, n_t, dt, volume, W);
  return hipGetLastError();
}

}  // namespace td
