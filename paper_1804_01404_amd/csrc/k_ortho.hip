// Orthonormalisation of the orbitals of every k-point (Gram-Schmidt in
// orbital order, as Cholesky-QR): S_k[i][j] = h^3 sum_r w_i(r) conj(w_j(r))
// formed on the device in FP64 (fixed-order reductions), S_k = L L^H factored
// on the host, and w <- L^{-1} w applied on the device. Used by the
// ground-state preparation that precedes the real-time run (Sec. 2.1).
#include "internal.h"

namespace td {

// one workgroup per (k, i, j <= i): a fixed-order reduction over the grid
template <typename T>
__global__ __launch_bounds__(256) void k_gram(const typename Vec2<T>::type* w, int n_orb, int N, double dV,
                                              double2* S) {
  __shared__ double red[256][2];
  const int npairs = n_orb * (n_orb + 1) / 2;
  const int k = blockIdx.x / npairs;
  int pr = blockIdx.x - k * npairs;
  int i = 0;
  while (pr >= i + 1) {
    pr -= i + 1;
    ++i;
  }
  const int j = pr;
  const auto* wi = w + ((size_t)k * n_orb + i) * N;
  const auto* wj = w + ((size_t)k * n_orb + j) * N;
  double sr = 0.0, si = 0.0;
  for (int p = threadIdx.x; p < N; p += blockDim.x) {
    const double ar = (double)wi[p].x, ai = (double)wi[p].y;
    const double br = (double)wj[p].x, bi = (double)wj[p].y;
    sr += ar * br + ai * bi;  // w_i conj(w_j)
    si += ai * br - ar * bi;
  }
  red[threadIdx.x][0] = sr;
  red[threadIdx.x][1] = si;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[threadIdx.x][0] += red[threadIdx.x + s][0];
      red[threadIdx.x][1] += red[threadIdx.x + s][1];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    S[((size_t)k * n_orb + i) * n_orb + j] = make_double2(dV * red[0][0], dV * red[0][1]);
    S[((size_t)k * n_orb + j) * n_orb + i] = make_double2(dV * red[0][0], -dV * red[0][1]);
  }
}

// out[k][i][p] = sum_{j <= i} M[k][i][j] w[k][j][p]
template <typename T>
__global__ void k_apply_lower(const typename Vec2<T>::type* w, const double2* M, int n_orb, int n_k, int N,
                              typename Vec2<T>::type* out) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)n_k * N) return;
  const int k = (int)(t / N);
  const int p = (int)(t - (size_t)k * N);
  const auto* wk = w + (size_t)k * n_orb * N;
  const double2* Mk = M + (size_t)k * n_orb * n_orb;
  for (int i = 0; i < n_orb; ++i) {
    double re = 0.0, im = 0.0;
    for (int j = 0; j <= i; ++j) {
      const double2 m = Mk[i * n_orb + j];
      const auto v = wk[(size_t)j * N + p];
      const double vr = (double)v.x, vi = (double)v.y;
      re += m.x * vr - m.y * vi;
      im += m.x * vi + m.y * vr;
    }
    typename Vec2<T>::type o;
    o.x = (T)re;
    o.y = (T)im;
    out[((size_t)k * n_orb + i) * N + p] = o;
  }
}

template <typename T>
hipError_t launch_gram(const typename Vec2<T>::type* w, int n_orb, int n_k, int N, double dV, double2* S,
                       hipStream_t s) {
  const int npairs = n_orb * (n_orb + 1) / 2;
  hipLaunchKernelGGL((k_gram<T>), dim3((unsigned)(n_k * npairs)), dim3(256), 0, s, w, n_orb, N, dV, S);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_apply_lower(const typename Vec2<T>::type* w, const double2* M, int n_orb, int n_k, int N,
                              typename Vec2<T>::type* out, hipStream_t s) {
  const size_t total = (size_t)n_k * N;
  hipLaunchKernelGGL((k_apply_lower<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, w, M, n_orb,
                     n_k, N, out);
  return hipGetLastError();
}

template hipError_t launch_gram<double>(const double2*, int, int, int, double, double2*, hipStream_t);
template hipError_t launch_gram<float>(const float2*, int, int, int, double, double2*, hipStream_t);
template hipError_t launch_apply_lower<double>(const double2*, const double2*, int, int, int, double2*, hipStream_t);
template hipError_t launch_apply_lower<float>(const float2*, const double2*, int, int, int, float2*, hipStream_t);

}  // namespace td
