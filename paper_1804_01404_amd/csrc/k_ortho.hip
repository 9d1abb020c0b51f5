// Orthonormalisation of the orbitals of every k-point (Gram-Schmidt in
// orbital order, as Cholesky-QR): S_k[i][j] = h^3 sum_r w_i(r) conj(w_j(r))
// formed on the device in FP64 (fixed-order reductions), S_k = L L^H factored
// and inverted on the device, and w <- L^{-1} w applied there too. Used by the
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

// Per k-point (one workgroup each): the Cholesky factor S = L L^H of the
// Hermitian positive overlap matrix (left-looking, column by column; L
// overwrites the lower triangle of S) and its inverse M = L^{-1} (lower
// triangular; the columns of M are independent, one thread each). A pivot
// that is not positive sets *bad (the orbitals became linearly dependent).
__global__ __launch_bounds__(256) void k_chol_inverse(double2* __restrict__ S, double2* __restrict__ M, int n,
                                                      int* __restrict__ bad) {
  __shared__ double piv;
  const int k = blockIdx.x;
  double2* L = S + (size_t)k * n * n;
  double2* Mk = M + (size_t)k * n * n;
  const int t = threadIdx.x, nt = blockDim.x;
  for (int j = 0; j < n; ++j) {
    // s_ij = S_ij - sum_{q<j} L_iq conj(L_jq), for i >= j
    for (int i = j + t; i < n; i += nt) {
      double sr = L[(size_t)i * n + j].x, si = L[(size_t)i * n + j].y;
      for (int q = 0; q < j; ++q) {
        const double2 a = L[(size_t)i * n + q], b = L[(size_t)j * n + q];
        sr -= a.x * b.x + a.y * b.y;
        si -= a.y * b.x - a.x * b.y;
      }
      L[(size_t)i * n + j] = make_double2(sr, si);
    }
    __syncthreads();
    if (t == 0) {
      const double d = L[(size_t)j * n + j].x;
      if (!(d > 0.0)) atomicOr(bad, 1);
      piv = d > 0.0 ? sqrt(d) : 1.0;
      L[(size_t)j * n + j] = make_double2(piv, 0.0);
    }
    __syncthreads();
    for (int i = j + 1 + t; i < n; i += nt) {
      const double2 v = L[(size_t)i * n + j];
      L[(size_t)i * n + j] = make_double2(v.x / piv, v.y / piv);
    }
    __syncthreads();
  }
  // M = L^{-1}: column c by forward substitution, M_ic = (delta_ic - sum_{q=c}^{i-1} L_iq M_qc) / L_ii
  for (int c = t; c < n; c += nt) {
    for (int i = 0; i < c; ++i) Mk[(size_t)i * n + c] = make_double2(0.0, 0.0);
    for (int i = c; i < n; ++i) {
      double br = (i == c) ? 1.0 : 0.0, bi = 0.0;
      for (int q = c; q < i; ++q) {
        const double2 l = L[(size_t)i * n + q], m = Mk[(size_t)q * n + c];
        br -= l.x * m.x - l.y * m.y;
        bi -= l.x * m.y + l.y * m.x;
      }
      const double d = L[(size_t)i * n + i].x;
      Mk[(size_t)i * n + c] = make_double2(br / d, bi / d);
    }
  }
}

hipError_t launch_chol_inverse(double2* S, double2* M, int n, int n_k, int* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_chol_inverse, dim3((unsigned)n_k), dim3(256), 0, s, S, M, n, bad);
  return hipGetLastError();
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

// Occupied weight kept in the reference space, per k-point:
//   S_k = sum_{m,n} |h^3 sum_r conj(ref_m(r)) w_n(r)|^2   (n_orb <= 64).
// One workgroup per k-point; the grid is walked in tiles of 16 points staged
// in LDS in FP64; thread t owns the orbital pairs t, t + 256, ... and the
// pair sums are combined by a fixed tree.
constexpr int kOvTile = 16;
constexpr int kOvMaxOrb = 64;

template <typename T>
__global__ __launch_bounds__(256) void k_overlap_weight(const typename Vec2<T>::type* __restrict__ ref,
                                                        const typename Vec2<T>::type* __restrict__ w, int n_orb,
                                                        int N, double dV, double* __restrict__ Sk) {
  __shared__ double2 tr[kOvMaxOrb][kOvTile + 1];
  __shared__ double2 tw[kOvMaxOrb][kOvTile + 1];
  __shared__ double red[256];
  constexpr int kPairs = kOvMaxOrb * kOvMaxOrb / 256;
  const int k = blockIdx.x;
  const int tid = threadIdx.x;
  const int npair = n_orb * n_orb;
  double ar[kPairs], ai[kPairs];
#pragma unroll
  for (int j = 0; j < kPairs; ++j) ar[j] = ai[j] = 0.0;
  const size_t base = (size_t)k * n_orb * N;
  for (int p0 = 0; p0 < N; p0 += kOvTile) {
    for (int t = tid; t < n_orb * kOvTile; t += 256) {
      const int m = t / kOvTile, q = t - m * kOvTile;
      const int p = p0 + q;
      double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
      if (p < N) {
        const auto va = ref[base + (size_t)m * N + p];
        const auto vb = w[base + (size_t)m * N + p];
        a = make_double2((double)va.x, (double)va.y);
        b = make_double2((double)vb.x, (double)vb.y);
      }
      tr[m][q] = a;
      tw[m][q] = b;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kPairs; ++j) {
      const int pr = tid + 256 * j;
      if (pr < npair) {
        const int m = pr / n_orb, n = pr - m * n_orb;
#pragma unroll
        for (int q = 0; q < kOvTile; ++q) {
          const double2 a = tr[m][q], b = tw[n][q];
          ar[j] += a.x * b.x + a.y * b.y;  // conj(a) b
          ai[j] += a.x * b.y - a.y * b.x;
        }
      }
    }
    __syncthreads();
  }
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < kPairs; ++j) s += dV * dV * (ar[j] * ar[j] + ai[j] * ai[j]);
  red[tid] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  if (tid == 0) Sk[k] = red[0];
}

template <typename T>
hipError_t launch_overlap_weight(const typename Vec2<T>::type* ref, const typename Vec2<T>::type* w, int n_orb,
                                 int n_k, int N, double dV, double* Sk, hipStream_t s) {
  if (n_orb > kOvMaxOrb) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_overlap_weight<T>), dim3((unsigned)n_k), dim3(256), 0, s, ref, w, n_orb, N, dV, Sk);
  return hipGetLastError();
}

template hipError_t launch_overlap_weight<double>(const double2*, const double2*, int, int, int, double, double*,
                                                  hipStream_t);
template hipError_t launch_overlap_weight<float>(const float2*, const float2*, int, int, int, double, double*,
                                                 hipStream_t);

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
