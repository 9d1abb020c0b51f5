// Kernels of the current surrogate that stands in for a microscopic cell in
// the multiscale coupling (Sec. 5): a causal window of the vector potential
// -> dense W->H, tanh -> dense H->H, tanh -> dense H->1, plus a linear skip
// W->1. FP32 throughout, the dense layers on the matrix cores; every reduction
// runs in a fixed order, so results do not depend on scheduling. Parameter layout (flat): W1 [H][W], b1 [H],
// W2 [H][H], b2 [H], w3 [H], b3 [1], ws [W]. Adam follows Kingma and Ba
// (ICLR 2015, Algorithm 1).
#include "internal.h"

namespace td {

constexpr int kTile = 16;      // output tile of one workgroup (the MFMA's 16 x 16)
constexpr int kGemmWaves = 4;  // wavefronts per tile, each a quarter of the k range

typedef float f32x4 __attribute__((ext_vector_type(4)));

// C[i][j] = sum_k A(i, k) B(k, j) for i < M, j < N, with A(i, k) = A[i*sai + k*sak]
// and B(k, j) = B[k*sbk + j*sbj]; epilogue: + bias[j] (if bias), tanh (if act),
// then * (1 - aux[i][j]^2) (if aux, the tanh derivative of a stored activation).
// On the matrix cores: v_mfma_f32_16x16x4f32 takes A(i, k) from lane i + 16 k
// and B(k, j) from lane j + 16 k of a 16 x 4 / 4 x 16 slice and leaves
// C(4 g + r, j) in element r of lane j + 16 g. Each of the four wavefronts of a
// tile runs a contiguous quarter of the k steps; the partial tiles are added in
// wavefront order, so the result does not depend on scheduling.
__global__ __launch_bounds__(kGemmWaves * 64) void k_gemm(const float* __restrict__ A, long sai, long sak,
                                                         const float* __restrict__ B, long sbk, long sbj,
                                                         float* __restrict__ C, int M, int N, int K,
                                                         const float* __restrict__ bias, int act,
                                                         const float* __restrict__ aux) {
  __shared__ float part[kGemmWaves - 1][kTile][kTile + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, q = lane >> 4;
  const int i0 = blockIdx.y * kTile, j0 = blockIdx.x * kTile;
  // rows and columns past the matrix load a clamped in-range element and use 0
  const bool aok = i0 + r < M, bok = j0 + r < N;
  const long ia = min(i0 + r, M - 1), jb = min(j0 + r, N - 1);
  const int steps = (K + 3) / 4;
  const int per = (steps + kGemmWaves - 1) / kGemmWaves;
  const int s0 = wave * per, s1 = min(steps, s0 + per);
  f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
  // chunks of kChunk k steps: every load of a chunk is issued before its
  // products (steps past s1 or K load a clamped element and use 0)
  constexpr int kChunk = 8;
  for (int c0 = s0; c0 < s1; c0 += kChunk) {
    float av[kChunk], bv[kChunk];
#pragma unroll
    for (int u = 0; u < kChunk; ++u) {
      const long kc = min(4 * (c0 + u) + q, K - 1);
      av[u] = A[ia * sai + kc * sak];
      bv[u] = B[kc * sbk + jb * sbj];
    }
#pragma unroll
    for (int u = 0; u < kChunk; ++u) {
      const bool kin = c0 + u < s1 && 4 * (c0 + u) + q < K;
      const float a = (aok && kin) ? av[u] : 0.0f;
      const float b = (bok && kin) ? bv[u] : 0.0f;
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
  }
  if (wave > 0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) part[wave - 1][4 * q + e][r] = acc[e];
  }
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      float v = acc[e];
#pragma unroll
      for (int w = 0; w < kGemmWaves - 1; ++w) v += part[w][4 * q + e][r];
      const int i = i0 + 4 * q + e, j = j0 + r;
      if (i < M && j < N) {
        if (bias) v += bias[j];
        if (act) v = tanhf(v);
        if (aux) {
          const float h = aux[(long)i * N + j];
          v *= 1.0f - h * h;
        }
        C[(long)i * N + j] = v;
      }
    }
  }
}

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// y[b] = w3 . h2[b] + b3 + ws . x[b]; one wavefront per sample
__global__ void k_nn_out(const float* __restrict__ h2, const float* __restrict__ x, const float* __restrict__ w3,
                         const float* __restrict__ b3, const float* __restrict__ ws, int B, int H, int W,
                         float* __restrict__ y) {
  const int b = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (b >= B) return;
  float s = 0.0f;
  for (int h = lane; h < H; h += 64) s = fmaf(h2[(long)b * H + h], w3[h], s);
  float t = 0.0f;
  for (int w = lane; w < W; w += 64) t = fmaf(x[(long)b * W + w], ws[w], t);
  s = wave_sum_f(s) + b3[0] + wave_sum_f(t);
  if (lane == 0) y[b] = s;
}

// dy[b] = 2 (y[b] - t[b]) / B and the loss (1/B) sum (y - t)^2 (one block)
__global__ __launch_bounds__(256) void k_nn_dy_loss(const float* __restrict__ y, const float* __restrict__ t, int B,
                                                    float* __restrict__ dy, float* __restrict__ loss) {
  __shared__ float red[256];
  float s = 0.0f;
  for (int b = threadIdx.x; b < B; b += 256) {
    const float r = y[b] - t[b];
    dy[b] = 2.0f * r / (float)B;
    s = fmaf(r, r, s);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = red[0] / (float)B;
}

// out[j] = sum_b M[b][j] * (wgt ? wgt[b] : 1), j < N (column sums in b order)
__global__ void k_colsum(const float* __restrict__ M, const float* __restrict__ wgt, int B, int N,
                         float* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  float s = 0.0f;
  for (int b = 0; b < B; ++b) s = fmaf(M[(long)b * N + j], wgt ? wgt[b] : 1.0f, s);
  out[j] = s;
}

// dz2[b][h] = dy[b] w3[h] (1 - h2[b][h]^2)
__global__ void k_nn_dz2(const float* __restrict__ dy, const float* __restrict__ w3, const float* __restrict__ h2,
                         int B, int H, float* __restrict__ dz2) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)B * H) return;
  const int b = (int)(t / H), h = (int)(t - (long)b * H);
  const float a = h2[t];
  dz2[t] = dy[b] * w3[h] * (1.0f - a * a);
}

// Adam: m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
// theta -= lr (m / c1) / (sqrt(v / c2) + eps), c1 = 1 - b1^t, c2 = 1 - b2^t
__global__ void k_adam(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, long n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  theta[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// training batch from trajectories: for sample s = idx[b] = traj * T + t,
// X[b][w] = seqA[traj][t - W + 1 + w] (0 before the start), target[b] = seqJ[traj][t]
__global__ void k_nn_gather(const float* __restrict__ seqA, const float* __restrict__ seqJ, int T, int W,
                            const int* __restrict__ idx, int B, float* __restrict__ X, float* __restrict__ target) {
  const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (long)B * W) return;
  const int b = (int)(q / W), w = (int)(q - (long)b * W);
  const int s = idx[b];
  const int tr = s / T, t = s - tr * T;
  const int src = t - W + 1 + w;
  X[q] = src >= 0 ? seqA[(long)tr * T + src] : 0.0f;
  if (w == W - 1) target[b] = seqJ[(long)tr * T + t];
}

// dst[0] += src[0]
__global__ void k_accum(const float* __restrict__ src, float* __restrict__ dst) {
  if (threadIdx.x == 0) dst[0] += src[0];
}

// ---------------------------------------------------------------- launchers
static hipError_t gemm(const float* A, long sai, long sak, const float* B, long sbk, long sbj, float* C, int M,
                       int N, int K, const float* bias, int act, const float* aux, hipStream_t s) {
  const dim3 grid((unsigned)((N + kTile - 1) / kTile), (unsigned)((M + kTile - 1) / kTile));
  hipLaunchKernelGGL(k_gemm, grid, dim3(kGemmWaves * 64), 0, s, A, sai, sak, B, sbk, sbj, C, M, N, K, bias, act,
                     aux);
  return hipGetLastError();
}

__global__ void k_zero_f(float* __restrict__ p, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

// G[i][i] += lambda_rel * trace(G) / n (one workgroup, fixed-order sum)
__global__ __launch_bounds__(1024) void k_lin_trace_scale(double* __restrict__ G, int n, double lambda_rel) {
  __shared__ double red[1024];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int i = t; i < n; i += 1024) s += G[(size_t)i * n + i];
  red[t] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  const double lam = lambda_rel * red[0] / n;
  __syncthreads();
  for (int i = t; i < n; i += 1024) G[(size_t)i * n + i] += lam;
}

// ---------------------------------------------------------------------------
// Least-squares fit of the linear part (skip weights and output bias) over a
// set of trajectories, FP64. With the regressors x = (window of A, 1), n = W + 1:
//   G[i][j] = sum over samples of x_i x_j,  b[i] = sum x_i y,
// then (G + lambda I) w = b by a Cholesky factorisation in one workgroup.
// Window entry i of the sample at time t of a trajectory is A(t - W + 1 + i),
// zero before t = 0; the sums run over trajectories and times in order.

__device__ __forceinline__ double lin_x(const double* __restrict__ a, int T, int W, int t, int i) {
  if (i == W) return 1.0;
  const int tt = t - W + 1 + i;
  return tt >= 0 ? a[tt] : 0.0;
}

// one thread per (i, j >= i) pair of G, and one per entry of b (j = n)
__global__ void k_lin_gram(const double* __restrict__ A, const double* __restrict__ Y, int n_traj, int T, int W,
                           double* __restrict__ G, double* __restrict__ b) {
  const int n = W + 1;
  const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long pairs = (long)n * (n + 1) / 2;
  if (id >= pairs + n) return;
  int i, j;
  bool rhs = id >= pairs;
  if (rhs) {
    i = (int)(id - pairs);
    j = -1;
  } else {
    // id -> (i, j) with 0 <= i <= j < n, row by row
    long r = id;
    i = 0;
    while (r >= n - i) {
      r -= n - i;
      ++i;
    }
    j = i + (int)r;
  }
  double acc = 0.0;
  for (int k = 0; k < n_traj; ++k) {
    const double* a = A + (size_t)k * T;
    const double* y = Y + (size_t)k * T;
    for (int t = 0; t < T; ++t) {
      const double xi = lin_x(a, T, W, t, i);
      acc += xi * (rhs ? y[t] : lin_x(a, T, W, t, j));
    }
  }
  if (rhs) {
    b[i] = acc;
  } else {
    G[(size_t)i * n + j] = acc;
    G[(size_t)j * n + i] = acc;
  }
}

// Solve (G + lambda I) w = b in place (G n x n, row-major): right-looking
// Cholesky G = L L^T (L in the lower triangle), then L z = b, L^T w = z.
// One workgroup; *ok = 0 if a pivot is not positive.
__global__ __launch_bounds__(1024) void k_lin_solve(double* __restrict__ G, double* __restrict__ b, int n,
                                                    double lambda, float* __restrict__ ws, float* __restrict__ b3,
                                                    int* __restrict__ ok) {
  __shared__ double piv;
  __shared__ int good;
  const int t = threadIdx.x, nt = blockDim.x;
  if (t == 0) good = 1;
  for (int i = t; i < n; i += nt) G[(size_t)i * n + i] += lambda;
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (t == 0) {
      const double d = G[(size_t)j * n + j];
      if (!(d > 0.0)) good = 0;
      piv = d > 0.0 ? sqrt(d) : 1.0;
      G[(size_t)j * n + j] = piv;
    }
    __syncthreads();
    for (int i = j + 1 + t; i < n; i += nt) G[(size_t)i * n + j] /= piv;
    __syncthreads();
    // trailing update of the lower triangle: G[i][k] -= L[i][j] L[k][j], j < k <= i
    const int m = n - j - 1;
    const long cnt = (long)m * (m + 1) / 2;
    for (long q = t; q < cnt; q += nt) {
      // q -> (ii, kk) with 0 <= kk <= ii < m
      const int ii = (int)((sqrt(8.0 * (double)q + 1.0) - 1.0) * 0.5);
      int i2 = ii;
      long base = (long)i2 * (i2 + 1) / 2;
      if (base > q) {
        --i2;
        base = (long)i2 * (i2 + 1) / 2;
      } else if (base + i2 + 1 <= q) {
        ++i2;
        base = (long)i2 * (i2 + 1) / 2;
      }
      const int kk = (int)(q - base);
      const int row = j + 1 + i2, col = j + 1 + kk;
      G[(size_t)row * n + col] -= G[(size_t)row * n + j] * G[(size_t)col * n + j];
    }
    __syncthreads();
  }
  // forward substitution L z = b (z in b), then back substitution L^T w = z
  for (int j = 0; j < n; ++j) {
    if (t == 0) b[j] /= G[(size_t)j * n + j];
    __syncthreads();
    for (int i = j + 1 + t; i < n; i += nt) b[i] -= G[(size_t)i * n + j] * b[j];
    __syncthreads();
  }
  for (int j = n - 1; j >= 0; --j) {
    if (t == 0) b[j] /= G[(size_t)j * n + j];
    __syncthreads();
    for (int i = t; i < j; i += nt) b[i] -= G[(size_t)j * n + i] * b[j];
    __syncthreads();
  }
  for (int i = t; i < n - 1; i += nt) ws[i] = (float)b[i];
  if (t == 0) {
    *b3 = (float)b[n - 1];
    *ok = good;
  }
}

hipError_t nn_fit_linear(const double* A, const double* Y, int n_traj, int T, int W, double lambda_rel, double* G,
                         double* b, float* ws, float* b3, int* ok, hipStream_t s) {
  const int n = W + 1;
  const long work = (long)n * (n + 1) / 2 + n;
  hipLaunchKernelGGL(k_lin_gram, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, s, A, Y, n_traj, T, W, G, b);
  // lambda relative to the mean diagonal of G, added by the solve kernel
  // (which reads the diagonal first)
  hipLaunchKernelGGL(k_lin_trace_scale, dim3(1), dim3(1024), 0, s, G, n, lambda_rel);
  hipLaunchKernelGGL(k_lin_solve, dim3(1), dim3(1024), 0, s, G, b, n, 0.0, ws, b3, ok);
  return hipGetLastError();
}

hipError_t nn_zero(float* p, long n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_f, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t nn_forward(const NNShape& sh, const float* theta, const float* X, int B, NNWork& wk, hipStream_t s) {
  const int W = sh.W, H = sh.H;
  const float* W1 = theta;
  const float* b1 = W1 + (long)H * W;
  const float* W2 = b1 + H;
  const float* b2 = W2 + (long)H * H;
  const float* w3 = b2 + H;
  const float* b3 = w3 + H;
  const float* ws = b3 + 1;
  hipError_t e;
  // h1 = tanh(X W1^T + b1): A = X [B][W], B(k=w, j=h) = W1[h][w]
  if ((e = gemm(X, W, 1, W1, 1, W, wk.h1, B, H, W, b1, 1, nullptr, s)) != hipSuccess) return e;
  if ((e = gemm(wk.h1, H, 1, W2, 1, H, wk.h2, B, H, H, b2, 1, nullptr, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_nn_out, dim3((unsigned)((B + 3) / 4)), dim3(256), 0, s, wk.h2, X, w3, b3, ws, B, H, W, wk.y);
  return hipGetLastError();
}

hipError_t nn_backward(const NNShape& sh, const float* theta, const float* X, const float* target, int B,
                       NNWork& wk, float* grad, hipStream_t s) {
  const int W = sh.W, H = sh.H;
  const float* W2 = theta + (long)H * W + H;
  const float* w3 = W2 + (long)H * H + H;
  float* gW1 = grad;
  float* gb1 = gW1 + (long)H * W;
  float* gW2 = gb1 + H;
  float* gb2 = gW2 + (long)H * H;
  float* gw3 = gb2 + H;
  float* gb3 = gw3 + H;
  float* gws = gb3 + 1;
  hipError_t e;
  hipLaunchKernelGGL(k_nn_dy_loss, dim3(1), dim3(256), 0, s, wk.y, target, B, wk.dy, wk.loss);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_colsum, dim3((unsigned)((H + 63) / 64)), dim3(64), 0, s, wk.h2, wk.dy, B, H, gw3);
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(64), 0, s, wk.dy, nullptr, B, 1, gb3);
  hipLaunchKernelGGL(k_colsum, dim3((unsigned)((W + 63) / 64)), dim3(64), 0, s, X, wk.dy, B, W, gws);
  hipLaunchKernelGGL(k_nn_dz2, dim3((unsigned)(((long)B * H + 255) / 256)), dim3(256), 0, s, wk.dy, w3, wk.h2, B,
                     H, wk.dz2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // gW2[h][k] = sum_b dz2[b][h] h1[b][k]: A(i=h, k=b) = dz2[b][h], B(k=b, j) = h1[b][j]
  if ((e = gemm(wk.dz2, 1, H, wk.h1, H, 1, gW2, H, H, B, nullptr, 0, nullptr, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_colsum, dim3((unsigned)((H + 63) / 64)), dim3(64), 0, s, wk.dz2, nullptr, B, H, gb2);
  // dz1[b][k] = (sum_h dz2[b][h] W2[h][k]) (1 - h1[b][k]^2)
  if ((e = gemm(wk.dz2, H, 1, W2, H, 1, wk.dz1, B, H, H, nullptr, 0, wk.h1, s)) != hipSuccess) return e;
  // gW1[h][w] = sum_b dz1[b][h] X[b][w]
  if ((e = gemm(wk.dz1, 1, H, X, W, 1, gW1, H, W, B, nullptr, 0, nullptr, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_colsum, dim3((unsigned)((H + 63) / 64)), dim3(64), 0, s, wk.dz1, nullptr, B, H, gb1);
  return hipGetLastError();
}

hipError_t nn_adam(float* theta, float* m, float* v, const float* g, long n, float lr, float b1, float b2,
                   float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, theta, m, v, g, n, lr, b1, b2, eps,
                     c1, c2);
  return hipGetLastError();
}

hipError_t nn_gather(const float* seqA, const float* seqJ, int T, int W, const int* idx, int B, float* X,
                     float* target, hipStream_t s) {
  const long n = (long)B * W;
  hipLaunchKernelGGL(k_nn_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, seqA, seqJ, T, W, idx, B, X,
                     target);
  return hipGetLastError();
}

hipError_t nn_accumulate(const float* src, float* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_accum, dim3(1), dim3(64), 0, s, src, dst);
  return hipGetLastError();
}

}  // namespace td
