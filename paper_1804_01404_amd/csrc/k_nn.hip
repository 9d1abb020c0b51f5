// Kernels of the current surrogate that stands in for a microscopic cell in
// the multiscale coupling (Sec. 5): a causal window of the vector potential
// -> dense W->H, tanh -> dense H->H, tanh -> dense H->1, plus a linear skip
// W->1. FP32 throughout; every reduction runs in a fixed order, so results do
// not depend on scheduling. Parameter layout (flat): W1 [H][W], b1 [H],
// W2 [H][H], b2 [H], w3 [H], b3 [1], ws [W]. Adam follows Kingma and Ba
// (ICLR 2015, Algorithm 1).
#include "internal.h"

namespace td {

constexpr int kTile = 16;

// C[i][j] = sum_k A(i, k) B(k, j) for i < M, j < N, with A(i, k) = A[i*sai + k*sak]
// and B(k, j) = B[k*sbk + j*sbj]; epilogue: + bias[j] (if bias), tanh (if act),
// then * (1 - aux[i][j]^2) (if aux, the tanh derivative of a stored activation).
__global__ __launch_bounds__(kTile* kTile) void k_gemm(const float* __restrict__ A, long sai, long sak,
                                                      const float* __restrict__ B, long sbk, long sbj,
                                                      float* __restrict__ C, int M, int N, int K,
                                                      const float* __restrict__ bias, int act,
                                                      const float* __restrict__ aux) {
  __shared__ float ta[kTile][kTile + 1];
  __shared__ float tb[kTile][kTile + 1];
  const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;
  const int i = blockIdx.y * kTile + ty;
  const int j = blockIdx.x * kTile + tx;
  float acc = 0.0f;
  for (int k0 = 0; k0 < K; k0 += kTile) {
    {
      const int ai = blockIdx.y * kTile + ty, ak = k0 + tx;
      ta[ty][tx] = (ai < M && ak < K) ? A[ai * sai + ak * sak] : 0.0f;
      const int bk = k0 + ty, bj = blockIdx.x * kTile + tx;
      tb[ty][tx] = (bk < K && bj < N) ? B[bk * sbk + bj * sbj] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kTile; ++kk) acc = fmaf(ta[ty][kk], tb[kk][tx], acc);
    __syncthreads();
  }
  if (i < M && j < N) {
    if (bias) acc += bias[j];
    if (act) acc = tanhf(acc);
    if (aux) {
      const float h = aux[(long)i * N + j];
      acc *= 1.0f - h * h;
    }
    C[(long)i * N + j] = acc;
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
  hipLaunchKernelGGL(k_gemm, grid, dim3(kTile * kTile), 0, s, A, sai, sak, B, sbk, sbj, C, M, N, K, bias, act,
                     aux);
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
