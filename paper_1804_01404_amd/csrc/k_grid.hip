// Grid-side kernels of one time step: per-step field parameters, the density
// (Eq. rho), the Hartree potential by FFT (periodic 4 pi / G^2; isolated
// free-space convolution on a doubled box), the adiabatic PZ81 LDA (Sec. 3.1),
// the macroscopic current reduction (Eq. macro_current) and the step counter.
// Every reduction runs in a fixed order, so two runs give identical bits.
#include "internal.h"

namespace td {

// ---------------------------------------------------------------- parameters
// A: table [..][3]; the step index n is *counter (or 0). Velocity gauge:
// kappa = k + (A_n + A_{n+1}) / (2c), kappaJ = k + A_{n+1} / c, and the
// matching sphere phases exp(i A.x / c). Length gauge: kappa = kappaJ = k,
// unit phases, E_n = -(A_{n+1} - A_n) / (c dt).
__device__ __forceinline__ void step_params_block(const double* A, const int* counter, int use_counter,
                                                  const double* kpt, int n_k, const double* ent_x, int S,
                                                  int gauge, double dt, double* kappa, double* kappaJ,
                                                  double* efield, double2* phA, double2* phAJ, double* Alast,
                                                  int bx) {
  const int n = use_counter ? *counter : 0;
  const double* A0 = A + 3 * (size_t)n;
  const double* A1 = A0 + 3;
  double ab[3], a1[3];
  for (int i = 0; i < 3; ++i) {
    ab[i] = 0.5 * (A0[i] + A1[i]);
    a1[i] = A1[i];
  }
  const bool vel = (gauge == 0);
  const int t = bx * blockDim.x + threadIdx.x;
  if (bx == 0) {
    for (int k = threadIdx.x; k < n_k; k += blockDim.x) {
      for (int i = 0; i < 3; ++i) {
        kappa[3 * k + i] = kpt[3 * k + i] + (vel ? ab[i] / kC : 0.0);
        kappaJ[3 * k + i] = kpt[3 * k + i] + (vel ? a1[i] / kC : 0.0);
      }
    }
    if (threadIdx.x < 3) {
      efield[threadIdx.x] = vel ? 0.0 : -(A1[threadIdx.x] - A0[threadIdx.x]) / (kC * dt);
      Alast[threadIdx.x] = a1[threadIdx.x];
    }
  }
  if (t < S) {
    const double* x = ent_x + 3 * (size_t)t;
    if (vel) {
      double s, c;
      sincos((ab[0] * x[0] + ab[1] * x[1] + ab[2] * x[2]) / kC, &s, &c);
      phA[t] = make_double2(c, s);
      sincos((a1[0] * x[0] + a1[1] * x[1] + a1[2] * x[2]) / kC, &s, &c);
      phAJ[t] = make_double2(c, s);
    } else {
      phA[t] = make_double2(1.0, 0.0);
      phAJ[t] = make_double2(1.0, 0.0);
    }
  }
}

__global__ void k_step_params(const double* A, const int* counter, int use_counter,
                              const double* kpt, int n_k, const double* ent_x, int S, int gauge,
                              double dt, double* kappa, double* kappaJ, double* efield,
                              double2* phA, double2* phAJ, double* Alast) {
  step_params_block(A, counter, use_counter, kpt, n_k, ent_x, S, gauge, dt, kappa, kappaJ, efield, phA, phAJ, Alast,
                    (int)blockIdx.x);
}

// the same for the cells of a group (cell blockIdx.y), each at its own step
__global__ void k_step_params_group(const ParamCell* __restrict__ tab) {
  const ParamCell& c = tab[blockIdx.y];
  if ((int)blockIdx.x > 0 && (int)blockIdx.x * (int)blockDim.x >= c.S) return;
  step_params_block(c.A, c.counter, 1, c.kpt, c.n_k, c.ent_x, c.S, c.gauge, c.dt, c.kappa, c.kappaJ, c.efield, c.phA,
                    c.phAJ, c.Alast, (int)blockIdx.x);
}

hipError_t launch_step_params_group(const ParamCell* tab, int ncells, int max_S, hipStream_t s) {
  const int blocks = max_S > 0 ? (max_S + 255) / 256 : 1;
  hipLaunchKernelGGL(k_step_params_group, dim3(blocks, ncells), dim3(256), 0, s, tab);
  return hipGetLastError();
}

hipError_t launch_step_params(const double* A, const int* counter, int use_counter,
                              const double* kpt, int n_k, const double* ent_x, int S, int gauge,
                              double dt, double* kappa, double* kappaJ, double* efield, double2* phA,
                              double2* phAJ, double* Alast, hipStream_t s) {
  const int blocks = S > 0 ? (S + 255) / 256 : 1;
  hipLaunchKernelGGL(k_step_params, dim3(blocks), dim3(256), 0, s, A, counter, use_counter, kpt, n_k,
                     ent_x, S, gauge, dt, kappa, kappaJ, efield, phA, phAJ, Alast);
  return hipGetLastError();
}

// ---------------------------------------------------------------- batch tables
__global__ void k_batch_tables_in(const IOCell* __restrict__ io, const double* __restrict__ staged, int len) {
  const IOCell& c = io[blockIdx.x];
  const double* src = staged + (size_t)blockIdx.x * len;
  for (int i = threadIdx.x; i < len; i += blockDim.x) c.A[i] = src[i];
  if (threadIdx.x == 0) *c.counter = 0;
}

__global__ void k_batch_tables_out(const IOCell* __restrict__ io, double* __restrict__ staged, int len) {
  const IOCell& c = io[blockIdx.x];
  double* dst = staged + (size_t)blockIdx.x * (len + 1);
  for (int i = threadIdx.x; i < len; i += blockDim.x) dst[i] = c.J[i];
  if (threadIdx.x == 0) dst[len] = (double)*c.nanflag;
}

hipError_t launch_batch_tables_in(const IOCell* io, int ncells, const double* staged, int len, hipStream_t s) {
  if (ncells <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_tables_in, dim3(ncells), dim3(64), 0, s, io, staged, len);
  return hipGetLastError();
}

hipError_t launch_batch_tables_out(const IOCell* io, int ncells, double* staged, int len, hipStream_t s) {
  if (ncells <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_tables_out, dim3(ncells), dim3(64), 0, s, io, staged, len);
  return hipGetLastError();
}

// ---------------------------------------------------------------- density
// part[c][p] = sum over orbitals o in chunk c of 2 w_k |w_o(p)|^2, in order.
template <typename T>
__device__ __forceinline__ void rho_partial_point(const typename Vec2<T>::type* w, const double* kw, int n_orb,
                                                  int n_k, int N, int chunk, int c, int p, double* part) {
  const int n_tot = n_orb * n_k;
  const int o0 = c * chunk;
  const int o1 = min(n_tot, o0 + chunk);
  double acc = 0.0;
  for (int o = o0; o < o1; ++o) {
    const auto v = w[(size_t)o * N + p];
    const double re = (double)v.x, im = (double)v.y;
    acc += 2.0 * kw[o / n_orb] * (re * re + im * im);
  }
  part[(size_t)c * N + p] = acc;
}

template <typename T>
__global__ void k_rho_partial(const typename Vec2<T>::type* w, const double* kw, int n_orb, int n_k,
                              int N, int chunk, double* part) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  rho_partial_point<T>(w, kw, n_orb, n_k, N, chunk, (int)blockIdx.y, p, part);
}

// the same for the cells of a group: cell blockIdx.z, chunk blockIdx.y
template <typename T>
__global__ void k_rho_partial_group(const TailCell* __restrict__ tab, int N, int chunk) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const TailCell& t = tab[blockIdx.z];
  if (p >= N || (int)blockIdx.y >= t.nchunks) return;
  rho_partial_point<T>(static_cast<const typename Vec2<T>::type*>(t.w), t.kw, t.n_orb, t.n_k, N, chunk,
                       (int)blockIdx.y, p, t.rho_out);
}

template <typename T>
hipError_t launch_rho_partial_group(const TailCell* tab, int ncells, int N, int chunk, int max_chunks,
                                    hipStream_t s) {
  hipLaunchKernelGGL((k_rho_partial_group<T>), dim3((N + 255) / 256, max_chunks, ncells), dim3(256), 0, s, tab,
                     N, chunk);
  return hipGetLastError();
}
template hipError_t launch_rho_partial_group<double>(const TailCell*, int, int, int, int, hipStream_t);
template hipError_t launch_rho_partial_group<float>(const TailCell*, int, int, int, int, hipStream_t);

template <typename T>
hipError_t launch_rho_partial(const typename Vec2<T>::type* w, const double* kw, int n_orb, int n_k,
                              int N, int chunk, double* part, hipStream_t s) {
  const int nchunks = (n_orb * n_k + chunk - 1) / chunk;
  hipLaunchKernelGGL((k_rho_partial<T>), dim3((N + 255) / 256, nchunks), dim3(256), 0, s, w, kw,
                     n_orb, n_k, N, chunk, part);
  return hipGetLastError();
}
template hipError_t launch_rho_partial<double>(const double2*, const double*, int, int, int, int,
                                               double*, hipStream_t);
template hipError_t launch_rho_partial<float>(const float2*, const double*, int, int, int, int,
                                              double*, hipStream_t);

// rho[p] = sum over chunks of part[c][p]. A workgroup takes 64 points and
// kRedSlices slices: slice j sums chunks j, j + kRedSlices, ... in order, then
// the slices combine by a fixed pairwise tree in LDS, so the result does not
// depend on scheduling. One thread per point looping over every chunk would
// leave the chip nearly idle (8000 points are 32 workgroups) behind a chain
// of dependent loads.
constexpr int kRedSlices = 16;

__device__ __forceinline__ void rho_reduce_block(const double* __restrict__ part, int nchunks, int N,
                                                 double* __restrict__ rho, double (*red)[64]) {
  const int i = threadIdx.x & 63, j = threadIdx.x >> 6;
  const int p = blockIdx.x * 64 + i;
  double acc = 0.0;
  if (p < N)
    for (int c = j; c < nchunks; c += kRedSlices) acc += part[(size_t)c * N + p];
  red[j][i] = acc;
  __syncthreads();
  for (int h = kRedSlices / 2; h > 0; h >>= 1) {
    if (j < h) red[j][i] += red[j + h][i];
    __syncthreads();
  }
  if (j == 0 && p < N) rho[p] = red[0][i];
}

__global__ __launch_bounds__(64 * kRedSlices) void k_rho_reduce(const double* __restrict__ part, int nchunks,
                                                                int N, double* __restrict__ rho) {
  __shared__ double red[kRedSlices][64];
  rho_reduce_block(part, nchunks, N, rho, red);
}

// the same for the cells of a group (cell blockIdx.y; cells with one chunk
// have their density already)
__global__ __launch_bounds__(64 * kRedSlices) void k_rho_reduce_group(const TailCell* __restrict__ tab, int N) {
  __shared__ double red[kRedSlices][64];
  const TailCell& t = tab[blockIdx.y];
  if (t.nchunks <= 1) return;
  rho_reduce_block(t.rho_part, t.nchunks, N, t.rho, red);
}

hipError_t launch_rho_reduce_group(const TailCell* tab, int ncells, int N, hipStream_t s) {
  hipLaunchKernelGGL(k_rho_reduce_group, dim3((N + 63) / 64, ncells), dim3(64 * kRedSlices), 0, s, tab, N);
  return hipGetLastError();
}

hipError_t launch_rho_reduce(const double* part, int nchunks, int N, double* rho, hipStream_t s) {
  hipLaunchKernelGGL(k_rho_reduce, dim3((N + 63) / 64), dim3(64 * kRedSlices), 0, s, part, nchunks, N, rho);
  return hipGetLastError();
}

// ---------------------------------------------------------------- FFT
// In-place FP64 complex FFT of every line along one axis of an M1 x M2 x M3
// array (M1 fastest), unnormalised, sign -1 forward / +1 inverse. A workgroup
// stages B lines in LDS and runs a Stockham mixed-radix (4, 2, 3, 5)
// transform: for radix R and Ns = product of the radices already applied,
// butterfly j reads in[j + r M/R], multiplies by exp(sign 2 pi i r (j mod Ns) / (Ns R)),
// does a length-R DFT and writes out[(j / Ns) Ns R + (j mod Ns) + r Ns].
struct FFTPlan {
  int M, nf;
  int f[12];
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// o_s = sum_q v_q exp(sign 2 pi i q s / R) for R = 2, 3, 4, 5
template <int R>
__device__ __forceinline__ void dft_small(double2* v, int sign);

template <>
__device__ __forceinline__ void dft_small<2>(double2* v, int) {
  const double2 a = v[0], b = v[1];
  v[0] = make_double2(a.x + b.x, a.y + b.y);
  v[1] = make_double2(a.x - b.x, a.y - b.y);
}

template <>
__device__ __forceinline__ void dft_small<4>(double2* v, int sign) {
  // omega = exp(sign i pi / 2) = sign * i
  const double2 a = v[0], b = v[1], c = v[2], d = v[3];
  const double2 s02 = make_double2(a.x + c.x, a.y + c.y), d02 = make_double2(a.x - c.x, a.y - c.y);
  const double2 s13 = make_double2(b.x + d.x, b.y + d.y), d13 = make_double2(b.x - d.x, b.y - d.y);
  // i * sign * d13
  const double2 r13 = make_double2(-sign * d13.y, sign * d13.x);
  v[0] = make_double2(s02.x + s13.x, s02.y + s13.y);
  v[1] = make_double2(d02.x + r13.x, d02.y + r13.y);
  v[2] = make_double2(s02.x - s13.x, s02.y - s13.y);
  v[3] = make_double2(d02.x - r13.x, d02.y - r13.y);
}

template <>
__device__ __forceinline__ void dft_small<3>(double2* v, int sign) {
  const double c1 = -0.5, s1 = sign * 0.86602540378443864676;  // exp(sign 2 pi i / 3)
  const double2 a = v[0], b = v[1], c = v[2];
  const double2 sbc = make_double2(b.x + c.x, b.y + c.y), dbc = make_double2(b.x - c.x, b.y - c.y);
  v[0] = make_double2(a.x + sbc.x, a.y + sbc.y);
  const double2 m = make_double2(a.x + c1 * sbc.x, a.y + c1 * sbc.y);
  // omega b + conj(omega) c = c1 (b + c) + i s1 (b - c)
  v[1] = make_double2(m.x - s1 * dbc.y, m.y + s1 * dbc.x);
  v[2] = make_double2(m.x + s1 * dbc.y, m.y - s1 * dbc.x);
}

template <>
__device__ __forceinline__ void dft_small<5>(double2* v, int sign) {
  const double cs[5] = {1.0, 0.30901699437494742410, -0.80901699437494742410, -0.80901699437494742410,
                        0.30901699437494742410};
  const double sn[5] = {0.0, 0.95105651629515357212, 0.58778525229247312917, -0.58778525229247312917,
                        -0.95105651629515357212};
  double2 o[5];
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const int e = (q * s) % 5;
      const double c = cs[e], sv = sign * sn[e];
      re += v[q].x * c - v[q].y * sv;
      im += v[q].x * sv + v[q].y * c;
    }
    o[s] = make_double2(re, im);
  }
#pragma unroll
  for (int s = 0; s < 5; ++s) v[s] = o[s];
}

// twiddles of a stage: tw[jm (R - 1) + r - 1] = exp(sign 2 pi i r jm / (Ns R)), jm < Ns
template <int R>
__device__ void stockham_stage(const double2* in, double2* out, int B, int M, int Ns, int sign,
                               const double2* tw) {
  const int nb = M / R;
  for (int t = threadIdx.x; t < B * nb; t += blockDim.x) {
    const int line = t / nb;
    const int jj = t - line * nb;
    const double2* li = in + (size_t)line * M;
    double2* lo = out + (size_t)line * M;
    double2 v[R];
    const int jm = jj % Ns;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      v[r] = li[jj + r * nb];
      if (r > 0 && jm != 0) v[r] = cmul(v[r], tw[jm * (R - 1) + r - 1]);
    }
    dft_small<R>(v, sign);
    const int d = (jj / Ns) * Ns * R + jm;
#pragma unroll
    for (int r = 0; r < R; ++r) lo[d + r * Ns] = v[r];
  }
}

// the twiddles of every stage of the plan, stage after stage (M - 1 values)
__device__ void fft_twiddles(const FFTPlan& plan, int sign, double2* tw) {
  int off = 0, Ns = 1;
  for (int f = 0; f < plan.nf; ++f) {
    const int R = plan.f[f];
    for (int t = threadIdx.x; t < Ns * (R - 1); t += blockDim.x) {
      const int jm = t / (R - 1), r = t - jm * (R - 1) + 1;
      double sn, cs;
      sincospi(2.0 * sign * (double)(r * jm) / (double)(Ns * R), &sn, &cs);
      tw[off + t] = make_double2(cs, sn);
    }
    off += Ns * (R - 1);
    Ns *= R;
  }
}

// the plan's stages on B lines of length M in LDS (in -> out alternating);
// returns the buffer that holds the result
__device__ double2* fft_lines_lds(const FFTPlan& plan, double2* in, double2* out, int nl, int sign,
                                  const double2* tw) {
  const int M = plan.M;
  int Ns = 1, off = 0;
  for (int f = 0; f < plan.nf; ++f) {
    const int R = plan.f[f];
    if (R == 4) stockham_stage<4>(in, out, nl, M, Ns, sign, tw + off);
    else if (R == 2) stockham_stage<2>(in, out, nl, M, Ns, sign, tw + off);
    else if (R == 3) stockham_stage<3>(in, out, nl, M, Ns, sign, tw + off);
    else stockham_stage<5>(in, out, nl, M, Ns, sign, tw + off);
    __syncthreads();
    off += Ns * (R - 1);
    Ns *= R;
    double2* t = in;
    in = out;
    out = t;
  }
  return in;
}

// Optional ends of the Poisson solve, so that they cost no launch of their
// own: rho (n1 x n2 x n3, zero beyond it in the M-box) is read in place of
// data by the first (x) pass, and the result is multiplied by K (the Poisson
// kernel) by the z pass.
struct FFTEnds {
  const double* rho;
  int n1, n2, n3;
  const double* K;
};

// The lines a pass transforms and the part of each it reads and writes: lines
// (i1, i2) with i1 < l1, i2 < l2 — (y, z) for the x axis, (x, z) for y, (x, y)
// for z — elements at or beyond n_in read as 0, elements at or beyond n_out
// not stored. fused (z axis): forward transform, times K, inverse transform
// with the opposite sign, in one pass.
struct FFTLines {
  int l1, l2, n_in, n_out, fused;
};

// B lines of one pass from line blk B on (smem_raw: the dynamic LDS)
__device__ __forceinline__ void fft_axis_block(double2* data, int M1, int M2, int M3, int axis, int sign, int B,
                                               const FFTPlan& plan, const FFTEnds& ends, const FFTLines& ln,
                                               long blk, unsigned char* smem_raw) {
  (void)M3;
  const int M = plan.M;
  double2* buf0 = reinterpret_cast<double2*>(smem_raw);
  double2* buf1 = buf0 + (size_t)B * M;
  double2* tw = buf1 + (size_t)B * M;   // M entries
  double2* twi = tw + M;                // M entries (fused: the inverse's)
  const long nlines = (long)ln.l1 * ln.l2;
  const long L0 = blk * B;
  const int nl = (int)min((long)B, nlines - L0);
  const long stride = (axis == 0) ? 1 : (axis == 1 ? M1 : (long)M1 * M2);
  auto line_base = [&](long L) -> long {
    const long i2 = L / ln.l1, i1 = L - i2 * ln.l1;
    if (axis == 0) return (i2 * M2 + i1) * M1;
    if (axis == 1) return i2 * (long)M1 * M2 + i1;
    return i2 * M1 + i1;
  };
  fft_twiddles(plan, sign, tw);
  if (ln.fused) fft_twiddles(plan, -sign, twi);
  // load
  for (int i = threadIdx.x; i < nl * M; i += blockDim.x) {
    int line, e;
    if (axis == 0) {
      line = i / M;
      e = i - line * M;
    } else {
      e = i / nl;
      line = i - e * nl;
    }
    double2 v = make_double2(0.0, 0.0);
    if (e < ln.n_in) {
      const long gi = line_base(L0 + line) + (long)e * stride;
      if (ends.rho) {
        const int x = (int)(gi % M1), y = (int)((gi / M1) % M2), z = (int)(gi / ((long)M1 * M2));
        if (x < ends.n1 && y < ends.n2 && z < ends.n3)
          v = make_double2(ends.rho[((size_t)z * ends.n2 + y) * ends.n1 + x], 0.0);
      } else {
        v = data[gi];
      }
    }
    buf0[line * M + e] = v;
  }
  __syncthreads();
  double2* res = fft_lines_lds(plan, buf0, buf1, nl, sign, tw);
  if (ln.fused) {
    for (int i = threadIdx.x; i < nl * M; i += blockDim.x) {
      const int e = i / nl, line = i - e * nl;
      const double k = ends.K[line_base(L0 + line) + (long)e * stride];
      const double2 v = res[line * M + e];
      res[line * M + e] = make_double2(v.x * k, v.y * k);
    }
    __syncthreads();
    res = fft_lines_lds(plan, res, res == buf0 ? buf1 : buf0, nl, -sign, twi);
  }
  for (int i = threadIdx.x; i < nl * M; i += blockDim.x) {
    int line, e;
    if (axis == 0) {
      line = i / M;
      e = i - line * M;
    } else {
      e = i / nl;
      line = i - e * nl;
    }
    if (e >= ln.n_out) continue;
    const long gi = line_base(L0 + line) + (long)e * stride;
    double2 v = res[line * M + e];
    if (ends.K && !ln.fused) {
      const double k = ends.K[gi];
      v = make_double2(v.x * k, v.y * k);
    }
    data[gi] = v;
  }
}

__global__ __launch_bounds__(256) void k_fft_axis(double2* data, int M1, int M2, int M3, int axis,
                                                  int sign, int B, FFTPlan plan, FFTEnds ends, FFTLines ln) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  fft_axis_block(data, M1, M2, M3, axis, sign, B, plan, ends, ln, (long)blockIdx.x, smem_raw);
}

// the same pass for the cells of a group (cell blockIdx.y)
__global__ __launch_bounds__(256) void k_fft_axis_group(const TailCell* __restrict__ tab, int M1, int M2, int M3,
                                                        int axis, int sign, int B, FFTPlan plan, FFTEnds ends,
                                                        FFTLines ln, int use_rho, int use_K) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const TailCell& t = tab[blockIdx.y];
  FFTEnds e = ends;
  e.rho = use_rho ? t.rho : nullptr;
  e.K = use_K ? t.Kfft : nullptr;
  fft_axis_block(t.fft, M1, M2, M3, axis, sign, B, plan, e, ln, (long)blockIdx.x, smem_raw);
}

// the radix plan of a transform of length M (false: M has other prime factors)
static bool fft_plan(int M, FFTPlan* plan) {
  plan->M = M;
  plan->nf = 0;
  int rem = M;
  const int radices[4] = {4, 2, 3, 5};
  for (int r : radices) {
    while (rem % r == 0 && plan->nf < 12) {
      plan->f[plan->nf++] = r;
      rem /= r;
    }
  }
  return rem == 1;
}

hipError_t launch_fft_lines_group(const TailCell* tab, int ncells, int M1, int M2, int M3, int axis, int sign,
                                  int use_rho, int n1, int n2, int n3, int use_K, int l1, int l2, int n_in,
                                  int n_out, int fused, hipStream_t s) {
  FFTPlan plan;
  if (!fft_plan(axis == 0 ? M1 : (axis == 1 ? M2 : M3), &plan)) return hipErrorInvalidValue;
  if (fused && (axis != 2 || !use_K)) return hipErrorInvalidValue;
  const long nlines = (long)l1 * l2;
  if (nlines <= 0 || ncells <= 0) return hipSuccess;
  // every line is transformed the same way whatever B is; with many cells
  // the grid is full without spreading one cell's lines thinly
  const int B = max(1, min(256, 2048 / plan.M));
  const size_t lds = ((size_t)2 * B * plan.M + 2 * (size_t)plan.M) * sizeof(double2);
  FFTEnds ends{nullptr, n1, n2, n3, nullptr};
  FFTLines ln{l1, l2, n_in, n_out, fused};
  hipLaunchKernelGGL(k_fft_axis_group, dim3((unsigned)((nlines + B - 1) / B), ncells), dim3(256), lds, s, tab, M1,
                     M2, M3, axis, sign, B, plan, ends, ln, use_rho, use_K);
  return hipGetLastError();
}

hipError_t launch_fft_lines(double2* data, int M1, int M2, int M3, int axis, int sign, hipStream_t s,
                            const double* rho, int n1, int n2, int n3, const double* K, int l1, int l2, int n_in,
                            int n_out, int fused) {
  FFTPlan plan;
  if (!fft_plan(axis == 0 ? M1 : (axis == 1 ? M2 : M3), &plan)) return hipErrorInvalidValue;
  if (fused && (axis != 2 || !K)) return hipErrorInvalidValue;
  const long nlines = (long)l1 * l2;
  if (nlines <= 0) return hipSuccess;
  // lines per workgroup: up to 2048 points, but small boxes are spread over at
  // least 64 workgroups (each line is transformed the same way wherever it runs)
  int B = max(1, min(256, 2048 / plan.M));
  while (B > 1 && nlines / B < 64) B /= 2;
  const size_t lds = ((size_t)2 * B * plan.M + 2 * (size_t)plan.M) * sizeof(double2);
  FFTEnds ends{rho, n1, n2, n3, K};
  FFTLines ln{l1, l2, n_in, n_out, fused};
  hipLaunchKernelGGL(k_fft_axis, dim3((unsigned)((nlines + B - 1) / B)), dim3(256), lds, s, data, M1, M2, M3,
                     axis, sign, B, plan, ends, ln);
  return hipGetLastError();
}

hipError_t launch_fft_axis(double2* data, int M1, int M2, int M3, int axis, int sign, hipStream_t s,
                           const double* rho, int n1, int n2, int n3, const double* K) {
  const int l1 = axis == 0 ? M2 : M1, l2 = axis == 2 ? M2 : M3;
  const int M = axis == 0 ? M1 : (axis == 1 ? M2 : M3);
  return launch_fft_lines(data, M1, M2, M3, axis, sign, s, rho, n1, n2, n3, K, l1, l2, M, M, 0);
}

// ---------------------------------------------------------------- LDA + V
// Perdew-Zunger 1981, spin-unpolarised; r_s >= 1 uses the Pade form in
// sqrt(r_s), r_s < 1 the high-density logarithmic form; rho < 1e-30 -> 0.
// exchange_too = 0 leaves out the LDA exchange potential (the BJ / TB09
// exchange replaces it); e is always the full LDA energy density
__device__ void pz81(double rho, int exchange_too, double* v, double* e) {
  if (!(rho >= 1e-30)) {
    *v = 0.0;
    *e = 0.0;
    return;
  }
  const double third = 1.0 / 3.0;
  const double pi = 3.14159265358979323846;
  const double rs = cbrt(3.0 / (4.0 * pi * rho));
  const double vx = -cbrt(3.0 * rho / pi);
  const double ex = 0.75 * vx;
  double ec, vc;
  if (rs >= 1.0) {
    const double g = -0.1423, b1 = 1.0529, b2 = 0.3334;
    const double sq = sqrt(rs);
    const double den = 1.0 + b1 * sq + b2 * rs;
    ec = g / den;
    vc = ec * (1.0 + 7.0 / 6.0 * b1 * sq + 4.0 / 3.0 * b2 * rs) / den;
  } else {
    const double A = 0.0311, B = -0.048, C = 0.0020, D = -0.0116;
    const double l = log(rs);
    ec = A * l + B + C * rs * l + D * rs;
    vc = A * l + (B - A * third) + 2.0 * third * C * rs * l + (2.0 * D - C) * third * rs;
  }
  *v = exchange_too ? vx + vc : vc;
  *e = ex + ec;
}

// xc: 0 none, 1 PZ81, 2 and 3 the exchange in vx_mgga plus PZ81 correlation
__device__ __forceinline__ void xc_point(const double2* data, int n1, int n2, int M1, int M2, double vh_scale,
                                         const double* rho, const double* Vloc, int hartree, int xc,
                                         const double* vx_mgga, double* Vd, float* Vf, double* vh_out,
                                         double* exc, size_t p) {
  const int x = (int)(p % n1);
  const int y = (int)((p / n1) % n2);
  const int z = (int)(p / ((size_t)n1 * n2));
  double vh = 0.0;
  if (hartree) vh = data[((size_t)z * M2 + y) * M1 + x].x * vh_scale;
  double vxc = 0.0, e = 0.0;
  if (xc) {
    pz81(rho[p], xc == 1, &vxc, &e);
    if (xc >= 2) vxc += vx_mgga[p];
  }
  const double v = Vloc[p] + vh + vxc;
  Vd[p] = v;
  Vf[p] = (float)v;
  vh_out[p] = vh;
  exc[p] = e;
}

__global__ void k_xc_assemble(const double2* data, int n1, int n2, int n3, int M1, int M2,
                              double vh_scale, const double* rho, const double* Vloc, int hartree,
                              int xc, const double* vx_mgga, double* Vd, float* Vf, double* vh_out,
                              double* exc) {
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t N = (size_t)n1 * n2 * n3;
  if (p >= N) return;
  xc_point(data, n1, n2, M1, M2, vh_scale, rho, Vloc, hartree, xc, vx_mgga, Vd, Vf, vh_out, exc, p);
}

// the same for the cells of a group (cell blockIdx.y; LDA or no xc)
__global__ void k_xc_group(const TailCell* __restrict__ tab, int n1, int n2, int n3, int M1, int M2, int hartree,
                           int xc) {
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t N = (size_t)n1 * n2 * n3;
  if (p >= N) return;
  const TailCell& t = tab[blockIdx.y];
  xc_point(t.fft, n1, n2, M1, M2, t.vh_scale, t.rho, t.Vloc, hartree, xc, nullptr, t.Vd, t.Vf, t.vh, t.exc, p);
}

hipError_t launch_xc_group(const TailCell* tab, int ncells, int n1, int n2, int n3, int M1, int M2, int hartree,
                           int xc, hipStream_t s) {
  if (xc >= 2) return hipErrorInvalidValue;
  const size_t N = (size_t)n1 * n2 * n3;
  hipLaunchKernelGGL(k_xc_group, dim3((unsigned)((N + 255) / 256), ncells), dim3(256), 0, s, tab, n1, n2, n3, M1,
                     M2, hartree, xc);
  return hipGetLastError();
}

hipError_t launch_xc_assemble(const double2* data, int n1, int n2, int n3, int M1, int M2, int M3,
                              double vh_scale, const double* rho, const double* Vloc, int hartree,
                              int xc, const double* vx_mgga, double* Vd, float* Vf, double* vh, double* exc,
                              hipStream_t s) {
  (void)M3;
  const size_t N = (size_t)n1 * n2 * n3;
  hipLaunchKernelGGL(k_xc_assemble, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, data, n1, n2,
                     n3, M1, M2, vh_scale, rho, Vloc, hartree, xc, vx_mgga, Vd, Vf, vh, exc);
  return hipGetLastError();
}

// ---------------------------------------------------------------- finish
// One workgroup: I = -(1/Omega) sum_o f_o [p_o + kappaJ_k norm_o + jNL_o],
// the orbital energy sum_o f_o [kin + kappaJ.p + 1/2 |kappaJ|^2 norm + vloc + E_NL],
// and the occupied norm; f_o = 2 w_k. Thread t sums orbitals t, t+1024, ...
// in order, then a fixed pairwise tree combines the threads. nanflag gets
// bit 0 for a non-finite norm or momentum, bit 1 (only when norm_tol > 0)
// for a norm further than norm_tol from 1.
__device__ __forceinline__ void finish_block(const double* obs, int tiles, const double* jnl, int use_nl,
                                             const double* kw, const double* kappaJ, int n_orb, int n_k,
                                             double dV, double volume, int* counter, int bump, double* Jtab,
                                             double* scalars, int* nanflag, double norm_tol, double (*red)[5]) {
  const int t = threadIdx.x;
  const int n_tot = n_orb * n_k;
  double cx = 0, cy = 0, cz = 0, en = 0, nr = 0;
  int bad = 0;
  for (int o = t; o < n_tot; o += blockDim.x) {
    const int k = o / n_orb;
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int tl = 0; tl < tiles; ++tl)
      for (int i = 0; i < 6; ++i) s[i] += obs[((size_t)o * tiles + tl) * 8 + i];
    for (int i = 0; i < 6; ++i) s[i] *= dV;
    const double f = 2.0 * kw[k];
    const double kx = kappaJ[3 * k], ky = kappaJ[3 * k + 1], kz = kappaJ[3 * k + 2];
    double jx = 0, jy = 0, jz = 0, enl = 0;
    if (use_nl) {
      jx = jnl[4 * (size_t)o];
      jy = jnl[4 * (size_t)o + 1];
      jz = jnl[4 * (size_t)o + 2];
      enl = jnl[4 * (size_t)o + 3];
    }
    cx += f * (s[1] + kx * s[0] + jx);
    cy += f * (s[2] + ky * s[0] + jy);
    cz += f * (s[3] + kz * s[0] + jz);
    en += f * (s[4] + kx * s[1] + ky * s[2] + kz * s[3] + 0.5 * (kx * kx + ky * ky + kz * kz) * s[0] +
               s[5] + enl);
    nr += f * s[0];
    if (!isfinite(s[0]) || !isfinite(s[1]) || !isfinite(s[2]) || !isfinite(s[3])) bad |= 1;
    else if (norm_tol > 0.0 && fabs(s[0] - 1.0) > norm_tol) bad |= 2;
  }
  red[t][0] = cx;
  red[t][1] = cy;
  red[t][2] = cz;
  red[t][3] = en;
  red[t][4] = nr;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w)
      for (int i = 0; i < 5; ++i) red[t][i] += red[t + w][i];
    __syncthreads();
  }
  if (bad) atomicOr(nanflag, bad);
  if (t == 0) {
    const double J[3] = {-red[0][0] / volume, -red[0][1] / volume, -red[0][2] / volume};
    for (int i = 0; i < 3; ++i) scalars[i] = J[i];
    scalars[3] = red[0][3];
    scalars[4] = red[0][4];
    if (bump) {
      const int n = *counter;
      for (int i = 0; i < 3; ++i) Jtab[3 * (size_t)n + i] = J[i];
      *counter = n + 1;
    }
  }
}

__global__ __launch_bounds__(1024) void k_finish(const double* obs, int tiles, const double* jnl,
                                                 int use_nl, const double* kw, const double* kappaJ,
                                                 int n_orb, int n_k, double dV, double volume,
                                                 int* counter, int bump, double* Jtab,
                                                 double* scalars, int* nanflag, double norm_tol) {
  __shared__ double red[1024][5];
  finish_block(obs, tiles, jnl, use_nl, kw, kappaJ, n_orb, n_k, dV, volume, counter, bump, Jtab, scalars, nanflag,
               norm_tol, red);
}

// one step's current of every cell of a group (one workgroup per cell)
__global__ __launch_bounds__(1024) void k_finish_group(const TailCell* __restrict__ tab, int tiles) {
  __shared__ double red[1024][5];
  const TailCell& c = tab[blockIdx.x];
  finish_block(c.obs, tiles, c.jnl, c.use_nl, c.kw, c.kappaJ, c.n_orb, c.n_k, c.dV, c.volume, c.counter, 1, c.Jtab,
               c.scalars, c.nanflag, c.norm_tol, red);
}

hipError_t launch_finish_group(const TailCell* tab, int ncells, int tiles, hipStream_t s) {
  hipLaunchKernelGGL(k_finish_group, dim3(ncells), dim3(1024), 0, s, tab, tiles);
  return hipGetLastError();
}

hipError_t launch_finish(const double* obs, int tiles, const double* jnl, int use_nl,
                         const double* kw, const double* kappaJ, int n_orb, int n_k, double dV,
                         double volume, int* counter, int bump, double* Jtab, double* scalars,
                         int* nanflag, double norm_tol, hipStream_t s) {
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, obs, tiles, jnl, use_nl, kw, kappaJ, n_orb,
                     n_k, dV, volume, counter, bump, Jtab, scalars, nanflag, norm_tol);
  return hipGetLastError();
}

// ---------------------------------------------------------------- grid sums
// out[0] = 1/2 h^3 sum rho V_H, out[1] = h^3 sum rho eps_xc,
// out[2..4] = -h^3 sum (r - centre)(rho - rho0), out[5] = h^3 sum rho.
__global__ __launch_bounds__(1024) void k_grid_sums(const double* rho, const double* rho0,
                                                    const double* vh, const double* exc, Geometry g,
                                                    double* out) {
  __shared__ double red[1024][6];
  const int t = threadIdx.x;
  const size_t N = (size_t)g.n1 * g.n2 * g.n3;
  double s[6] = {0, 0, 0, 0, 0, 0};
  for (size_t p = t; p < N; p += blockDim.x) {
    const int x = (int)(p % g.n1);
    const int y = (int)((p / g.n1) % g.n2);
    const int z = (int)(p / ((size_t)g.n1 * g.n2));
    const double r = rho[p];
    const double dr = r - rho0[p];
    s[0] += r * vh[p];
    s[1] += r * exc[p];
    s[2] += (x - 0.5 * (g.n1 - 1)) * g.h1 * dr;
    s[3] += (y - 0.5 * (g.n2 - 1)) * g.h2 * dr;
    s[4] += (z - 0.5 * (g.n3 - 1)) * g.h3 * dr;
    s[5] += r;
  }
  for (int i = 0; i < 6; ++i) red[t][i] = s[i];
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (t < w)
      for (int i = 0; i < 6; ++i) red[t][i] += red[t + w][i];
    __syncthreads();
  }
  if (t == 0) {
    const double dV = g.h1 * g.h2 * g.h3;
    out[0] = 0.5 * dV * red[0][0];
    out[1] = dV * red[0][1];
    out[2] = -dV * red[0][2];
    out[3] = -dV * red[0][3];
    out[4] = -dV * red[0][4];
    out[5] = dV * red[0][5];
  }
}

hipError_t launch_grid_sums(const double* rho, const double* rho0, const double* vh,
                            const double* exc, Geometry g, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_grid_sums, dim3(1), dim3(1024), 0, s, rho, rho0, vh, exc, g, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- conversions
template <typename T>
__global__ void k_convert_in(const double2* src, typename Vec2<T>::type* dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 v = src[i];
  typename Vec2<T>::type o;
  o.x = (T)v.x;
  o.y = (T)v.y;
  dst[i] = o;
}
template <typename T>
__global__ void k_convert_out(const typename Vec2<T>::type* src, double2* dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const auto v = src[i];
  dst[i] = make_double2((double)v.x, (double)v.y);
}
template <typename T>
hipError_t launch_convert_in(const double2* src, typename Vec2<T>::type* dst, size_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_convert_in<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_convert_out(const typename Vec2<T>::type* src, double2* dst, size_t n, hipStream_t s) {
  hipLaunchKernelGGL((k_convert_out<T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}
template hipError_t launch_convert_in<double>(const double2*, double2*, size_t, hipStream_t);
template hipError_t launch_convert_in<float>(const double2*, float2*, size_t, hipStream_t);
template hipError_t launch_convert_out<double>(const double2*, double2*, size_t, hipStream_t);
template hipError_t launch_convert_out<float>(const float2*, double2*, size_t, hipStream_t);

// w <- exp(-i F0 r_axis) w with r from the box centre (isolated kick, Sec. 3.1)
template <typename T>
__global__ void k_kick(typename Vec2<T>::type* w, Geometry g, double F0, int axis, size_t total) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const size_t N = (size_t)g.n1 * g.n2 * g.n3;
  const size_t p = i % N;
  int c;
  double h;
  int n;
  if (axis == 0) {
    c = (int)(p % g.n1);
    h = g.h1;
    n = g.n1;
  } else if (axis == 1) {
    c = (int)((p / g.n1) % g.n2);
    h = g.h2;
    n = g.n2;
  } else {
    c = (int)(p / ((size_t)g.n1 * g.n2));
    h = g.h3;
    n = g.n3;
  }
  const double r = (c - 0.5 * (n - 1)) * h;
  double sn, cs;
  sincos(-F0 * r, &sn, &cs);
  auto v = w[i];
  const double re = (double)v.x, im = (double)v.y;
  v.x = (T)(re * cs - im * sn);
  v.y = (T)(re * sn + im * cs);
  w[i] = v;
}
template <typename T>
hipError_t launch_kick(typename Vec2<T>::type* w, Geometry g, double F0, int axis, size_t n_orb_tot,
                       hipStream_t s) {
  const size_t total = n_orb_tot * (size_t)g.n1 * g.n2 * g.n3;
  hipLaunchKernelGGL((k_kick<T>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, w, g, F0,
                     axis, total);
  return hipGetLastError();
}
template hipError_t launch_kick<double>(double2*, Geometry, double, int, size_t, hipStream_t);
template hipError_t launch_kick<float>(float2*, Geometry, double, int, size_t, hipStream_t);

__global__ void k_real_part(const double2* src, double* dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i].x;
}
hipError_t launch_real_part(const double2* src, double* dst, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_real_part, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

__global__ void k_fill(double* p, double v, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
hipError_t launch_fill(double* p, double v, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

// dst = src, 8 bytes per thread (both 8-byte aligned, bytes a multiple of 8)
__global__ void k_copy8(const double* __restrict__ src, double* __restrict__ dst, size_t n8) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n8) dst[i] = src[i];
}
hipError_t launch_copy8(const void* src, void* dst, size_t bytes, hipStream_t s) {
  const size_t n8 = bytes / 8;
  if (n8 == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy8, dim3((unsigned)((n8 + 255) / 256)), dim3(256), 0, s,
                     static_cast<const double*>(src), static_cast<double*>(dst), n8);
  return hipGetLastError();
}

// predictor-corrector: V = (V_n + V_pred) / 2 in FP64 and its stage-precision copy
__global__ void k_mid_potential(const double* __restrict__ Vn, double* __restrict__ Vd, float* __restrict__ Vf,
                                size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = 0.5 * (Vn[i] + Vd[i]);
  Vd[i] = v;
  Vf[i] = (float)v;
}
hipError_t launch_mid_potential(const double* Vn, double* Vd, float* Vf, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_mid_potential, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Vn, Vd, Vf, n);
  return hipGetLastError();
}

__global__ void k_set_int(int* p, int v) { *p = v; }
hipError_t launch_set_int(int* p, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, p, v);
  return hipGetLastError();
}

}  // namespace td
