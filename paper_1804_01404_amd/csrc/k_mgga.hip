// Becke-Johnson and Tran-Blaha exchange potentials (Sec. 4.1 names both as
// alternatives to the adiabatic LDA; the formulas are the published ones:
// Becke and Johnson 2006, Tran and Blaha 2009, with the Becke-Roussel 1989
// exchange-hole potential at gamma = 1). Spin-saturated: rho_s = rho/2,
// t_s = tau/2.
//
//   tau(r)  = sum_k w_k sum_n |(grad_h + i kappa_k) w_nk(r)|^2   (= 2 x 1/2 |.|^2)
//   v_x     = c v_BR + (3c - 2) (1/pi) sqrt(5/12) sqrt(2 t_s / rho_s)
//   v_BR    = -(1 - e^-x - x e^-x / 2) / b,   b^3 = x^3 e^-x / (8 pi rho_s)
//   x       : x e^(-2x/3) / (x - 2) = (2/3) pi^(2/3) rho_s^(5/3) / Q_s
//   Q_s     = (lap rho_s - 2 (T_s - |grad rho_s|^2 / (4 rho_s))) / 6,  T_s = tau
//   c       = 1 (BJ) or -0.012 + 1.023 sqrt(g), g = (1/Omega) int |grad rho| / rho (TB09)
//
// kappa_k = k + A/c for the A at the orbitals' time (kappaJ of the last step),
// grad and lap of rho use the same 9-point differences as the Hamiltonian,
// and points with rho < 1e-30 get v_x = 0. Everything is FP64; reductions
// run in a fixed order.
#include "internal.h"

namespace td {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kRhoMin = 1e-30;

// neighbour offset along one axis: j + m wrapped (periodic) or -1 outside
__device__ __forceinline__ int nb(int j, int m, int n, int periodic) {
  int q = j + m;
  if (periodic) {
    q = q < 0 ? q + n : (q >= n ? q - n : q);
    return q;
  }
  return (q < 0 || q >= n) ? -1 : q;
}

// the 9-point first derivatives of a real grid field at (x, y, z)
__device__ void grad_field(const double* f, const MggaArgs& a, int x, int y, int z, double out[3]) {
  const Geometry& g = a.g;
  const size_t row = (size_t)g.n1;
  const size_t plane = (size_t)g.n1 * g.n2;
  const size_t base_x = (size_t)z * plane + (size_t)y * row;
  const size_t base_y = (size_t)z * plane + x;
  const size_t base_z = (size_t)y * row + x;
  double d[3] = {0.0, 0.0, 0.0};
  for (int m = 1; m <= kHalf; ++m) {
    const int xp = nb(x, m, g.n1, g.periodic), xm = nb(x, -m, g.n1, g.periodic);
    const int yp = nb(y, m, g.n2, g.periodic), ym = nb(y, -m, g.n2, g.periodic);
    const int zp = nb(z, m, g.n3, g.periodic), zm = nb(z, -m, g.n3, g.periodic);
    const double fxp = xp >= 0 ? f[base_x + xp] : 0.0, fxm = xm >= 0 ? f[base_x + xm] : 0.0;
    const double fyp = yp >= 0 ? f[base_y + yp * row] : 0.0, fym = ym >= 0 ? f[base_y + ym * row] : 0.0;
    const double fzp = zp >= 0 ? f[base_z + zp * plane] : 0.0, fzm = zm >= 0 ? f[base_z + zm * plane] : 0.0;
    d[0] += a.d1[0][m - 1] * (fxp - fxm);
    d[1] += a.d1[1][m - 1] * (fyp - fym);
    d[2] += a.d1[2][m - 1] * (fzp - fzm);
  }
  out[0] = d[0];
  out[1] = d[1];
  out[2] = d[2];
}

// the 9-point Laplacian of a real grid field at (x, y, z)
__device__ double lap_field(const double* f, const MggaArgs& a, int x, int y, int z) {
  const Geometry& g = a.g;
  const size_t row = (size_t)g.n1;
  const size_t plane = (size_t)g.n1 * g.n2;
  const size_t p = (size_t)z * plane + (size_t)y * row + x;
  const double f0 = f[p];
  double s = (a.d2[0][0] + a.d2[1][0] + a.d2[2][0]) * f0;
  const size_t base_x = (size_t)z * plane + (size_t)y * row;
  const size_t base_y = (size_t)z * plane + x;
  const size_t base_z = (size_t)y * row + x;
  for (int m = 1; m <= kHalf; ++m) {
    const int xp = nb(x, m, g.n1, g.periodic), xm = nb(x, -m, g.n1, g.periodic);
    const int yp = nb(y, m, g.n2, g.periodic), ym = nb(y, -m, g.n2, g.periodic);
    const int zp = nb(z, m, g.n3, g.periodic), zm = nb(z, -m, g.n3, g.periodic);
    const double sx = (xp >= 0 ? f[base_x + xp] : 0.0) + (xm >= 0 ? f[base_x + xm] : 0.0);
    const double sy = (yp >= 0 ? f[base_y + yp * row] : 0.0) + (ym >= 0 ? f[base_y + ym * row] : 0.0);
    const double sz = (zp >= 0 ? f[base_z + zp * plane] : 0.0) + (zm >= 0 ? f[base_z + zm * plane] : 0.0);
    s += a.d2[0][m] * sx + a.d2[1][m] * sy + a.d2[2][m] * sz;
  }
  return s;
}

__device__ __forceinline__ double br_f(double x) { return x * exp(-2.0 * x / 3.0) / (x - 2.0); }

// Root of x e^(-2x/3) / (x - 2) = y: (0, 2) for y < 0, (2, inf) for y > 0,
// 2 for y = +-inf; bisection until the midpoint meets an end of the bracket.
__device__ double br_root(double y) {
  if (!isfinite(y)) return 2.0;
  double lo, hi;
  if (y < 0.0) {
    lo = 0.0;
    hi = 2.0;
  } else {
    lo = 2.0;
    hi = 4.0;
    for (int i = 0; i < 64 && br_f(hi) > y; ++i) {
      lo = hi;
      hi *= 2.0;
    }
  }
  for (int i = 0; i < 2200; ++i) {
    const double mid = 0.5 * (lo + hi);
    if (!(mid > lo && mid < hi)) break;
    if (br_f(mid) > y)
      lo = mid;
    else
      hi = mid;
  }
  return 0.5 * (lo + hi);
}

}  // namespace

// ---------------------------------------------------------------- rho and tau
// part_rho[c][p] = sum_{o in chunk c} 2 w_k |w_o(p)|^2 and
// part_tau[c][p] = sum_{o in chunk c} w_k |(grad_h + i kappa_k) w_o(p)|^2, in order.
// The 24 neighbour loads of an orbital carry no branch (outside an isolated
// box the index points back at p and the value is masked to 0), so they
// issue back to back. Launch ids are mapped so that the point blocks of one
// orbital chunk run on one XCD and share its L2: hardware block b runs on
// XCD b mod 8, and the blocks of each XCD take consecutive logical ids.
template <typename T, bool PERIODIC>
__global__ __launch_bounds__(256) void k_rho_tau_partial(const typename Vec2<T>::type* __restrict__ w,
                                                         const double* __restrict__ kw,
                                                         const double* __restrict__ kappa, MggaArgs a, int chunk,
                                                         double* __restrict__ part_rho,
                                                         double* __restrict__ part_tau) {
  const Geometry& g = a.g;
  const int N = g.n1 * g.n2 * g.n3;
  const int nbx = (N + 255) / 256;
  const int total = gridDim.x, b8 = blockIdx.x % 8, q8 = total / 8, r8 = total % 8;
  const int L = b8 * q8 + min(b8, r8) + blockIdx.x / 8;
  const int cy = L / nbx;
  const int p = (L % nbx) * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const int x = p % g.n1, y = (p / g.n1) % g.n2, z = p / (g.n1 * g.n2);
  // flat indices of the 24 neighbours (+m, -m per axis); outside an isolated box: p, masked
  int off[3][2 * kHalf];
  bool in[3][2 * kHalf];
  for (int m = 1; m <= kHalf; ++m) {
    const int qs[6] = {nb(x, m, g.n1, PERIODIC), nb(x, -m, g.n1, PERIODIC), nb(y, m, g.n2, PERIODIC),
                       nb(y, -m, g.n2, PERIODIC), nb(z, m, g.n3, PERIODIC), nb(z, -m, g.n3, PERIODIC)};
    const int js[3] = {x, y, z};
    const int st[3] = {1, g.n1, g.n1 * g.n2};
    for (int mu = 0; mu < 3; ++mu)
      for (int sgn = 0; sgn < 2; ++sgn) {
        const int q = qs[2 * mu + sgn];
        in[mu][2 * (m - 1) + sgn] = q >= 0;
        off[mu][2 * (m - 1) + sgn] = q >= 0 ? p + (q - js[mu]) * st[mu] : p;
      }
  }
  const int n_tot = g.n_orb * g.n_k;
  const int o0 = cy * chunk;
  const int o1 = min(n_tot, o0 + chunk);
  double acc_r = 0.0, acc_t = 0.0;
  for (int o = o0; o < o1; ++o) {
    const int k = o / g.n_orb;
    const auto* wo = w + (size_t)o * N;
    typename Vec2<T>::type v[3][2 * kHalf];
    for (int mu = 0; mu < 3; ++mu)
      for (int j = 0; j < 2 * kHalf; ++j) v[mu][j] = wo[off[mu][j]];
    const auto c0 = wo[p];
    const double re = (double)c0.x, im = (double)c0.y;
    double t = 0.0;
    for (int mu = 0; mu < 3; ++mu) {
      double dr = 0.0, di = 0.0;
      for (int m = 0; m < kHalf; ++m) {
        double pr = (double)v[mu][2 * m].x, pi = (double)v[mu][2 * m].y;
        double mr = (double)v[mu][2 * m + 1].x, mi = (double)v[mu][2 * m + 1].y;
        if (!PERIODIC) {
          pr = in[mu][2 * m] ? pr : 0.0;
          pi = in[mu][2 * m] ? pi : 0.0;
          mr = in[mu][2 * m + 1] ? mr : 0.0;
          mi = in[mu][2 * m + 1] ? mi : 0.0;
        }
        dr += a.d1[mu][m] * (pr - mr);
        di += a.d1[mu][m] * (pi - mi);
      }
      // (d + i kappa w)
      const double km = kappa[3 * k + mu];
      const double gr = dr - km * im, gi = di + km * re;
      t += gr * gr + gi * gi;
    }
    acc_r += 2.0 * kw[k] * (re * re + im * im);
    acc_t += kw[k] * t;
  }
  part_rho[(size_t)cy * N + p] = acc_r;
  part_tau[(size_t)cy * N + p] = acc_t;
}

// The same partial sums for periodic cells whose xy plane fits one workgroup:
// a thread owns one column of a z slab (kTauSlab planes), the x/y
// neighbours of the current plane come from LDS (double-buffered, one
// barrier per plane) and the z neighbours from a queue in registers, so each
// orbital value is read once from memory (plus the 8 halo planes of the
// slab) instead of 25 times. Per point the orbitals are summed in the same
// order as above.
constexpr int kTauSlab = 10;

template <typename T>
__global__ __launch_bounds__(1024) void k_rho_tau_plane(const typename Vec2<T>::type* __restrict__ w,
                                                        const double* __restrict__ kw,
                                                        const double* __restrict__ kappa, MggaArgs a, int chunk,
                                                        double* __restrict__ part_rho,
                                                        double* __restrict__ part_tau) {
  using T2 = typename Vec2<T>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T2* pl = reinterpret_cast<T2*>(smem_raw);
  const Geometry& g = a.g;
  const int n1 = g.n1, n2 = g.n2, n3 = g.n3, plane = n1 * n2;
  const size_t N = (size_t)plane * n3;
  const int nsl = (n3 + kTauSlab - 1) / kTauSlab;
  const int cy = blockIdx.x / nsl, slab = blockIdx.x - cy * nsl;
  const int z0 = slab * kTauSlab, z1 = min(n3, z0 + kTauSlab);
  const int tid = threadIdx.x;
  const bool active = tid < plane;
  const int col = active ? tid : 0;
  const int x = col % n1, y = col / n1;
  int ox[2 * kHalf], oy[2 * kHalf];  // +m, -m for m = 1..4, wrapped in the plane
  for (int m = 1; m <= kHalf; ++m) {
    ox[2 * (m - 1)] = y * n1 + (x + m) % n1;
    ox[2 * (m - 1) + 1] = y * n1 + (x - m + n1) % n1;
    oy[2 * (m - 1)] = ((y + m) % n2) * n1 + x;
    oy[2 * (m - 1) + 1] = ((y - m + n2) % n2) * n1 + x;
  }
  double ar[kTauSlab], at[kTauSlab];
#pragma unroll
  for (int i = 0; i < kTauSlab; ++i) ar[i] = at[i] = 0.0;
  const int n_tot = g.n_orb * g.n_k;
  const int o0 = cy * chunk;
  const int o1 = min(n_tot, o0 + chunk);
  int step = 0;
  for (int o = o0; o < o1; ++o) {
    const int k = o / g.n_orb;
    const T2* wo = w + (size_t)o * N;
    auto ld = [&](int z) {
      z = (z % n3 + n3) % n3;
      return wo[(size_t)z * plane + col];
    };
    T2 q[9];
#pragma unroll
    for (int i = 0; i < 8; ++i) q[i] = ld(z0 + i - 4);
    T2 nxt = ld(z0 + 4);
#pragma unroll
    for (int zz = 0; zz < kTauSlab; ++zz) {
      const int z = z0 + zz;
      if (z < z1) {  // uniform over the workgroup
        q[8] = nxt;
        if (z + 1 < z1) nxt = ld(z + 5);
        T2* buf = pl + (step & 1) * plane;
        ++step;
        if (active) buf[tid] = q[4];
        __syncthreads();
        if (active) {
          const double re = (double)q[4].x, im = (double)q[4].y;
          double t = 0.0;
#pragma unroll
          for (int mu = 0; mu < 3; ++mu) {
            // the differences and their weighted sum in the orbitals' own
            // precision (for complex FP32 an error at the orbitals' own
            // rounding level), the kappa term and the square in FP64
            T dr = 0, di = 0;
#pragma unroll
            for (int m = 0; m < kHalf; ++m) {
              T2 pv, mv;
              if (mu == 0) {
                pv = buf[ox[2 * m]];
                mv = buf[ox[2 * m + 1]];
              } else if (mu == 1) {
                pv = buf[oy[2 * m]];
                mv = buf[oy[2 * m + 1]];
              } else {
                pv = q[5 + m];
                mv = q[3 - m];
              }
              const T cm = (T)a.d1[mu][m];
              dr += cm * (pv.x - mv.x);
              di += cm * (pv.y - mv.y);
            }
            const double km = kappa[3 * k + mu];
            const double gr = dr - km * im, gi = di + km * re;
            t += gr * gr + gi * gi;
          }
          ar[zz] += 2.0 * kw[k] * (re * re + im * im);
          at[zz] += kw[k] * t;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) q[i] = q[i + 1];
      }
    }
  }
  if (active) {
#pragma unroll
    for (int zz = 0; zz < kTauSlab; ++zz) {
      const int z = z0 + zz;
      if (z < z1) {
        part_rho[(size_t)cy * N + (size_t)z * plane + tid] = ar[zz];
        part_tau[(size_t)cy * N + (size_t)z * plane + tid] = at[zz];
      }
    }
  }
}

// Orbitals per chunk of the partial sums. The plane sweep runs one workgroup
// per (chunk, z slab), each walking its chunk's orbitals in order, so with 64
// orbitals a chunk a 20^3 cell of 8192 orbitals fills only one workgroup per
// compute unit; smaller chunks (down to 8) give at least about 1024
// workgroups at the price of more partial planes to reduce.
int rho_tau_chunk(const Geometry& g, int n_tot) {
  const int plane = g.n1 * g.n2;
  if (!(g.periodic && plane <= 1024)) return 64;
  const int nsl = (g.n3 + kTauSlab - 1) / kTauSlab;
  const long want = (long)n_tot * nsl / 1024;
  return (int)std::max(8L, std::min(64L, want));
}

template <typename T>
hipError_t launch_rho_tau_partial(const typename Vec2<T>::type* w, const double* kw, const double* kappa,
                                  const MggaArgs& a, int chunk, double* part_rho, double* part_tau,
                                  hipStream_t s) {
  const int N = a.g.n1 * a.g.n2 * a.g.n3;
  const int nchunks = (a.g.n_orb * a.g.n_k + chunk - 1) / chunk;
  const int plane = a.g.n1 * a.g.n2;
  if (a.g.periodic && plane <= 1024) {
    const int nsl = (a.g.n3 + kTauSlab - 1) / kTauSlab;
    const size_t lds = (size_t)2 * plane * sizeof(typename Vec2<T>::type);
    hipLaunchKernelGGL((k_rho_tau_plane<T>), dim3((unsigned)(nchunks * nsl)), dim3(((plane + 63) / 64) * 64), lds,
                       s, w, kw, kappa, a, chunk, part_rho, part_tau);
    return hipGetLastError();
  }
  const dim3 grid(((N + 255) / 256) * nchunks);
  if (a.g.periodic)
    hipLaunchKernelGGL((k_rho_tau_partial<T, true>), grid, dim3(256), 0, s, w, kw, kappa, a, chunk, part_rho,
                       part_tau);
  else
    hipLaunchKernelGGL((k_rho_tau_partial<T, false>), grid, dim3(256), 0, s, w, kw, kappa, a, chunk, part_rho,
                       part_tau);
  return hipGetLastError();
}
template hipError_t launch_rho_tau_partial<double>(const double2*, const double*, const double*, const MggaArgs&,
                                                   int, double*, double*, hipStream_t);
template hipError_t launch_rho_tau_partial<float>(const float2*, const double*, const double*, const MggaArgs&,
                                                  int, double*, double*, hipStream_t);

// ---------------------------------------------------------------- c of TB09
// gpart[b] = sum over the points of block b of |grad_h rho| / rho (rho >= 1e-30),
// combined by a fixed pairwise tree.
__global__ __launch_bounds__(256) void k_mgga_gpart(const double* __restrict__ rho, MggaArgs a,
                                                    double* __restrict__ gpart) {
  __shared__ double red[256];
  const Geometry& g = a.g;
  const int N = g.n1 * g.n2 * g.n3;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (p < N && rho[p] >= kRhoMin) {
    const int x = p % g.n1, y = (p / g.n1) % g.n2, z = p / (g.n1 * g.n2);
    double d[3];
    grad_field(rho, a, x, y, z, d);
    v = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) / rho[p];
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) gpart[blockIdx.x] = red[0];
}

// one workgroup: g = dV / Omega * sum_b gpart[b] (thread t sums b = t, t + 256,
// ... in order, then the tree); cval[0] = c, cval[1] = g
__global__ __launch_bounds__(256) void k_mgga_c(const double* __restrict__ gpart, int nblocks, double scale,
                                                int tb09, double* __restrict__ cval) {
  __shared__ double red[256];
  double v = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += 256) v += gpart[b];
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double gg = red[0] * scale;
    cval[0] = tb09 ? -0.012 + 1.023 * sqrt(gg) : 1.0;
    cval[1] = gg;
  }
}

// ---------------------------------------------------------------- v_x
__global__ __launch_bounds__(256) void k_mgga_vx(const double* __restrict__ rho, const double* __restrict__ tau,
                                                 const double* __restrict__ cval, MggaArgs a,
                                                 double* __restrict__ vx) {
  const Geometry& g = a.g;
  const int N = g.n1 * g.n2 * g.n3;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const double r = rho[p];
  if (!(r >= kRhoMin)) {
    vx[p] = 0.0;
    return;
  }
  const int x = p % g.n1, y = (p / g.n1) % g.n2, z = p / (g.n1 * g.n2);
  double d[3];
  grad_field(rho, a, x, y, z, d);
  const double lap = lap_field(rho, a, x, y, z);
  const double c = cval[0];
  // one spin channel of the saturated density
  const double rs = 0.5 * r;
  const double gsq = 0.25 * (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  const double ls = 0.5 * lap;
  const double ts = 0.5 * tau[p];
  const double Ts = 2.0 * ts;
  const double D = Ts - 0.25 * gsq / rs;
  const double Q = (ls - 2.0 * D) / 6.0;
  const double yv = (2.0 / 3.0) * pow(kPi, 2.0 / 3.0) * pow(rs, 5.0 / 3.0) / Q;
  const double xr = br_root(yv);
  const double ex = exp(-xr);
  const double b = cbrt(xr * xr * xr * ex / (8.0 * kPi * rs));
  const double vbr = -(1.0 - ex - 0.5 * xr * ex) / b;
  const double kin = sqrt(5.0 / 12.0) / kPi * sqrt(2.0 * ts / rs);
  vx[p] = c * vbr + (3.0 * c - 2.0) * kin;
}

hipError_t launch_mgga_potential(const double* rho, const double* tau, const MggaArgs& a, int tb09, double dV,
                                 double volume, double* gpart, double* cval, double* vx, hipStream_t s) {
  const int N = a.g.n1 * a.g.n2 * a.g.n3;
  const int nb = (N + 255) / 256;
  hipLaunchKernelGGL(k_mgga_gpart, dim3(nb), dim3(256), 0, s, rho, a, gpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mgga_c, dim3(1), dim3(256), 0, s, gpart, nb, dV / volume, tb09, cval);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mgga_vx, dim3(nb), dim3(256), 0, s, rho, tau, cval, a, vx);
  return hipGetLastError();
}

}  // namespace td
