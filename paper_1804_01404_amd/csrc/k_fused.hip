// Whole time step of one orbital with the orbital resident in LDS.
//
// For cells whose orbital fits in LDS (n1 n2 <= 512, n3 in {12, 16, 20},
// N * sizeof(complex) + tables <= 160 KB), one workgroup owns one orbital and
// runs all four Horner stages u_{s-1} = w + (-i dt / s) h u_s, s = 4..1
// (Program Summary: fourth-order truncated Taylor expansion; Sec. 4.1,
// Eq. TDKS_solid for h), with
//   * u_s in LDS, w and u_{s-1} in registers (thread = one (x, y) column);
//   * the Kleinman-Bylander projections u_p = <beta_p^kappa|u_s> of every atom
//     formed in the workgroup before each stage (one wavefront per atom,
//     fixed-order shuffle reductions, FP64) and added back by a scatter over
//     each atom's sphere into the LDS copy (atoms coloured so that spheres of
//     one colour are disjoint: no atomics, a fixed summation order);
//   * after the last stage: w_new written once, then the observables of
//     w_new (norm, momentum, kinetic and local sums, FP64 accumulation) and
//     the moment projections for the nonlocal current at t_{n+1}.
// HBM traffic per orbital point and step: read w once, write w_new once.
#include "internal.h"

namespace td {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename T, int N3, bool PERIODIC, int MAXT>
__global__ __launch_bounds__(MAXT) void k_fused(FusedArgs<T> a) {
  using T2 = typename Vec2<T>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const Geometry& g = a.g;
  const int n1 = g.n1, n2 = g.n2;
  const int plane = n1 * n2;
  const int N = plane * N3;
  const int n_atoms = a.nl.n_atoms;
  const int S = a.nl.n_ent;
  T2* u = reinterpret_cast<T2*>(smem_raw);
  const size_t ubytes = ((size_t)N * sizeof(T2) + 15) & ~(size_t)15;
  double2* eu = reinterpret_cast<double2*>(smem_raw + ubytes);            // [n_atoms][4]
  double* red = reinterpret_cast<double*>(eu + (size_t)n_atoms * kMaxProj);  // [16][8]

  const int o = blockIdx.x;
  const int k = o / g.n_orb;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6, nwaves = blockDim.x >> 6;
  const int tx = tid % n1, ty = tid / n1;
  const bool active = ty < n2;
  const int col = active ? ty * n1 + tx : 0;

  // in-plane neighbour offsets (periodic wrap) and validity (isolated)
  int oxp[4], oxm[4], oyp[4], oym[4];
  bool vxp[4], vxm[4], vyp[4], vym[4];
#pragma unroll
  for (int m = 1; m <= 4; ++m) {
    const int xp = tx + m, xm = tx - m, yp = ty + m, ym = ty - m;
    vxp[m - 1] = PERIODIC || xp < n1;
    vxm[m - 1] = PERIODIC || xm >= 0;
    vyp[m - 1] = PERIODIC || yp < n2;
    vym[m - 1] = PERIODIC || ym >= 0;
    oxp[m - 1] = ty * n1 + (xp % n1);
    oxm[m - 1] = ty * n1 + ((xm + n1) % n1);
    oyp[m - 1] = (yp % n2) * n1 + tx;
    oym[m - 1] = ((ym + n2) % n2) * n1 + tx;
  }

  T2* __restrict__ wg = a.w + (size_t)o * N;
  T2 w[N3], un[N3];
#pragma unroll
  for (int z = 0; z < N3; ++z) {
    T2 v;
    v.x = 0;
    v.y = 0;
    if (active) v = wg[z * plane + col];
    w[z] = v;
    if (active) u[z * plane + col] = v;
  }

  const double kx = a.kappa[3 * k], ky = a.kappa[3 * k + 1], kz = a.kappa[3 * k + 2];
  T cx[4], cy[4], cz[4], bx[4], by[4], bz[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    cx[m] = (T)a.lap[0][m + 1];
    cy[m] = (T)a.lap[1][m + 1];
    cz[m] = (T)a.lap[2][m + 1];
    bx[m] = (T)(kx * a.dh[0][m]);
    by[m] = (T)(ky * a.dh[1][m]);
    bz[m] = (T)(kz * a.dh[2][m]);
  }
  const T diag = (T)(a.cdiag + 0.5 * (kx * kx + ky * ky + kz * kz));
  T ext = 0, ez = 0;
  if (a.efield) {
    ext = (T)(a.efield[0] * (tx - 0.5 * (n1 - 1)) * g.h1 + a.efield[1] * (ty - 0.5 * (n2 - 1)) * g.h2);
    ez = (T)(a.efield[2] * g.h3);
  }
  const double2* __restrict__ phk = a.nl.phk + (size_t)k * S;
  __syncthreads();

#pragma unroll 1
  for (int s = 4; s >= 1; --s) {
    // ---- projections of u_s: one wavefront per atom, FP64
    if (n_atoms > 0) {
      for (int at = wave; at < n_atoms; at += nwaves) {
        const int e0 = a.nl.atom_start[at], e1 = a.nl.atom_start[at + 1];
        double acc[2 * kMaxProj] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int e = e0 + lane; e < e1; e += 64) {
          const T2 v = u[a.nl.ent_idx[e]];
          const double2 p1 = phk[e], p2 = a.phA[e];
          const double pr = p1.x * p2.x - p1.y * p2.y, pim = p1.x * p2.y + p1.y * p2.x;
          const double gr = pr * (double)v.x - pim * (double)v.y;
          const double gi = pr * (double)v.y + pim * (double)v.x;
#pragma unroll
          for (int p = 0; p < kMaxProj; ++p) {
            const double b = a.ent_beta[(size_t)e * kMaxProj + p];
            acc[2 * p] += b * gr;
            acc[2 * p + 1] += b * gi;
          }
        }
#pragma unroll
        for (int i = 0; i < 2 * kMaxProj; ++i) acc[i] = wave_sum(acc[i]);
        if (lane < kMaxProj) {
          double re = acc[0], im = acc[1];
#pragma unroll
          for (int p = 1; p < kMaxProj; ++p)
            if (lane == p) {
              re = acc[2 * p];
              im = acc[2 * p + 1];
            }
          const double E = a.nl.atom_E[at * kMaxProj + lane] * a.dV;
          eu[at * kMaxProj + lane] = make_double2(E * re, E * im);
        }
      }
      __syncthreads();
    }
    // ---- h u_s and the Horner update, column by column. The LDS offsets are
    // re-materialised per stage so that the compiler does not keep every
    // address of the unrolled column loop live across the stage loop.
    const T tau = (T)(a.dt / s);
    int sxp[4], sxm[4], syp[4], sym[4], scol = col;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      sxp[m] = oxp[m];
      sxm[m] = oxm[m];
      syp[m] = oyp[m];
      sym[m] = oym[m];
      asm volatile("" : "+v"(sxp[m]), "+v"(sxm[m]), "+v"(syp[m]), "+v"(sym[m]));
    }
    asm volatile("" : "+v"(scol));
    if (active) {
#pragma unroll
      for (int z = 0; z < N3; ++z) {
        const T2* pl = u + z * plane;
        const T2 c = pl[scol];
        T dg = diag + a.V[z * plane + scol];
        if (a.efield) dg += ext + ez * ((T)z - (T)(0.5 * (N3 - 1)));
        T hr = dg * c.x, hi = dg * c.y;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          T2 p = pl[sxp[m]], n = pl[sxm[m]];
          if (!PERIODIC) {
            if (!vxp[m]) p.x = p.y = 0;
            if (!vxm[m]) n.x = n.y = 0;
          }
          hr += cx[m] * (p.x + n.x) + bx[m] * (p.y - n.y);
          hi += cx[m] * (p.y + n.y) - bx[m] * (p.x - n.x);
          p = pl[syp[m]];
          n = pl[sym[m]];
          if (!PERIODIC) {
            if (!vyp[m]) p.x = p.y = 0;
            if (!vym[m]) n.x = n.y = 0;
          }
          hr += cy[m] * (p.x + n.x) + by[m] * (p.y - n.y);
          hi += cy[m] * (p.y + n.y) - by[m] * (p.x - n.x);
          const int zp = z + m + 1, zm = z - m - 1;
          T2 q, r;
          q.x = q.y = r.x = r.y = 0;
          if (PERIODIC || zp < N3) q = u[((zp) % N3) * plane + scol];
          if (PERIODIC || zm >= 0) r = u[((zm + N3) % N3) * plane + scol];
          hr += cz[m] * (q.x + r.x) + bz[m] * (q.y - r.y);
          hi += cz[m] * (q.y + r.y) - bz[m] * (q.x - r.x);
        }
        un[z].x = w[z].x + tau * hi;
        un[z].y = w[z].y - tau * hr;
      }
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int z = 0; z < N3; ++z) u[z * plane + col] = un[z];
    }
    __syncthreads();
    // ---- nonlocal part of the stage, scattered over each atom's sphere:
    // u_{s-1}(x_e) += (-i tau) exp(-i kappa.x_e) sum_p beta_p(x_e) E_p u_p.
    // Atoms of one colour have disjoint spheres, colours run in a fixed order.
    if (n_atoms > 0) {
      const double taud = a.dt / s;
      for (int cl = 0; cl < a.n_colors; ++cl) {
        for (int ii = a.color_start[cl] + wave; ii < a.color_start[cl + 1]; ii += nwaves) {
          const int at = a.color_atoms[ii];
          const int e0 = a.nl.atom_start[at], e1 = a.nl.atom_start[at + 1];
          double2 E4[kMaxProj];
#pragma unroll
          for (int p = 0; p < kMaxProj; ++p) E4[p] = eu[at * kMaxProj + p];
          for (int e = e0 + lane; e < e1; e += 64) {
            const int idx = a.nl.ent_idx[e];
            const double2 p1 = phk[e], p2 = a.phA[e];
            const double pr = p1.x * p2.x - p1.y * p2.y, pim = p1.x * p2.y + p1.y * p2.x;
            double sr = 0.0, si = 0.0;
#pragma unroll
            for (int p = 0; p < kMaxProj; ++p) {
              const double b = a.ent_beta[(size_t)e * kMaxProj + p];
              sr += b * E4[p].x;
              si += b * E4[p].y;
            }
            const double cr = pr * sr + pim * si, ci = pr * si - pim * sr;
            T2 v = u[idx];
            v.x += (T)(taud * ci);
            v.y -= (T)(taud * cr);
            u[idx] = v;
          }
        }
        __syncthreads();
      }
    }
  }

  // ---- w_new to HBM
  if (active) {
#pragma unroll
    for (int z = 0; z < N3; ++z) wg[z * plane + col] = u[z * plane + col];
  }

  // ---- observables of w_new (FP64): norm, p_x, p_y, p_z, kin, vloc
  double sv[6] = {0, 0, 0, 0, 0, 0};
  if (active) {
#pragma unroll
    for (int z = 0; z < N3; ++z) {
      const T2* pl = u + z * plane;
      const T2 cv = pl[col];
      const double cr = (double)cv.x, ci = (double)cv.y;
      double lr = a.cdiag * cr, li = a.cdiag * ci;
      double dxr = 0, dxi = 0, dyr = 0, dyi = 0, dzr = 0, dzi = 0;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        T2 p = pl[oxp[m]], n = pl[oxm[m]];
        if (!PERIODIC) {
          if (!vxp[m]) p.x = p.y = 0;
          if (!vxm[m]) n.x = n.y = 0;
        }
        lr += a.lap[0][m + 1] * ((double)p.x + (double)n.x);
        li += a.lap[0][m + 1] * ((double)p.y + (double)n.y);
        dxr += a.dh[0][m] * ((double)p.x - (double)n.x);
        dxi += a.dh[0][m] * ((double)p.y - (double)n.y);
        p = pl[oyp[m]];
        n = pl[oym[m]];
        if (!PERIODIC) {
          if (!vyp[m]) p.x = p.y = 0;
          if (!vym[m]) n.x = n.y = 0;
        }
        lr += a.lap[1][m + 1] * ((double)p.x + (double)n.x);
        li += a.lap[1][m + 1] * ((double)p.y + (double)n.y);
        dyr += a.dh[1][m] * ((double)p.x - (double)n.x);
        dyi += a.dh[1][m] * ((double)p.y - (double)n.y);
        const int zp = z + m + 1, zm = z - m - 1;
        T2 q, r;
        q.x = q.y = r.x = r.y = 0;
        if (PERIODIC || zp < N3) q = u[((zp) % N3) * plane + col];
        if (PERIODIC || zm >= 0) r = u[((zm + N3) % N3) * plane + col];
        lr += a.lap[2][m + 1] * ((double)q.x + (double)r.x);
        li += a.lap[2][m + 1] * ((double)q.y + (double)r.y);
        dzr += a.dh[2][m] * ((double)q.x - (double)r.x);
        dzi += a.dh[2][m] * ((double)q.y - (double)r.y);
      }
      const double nn = cr * cr + ci * ci;
      sv[0] += nn;
      sv[1] += cr * dxi - ci * dxr;
      sv[2] += cr * dyi - ci * dyr;
      sv[3] += cr * dzi - ci * dzr;
      sv[4] += cr * lr + ci * li;
      sv[5] += a.Vloc[z * plane + col] * nn;
    }
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) sv[i] = wave_sum(sv[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < 6; ++i) red[wave * 8 + i] = sv[i];
  }
  __syncthreads();
  if (tid < 6) {
    double acc = 0;
    for (int wv = 0; wv < nwaves; ++wv) acc += red[wv * 8 + tid];
    a.obs[(size_t)o * 8 + tid] = acc;
  }
  __syncthreads();

  // ---- nonlocal current and energy at t_{n+1}: moments (1, x, y, z) of the
  // projections with the phase of A_{n+1}; one wavefront per atom
  double jl[4] = {0, 0, 0, 0};  // lane 0 of each wave: J_x, J_y, J_z, E_NL
  if (n_atoms > 0) {
    for (int at = wave; at < n_atoms; at += nwaves) {
      const int e0 = a.nl.atom_start[at], e1 = a.nl.atom_start[at + 1];
      double acc[kMaxProj][4][2];
#pragma unroll
      for (int p = 0; p < kMaxProj; ++p)
#pragma unroll
        for (int m = 0; m < 4; ++m) acc[p][m][0] = acc[p][m][1] = 0.0;
      for (int e = e0 + lane; e < e1; e += 64) {
        const T2 v = u[a.nl.ent_idx[e]];
        const double2 p1 = phk[e], p2 = a.phAJ[e];
        const double pr = p1.x * p2.x - p1.y * p2.y, pim = p1.x * p2.y + p1.y * p2.x;
        const double gr = pr * (double)v.x - pim * (double)v.y;
        const double gi = pr * (double)v.y + pim * (double)v.x;
        const double mom[4] = {1.0, a.ent_x[3 * (size_t)e], a.ent_x[3 * (size_t)e + 1],
                               a.ent_x[3 * (size_t)e + 2]};
#pragma unroll
        for (int p = 0; p < kMaxProj; ++p) {
          const double b = a.ent_beta[(size_t)e * kMaxProj + p];
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            acc[p][m][0] += b * mom[m] * gr;
            acc[p][m][1] += b * mom[m] * gi;
          }
        }
      }
#pragma unroll
      for (int p = 0; p < kMaxProj; ++p) {
        double ur = wave_sum(acc[p][0][0]) * a.dV, ui = wave_sum(acc[p][0][1]) * a.dV;
        const double E = a.nl.atom_E[at * kMaxProj + p];
        jl[3] += E * (ur * ur + ui * ui);
#pragma unroll
        for (int m = 1; m < 4; ++m) {
          const double vr = wave_sum(acc[p][m][0]) * a.dV, vi = wave_sum(acc[p][m][1]) * a.dV;
          jl[m - 1] += 2.0 * E * (vr * ui - vi * ur);
        }
      }
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) red[wave * 8 + i] = jl[i];
  }
  __syncthreads();
  if (tid < 4) {
    double acc = 0;
    for (int wv = 0; wv < nwaves; ++wv) acc += red[wv * 8 + tid];
    a.jnl[(size_t)o * 4 + tid] = acc;
  }
}

size_t fused_lds_bytes(const Geometry& g, int n_atoms, size_t elem) {
  const size_t N = (size_t)g.n1 * g.n2 * g.n3;
  return ((N * elem + 15) & ~(size_t)15) + (size_t)n_atoms * kMaxProj * sizeof(double2) + 16 * 8 * sizeof(double);
}

bool fused_supported(const Geometry& g, int n_atoms, size_t elem) {
  const int n3 = g.n3;
  if (n3 != 12 && n3 != 16 && n3 != 20) return false;
  if (g.n1 * g.n2 > 512) return false;
  return fused_lds_bytes(g, n_atoms, elem) <= 160 * 1024;
}

template <typename T, int N3, int MAXT>
static void launch_n3(bool periodic, const FusedArgs<T>& a, size_t lds, hipStream_t s) {
  const int threads = ((a.g.n1 * a.g.n2 + 63) / 64) * 64;
  const dim3 grid((unsigned)((size_t)a.g.n_orb * a.g.n_k));
  if (periodic)
    hipLaunchKernelGGL((k_fused<T, N3, true, MAXT>), grid, dim3(threads), lds, s, a);
  else
    hipLaunchKernelGGL((k_fused<T, N3, false, MAXT>), grid, dim3(threads), lds, s, a);
}

template <typename T>
hipError_t launch_fused(const FusedArgs<T>& a, hipStream_t s) {
  using T2 = typename Vec2<T>::type;
  if (!fused_supported(a.g, a.nl.n_atoms, sizeof(T2))) return hipErrorInvalidValue;
  const size_t lds = fused_lds_bytes(a.g, a.nl.n_atoms, sizeof(T2));
  const bool per = a.g.periodic != 0;
  switch (a.g.n3) {
    case 12: launch_n3<T, 12, 512>(per, a, lds, s); break;
    case 16: launch_n3<T, 16, 512>(per, a, lds, s); break;
    default: launch_n3<T, 20, 512>(per, a, lds, s); break;
  }
  return hipGetLastError();
}

template hipError_t launch_fused<double>(const FusedArgs<double>&, hipStream_t);
template hipError_t launch_fused<float>(const FusedArgs<float>&, hipStream_t);

}  // namespace td
