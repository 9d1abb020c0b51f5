// Whole time step of one orbital with the orbital resident in LDS.
//
// For cubic cells whose orbital fits in LDS (n = 12, 16, 20 or 24 per axis,
// N * sizeof(complex) + tables <= 160 KB), one workgroup owns one orbital and
// runs all four Horner stages u_{s-1} = w + (-i dt / s) h u_s, s = 4..1
// (Program Summary: fourth-order truncated Taylor expansion; Sec. 4.1,
// Eq. TDKS_solid for h), with
//   * u_s in LDS; w and u_{s-1} in registers. A thread owns one (x, y)
//     column, or one half of it (ZS = 2: the two halves sit in different
//     wavefronts, which halves the register arrays and doubles the waves);
//   * the Kleinman-Bylander projections u_p = <beta_p^kappa|u_s> of every atom
//     formed in the workgroup before each stage (one wavefront per atom,
//     fixed-order shuffle reductions, FP64) and added back by a scatter over
//     each atom's sphere into the LDS copy (atoms coloured so that spheres of
//     one colour are disjoint: no atomics, a fixed summation order);
//   * after the last stage: w_new written once, then the observables of
//     w_new that the current needs (norm and momentum, FP64 accumulation) and
//     the moment projections for the nonlocal current at t_{n+1}.
// HBM traffic per orbital point and step: read w once, write w_new once.
#include "internal.h"

namespace td {

// Global-memory views of the argument pointers. The persistent kernel reads
// its arguments from a device array, and a pointer loaded from memory is a
// generic (flat) pointer to the compiler; flat accesses also count on the LDS
// counter, so every LDS wait would wait for them. Accesses through these
// views are plain global (or scalar) loads and stores.
// (The host pass of this single-source file also parses the device templates;
// the address space exists only in the device pass.)
#if defined(__HIP_DEVICE_COMPILE__)
template <class X>
using gp = __attribute__((address_space(1))) X*;
#else
template <class X>
using gp = X*;
#endif
template <class X>
__device__ __forceinline__ gp<X> G(X* p) {
  return (gp<X>)p;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Wavefront sums of 16 values by recursive halving over lane bits 5..2 (8 +
// 4 + 2 + 1 shuffles, then two over bits 1 and 0): every lane returns the full
// sum of value lane >> 2.
__device__ __forceinline__ double wave_sum16(const double (&v)[16], int lane) {
  double a[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const bool hi = lane & 32;
    const double send = hi ? v[i] : v[i + 8], keep = hi ? v[i + 8] : v[i];
    a[i] = keep + __shfl_xor(send, 32, 64);
  }
#pragma unroll
  for (int w = 4, bit = 16; w >= 1; w >>= 1, bit >>= 1) {
#pragma unroll
    for (int i = 0; i < w; ++i) {
      const bool hi = lane & bit;
      const double send = hi ? a[i] : a[i + w], keep = hi ? a[i + w] : a[i];
      a[i] = keep + __shfl_xor(send, bit, 64);
    }
  }
  a[0] += __shfl_xor(a[0], 2, 64);
  return a[0] + __shfl_xor(a[0], 1, 64);
}

// Wavefront sums of eight values at once by recursive halving: at each of the
// exchanges over lane bits 5, 4, 3 a lane keeps half of its values and sends
// the other half, so 4 + 2 + 1 shuffles leave value j = (lane >> 3) & 7
// summed over those bits; three more finish the sum over bits 2..0. Every lane
// returns the full sum of value (lane >> 3) & 7 (11 shuffles instead of 48).
__device__ __forceinline__ double wave_sum8(const double (&v)[8], int lane) {
  double a[4];
  const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double send = b5 ? v[i] : v[i + 4], keep = b5 ? v[i + 4] : v[i];
    a[i] = keep + __shfl_xor(send, 32, 64);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double send = b4 ? a[i] : a[i + 2], keep = b4 ? a[i + 2] : a[i];
    a[i] = keep + __shfl_xor(send, 16, 64);
  }
  {
    const double send = b3 ? a[0] : a[1], keep = b3 ? a[1] : a[0];
    a[0] = keep + __shfl_xor(send, 8, 64);
  }
  a[0] += __shfl_xor(a[0], 4, 64);
  a[0] += __shfl_xor(a[0], 2, 64);
  a[0] += __shfl_xor(a[0], 1, 64);
  return a[0];
}

// in-plane neighbour offsets of one column (periodic wrap) and its own offset
struct Nbr {
  int xp[4], xm[4], yp[4], ym[4];
  int c;
};

struct FusedCoefIn {
  double dh[3][4];
  double cdiag;
};

template <typename T>
struct Coef {
  T cx[4], cy[4], cz[4], bx[4], by[4], bz[4];
  T diag, ext, ez;
};

// A copy of the offsets that the compiler cannot see through: rebuilding the
// addresses per stage keeps the unrolled column loop from holding every one
// of them live across the stage loop.
__device__ __forceinline__ float opaque_t(float v) {
  asm volatile("" : "+v"(v));
  return v;
}
__device__ __forceinline__ double opaque_t(double v) {
  asm volatile("" : "+v"(v));
  return v;
}

__device__ __forceinline__ Nbr opaque(const Nbr& n) {
  Nbr r = n;
#pragma unroll
  for (int m = 0; m < 4; ++m) asm volatile("" : "+v"(r.xp[m]), "+v"(r.xm[m]), "+v"(r.yp[m]), "+v"(r.ym[m]));
  asm volatile("" : "+v"(r.c));
  return r;
}

template <typename T, bool PERIODIC>
__device__ __forceinline__ typename Vec2<T>::type lds_xy(const typename Vec2<T>::type* pl, int off, bool valid) {
  typename Vec2<T>::type v = pl[off];
  if (!PERIODIC && !valid) v.x = v.y = 0;
  return v;
}

// h u_s (local part) and the Horner update for the planes Z0 .. Z0 + ZN - 1
template <typename T, int N, int ZN, int Z0, bool PERIODIC>
__device__ __forceinline__ void stencil_part(const typename Vec2<T>::type* u, gp<const T> V,
                                             const Coef<T>& cf, const Nbr& nb, const bool (&ok)[16],
                                             gp<const typename Vec2<T>::type> wg,
                                             typename Vec2<T>::type (&un)[ZN], T tau, bool length) {
  using T2 = typename Vec2<T>::type;
  constexpr int plane = N * N;
  const T ez = opaque_t(cf.ez);
#pragma unroll
  for (int zz = 0; zz < ZN; ++zz) {
    const int z = Z0 + zz;
    const T2* pl = u + z * plane;
    const T2 c = pl[nb.c];
    T dg = cf.diag + V[z * plane + nb.c];
    if (!PERIODIC && length) dg += cf.ext + ez * (T)z;
    T hr = dg * c.x, hi = dg * c.y;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      T2 p = lds_xy<T, PERIODIC>(pl, nb.xp[m], ok[m]);
      T2 n = lds_xy<T, PERIODIC>(pl, nb.xm[m], ok[4 + m]);
      hr += cf.cx[m] * (p.x + n.x) + cf.bx[m] * (p.y - n.y);
      hi += cf.cx[m] * (p.y + n.y) - cf.bx[m] * (p.x - n.x);
      p = lds_xy<T, PERIODIC>(pl, nb.yp[m], ok[8 + m]);
      n = lds_xy<T, PERIODIC>(pl, nb.ym[m], ok[12 + m]);
      hr += cf.cy[m] * (p.x + n.x) + cf.by[m] * (p.y - n.y);
      hi += cf.cy[m] * (p.y + n.y) - cf.by[m] * (p.x - n.x);
      const int zp = z + m + 1, zm = z - m - 1;
      T2 q, r;
      q.x = q.y = r.x = r.y = 0;
      if (PERIODIC || zp < N) q = u[(zp % N) * plane + nb.c];
      if (PERIODIC || zm >= 0) r = u[((zm + N) % N) * plane + nb.c];
      hr += cf.cz[m] * (q.x + r.x) + cf.bz[m] * (q.y - r.y);
      hi += cf.cz[m] * (q.y + r.y) - cf.bz[m] * (q.x - r.x);
    }
    // w is re-read (from cache) rather than held in registers for all stages
    const T2 wv = wg[z * plane + nb.c];
    un[zz].x = wv.x + tau * hi;
    un[zz].y = wv.y - tau * hr;
    // one plane at a time: bounds the loads in flight and so the registers
    __builtin_amdgcn_sched_barrier(0);
  }
}

// norm and momentum sums of w_new for the planes Z0 .. Z0 + ZN - 1: the
// weighted neighbour sums in the stage precision, their products with w and
// the running sums in FP64 (as in the streaming observables kernel)
template <typename T, int N, int ZN, int Z0, bool PERIODIC>
__device__ __forceinline__ void observe_part(const typename Vec2<T>::type* u, const T (&dw)[3][4],
                                             const Nbr& nb, const bool (&ok)[16], double (&sv)[4]) {
  // Summed over the whole grid, Im(conj(w) D w) with the antisymmetric
  // difference D = sum_m d_m (S_m - S_-m) equals 2 sum_m d_m Im(conj(w) S_m w)
  // (shift r -> r - m in the backward half; zero outside an isolated box), so
  // each point needs only its forward neighbours.
  using T2 = typename Vec2<T>::type;
  constexpr int plane = N * N;
#pragma unroll
  for (int zz = 0; zz < ZN; ++zz) {
    const int z = Z0 + zz;
    const T2* pl = u + z * plane;
    const T2 cv = pl[nb.c];
    const double cr = (double)cv.x, ci = (double)cv.y;
    T sxr = 0, sxi = 0, syr = 0, syi = 0, szr = 0, szi = 0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const T2 p = lds_xy<T, PERIODIC>(pl, nb.xp[m], ok[m]);
      const T2 q = lds_xy<T, PERIODIC>(pl, nb.yp[m], ok[8 + m]);
      const int zp = z + m + 1;
      T2 r;
      r.x = r.y = 0;
      if (PERIODIC || zp < N) r = u[(zp % N) * plane + nb.c];
      sxr += dw[0][m] * p.x;
      sxi += dw[0][m] * p.y;
      syr += dw[1][m] * q.x;
      syi += dw[1][m] * q.y;
      szr += dw[2][m] * r.x;
      szi += dw[2][m] * r.y;
    }
    sv[0] += cr * cr + ci * ci;
    sv[1] += 2.0 * (cr * (double)sxi - ci * (double)sxr);
    sv[2] += 2.0 * (cr * (double)syi - ci * (double)syr);
    sv[3] += 2.0 * (cr * (double)szi - ci * (double)szr);
  }
}

// ITEMS: the body runs once per item of a loop (the persistent form)
template <typename T, int N, int ZS, bool PERIODIC, bool ITEMS = false>
__device__ __forceinline__ void fused_body(const FusedArgs<T>& a, const int o, unsigned char* smem_raw) {
  using T2 = typename Vec2<T>::type;
  constexpr int plane = N * N;
  constexpr int NP = plane * N;
  constexpr int ZN = N / ZS;                      // planes per thread
  constexpr int HALF = ((plane + 63) / 64) * 64;  // threads per column half (whole waves)
  const int n_atoms = a.nl.n_atoms;
  const int S = a.nl.n_ent;
  const gp<const int> atom_start = G(a.nl.atom_start);
  const gp<const int> ent_idx = G(a.nl.ent_idx);
  const gp<const double> atom_E = G(a.nl.atom_E);
  const gp<const double> ent_beta = G(a.ent_beta);
  const gp<const double> ent_x = G(a.ent_x);
  const gp<const int> color_start = G(a.color_start);
  const gp<const int> color_atoms = G(a.color_atoms);
  const gp<const double2> phAJ = G(a.phAJ);
  T2* u = reinterpret_cast<T2*>(smem_raw);
  constexpr size_t ubytes = ((size_t)NP * sizeof(T2) + 15) & ~(size_t)15;
  double2* eu = reinterpret_cast<double2*>(smem_raw + ubytes);               // [n_atoms][4]
  double* red = reinterpret_cast<double*>(eu + (size_t)n_atoms * kMaxProj);  // [16][8]
  double* ja = red + 16 * 8;                                                 // [n_atoms][4]

  const int k = o / a.g.n_orb;
  // in the persistent form the thread index is opaque to the compiler, so
  // that the values derived from it are formed per item instead of being
  // hoisted out of the item loop and held in registers across it
  int tid = threadIdx.x;
  if (ITEMS) asm volatile("" : "+v"(tid));
  const int lane = tid & 63, wave = tid >> 6, nwaves = blockDim.x >> 6;
  const int half = (ZS == 2 && tid >= HALF) ? 1 : 0;  // uniform per wavefront
  const int ctid = tid - half * HALF;
  const int tx = ctid % N, ty = ctid / N;
  const bool active = ctid < plane;

  Nbr nb;
  bool ok[16];
#pragma unroll
  for (int m = 1; m <= 4; ++m) {
    const int xp = tx + m, xm = tx - m, yp = ty + m, ym = ty - m;
    ok[m - 1] = PERIODIC || xp < N;
    ok[4 + m - 1] = PERIODIC || xm >= 0;
    ok[8 + m - 1] = PERIODIC || yp < N;
    ok[12 + m - 1] = PERIODIC || ym >= 0;
    nb.xp[m - 1] = ty * N + (xp % N);
    nb.xm[m - 1] = ty * N + ((xm + N) % N);
    nb.yp[m - 1] = (yp % N) * N + tx;
    nb.ym[m - 1] = ((ym + N) % N) * N + tx;
  }
  nb.c = active ? ctid : 0;

  const gp<T2> wg = G(a.w) + (size_t)o * NP;
  T2 un[ZN];
  const int z0 = half * ZN;
#pragma unroll
  for (int zz = 0; zz < ZN; ++zz) {
    T2 v;
    v.x = v.y = 0;
    if (active) v = wg[(z0 + zz) * plane + nb.c];
    if (active) u[(z0 + zz) * plane + nb.c] = v;
  }

  Coef<T> cf;
  {
    // wave-uniform: the k-point table is read with scalar loads
    const gp<const T> ck = G(a.coef) + (size_t)k * kCoef;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      cf.cx[m] = a.lapc[0][m];
      cf.cy[m] = a.lapc[1][m];
      cf.cz[m] = a.lapc[2][m];
      cf.bx[m] = ck[m];
      cf.by[m] = ck[4 + m];
      cf.bz[m] = ck[8 + m];
    }
    cf.diag = ck[12];
    cf.ext = cf.ez = 0;
    if (!PERIODIC && a.efield) {
      // E . r with r from the box centre; the z part is added per plane
      const gp<const double> ef = G(a.efield);
      cf.ext = (T)(ef[0] * (tx - 0.5 * (N - 1)) * a.g.h1 + ef[1] * (ty - 0.5 * (N - 1)) * a.g.h2 -
                   ef[2] * a.g.h3 * 0.5 * (N - 1));
      cf.ez = (T)(ef[2] * a.g.h3);
    }
  }
  const bool length = !PERIODIC && a.efield != nullptr;
  const gp<const double2> phk = G(a.nl.phk) + (size_t)k * S;
  const gp<const double2> phkA = G(a.phkA) + (size_t)k * S;  // exp(i kappa . x_e) of this step
  __syncthreads();

  // ---- projections of u_s: one wavefront per atom, FP64
  auto project = [&]() {
    for (int at = wave; at < n_atoms; at += nwaves) {
      const int e0 = atom_start[at], e1 = atom_start[at + 1];
      double acc[2 * kMaxProj] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (int e = e0 + lane; e < e1; e += 64) {
        const T2 v = u[ent_idx[e]];
        const double2 ph = phkA[e];
        const double pr = ph.x, pim = ph.y;
        const double gr = pr * (double)v.x - pim * (double)v.y;
        const double gi = pr * (double)v.y + pim * (double)v.x;
#pragma unroll
        for (int p = 0; p < kMaxProj; ++p) {
          const double b = ent_beta[(size_t)e * kMaxProj + p];
          acc[2 * p] += b * gr;
          acc[2 * p + 1] += b * gi;
        }
      }
      // value 2p (real) sits in lanes 16p.., value 2p + 1 (imaginary) 8 lanes up
      const double tot = wave_sum8(acc, lane);
      const double im = __shfl_down(tot, 8, 64);
      if ((lane & 15) == 0) {
        const int p = lane >> 4;
        const double E = atom_E[at * kMaxProj + p] * a.dV;
        eu[at * kMaxProj + p] = make_double2(E * tot, E * im);
      }
    }
    __syncthreads();
  };
  // With disjoint spheres (one colour) every sphere point belongs to one
  // atom, so the wavefront that adds an atom's nonlocal term of stage s to
  // its points can go on to form that atom's projections of the completed
  // u_{s-1} without waiting for the other atoms: one barrier fewer per stage.
  const bool one_colour = a.n_colors == 1;
  if (n_atoms > 0) project();

#pragma unroll 1
  for (int s = 4; s >= 1; --s) {
    // ---- local part of h u_s and the Horner update
    const T tau = (T)(a.dt / s);
    {
      const Nbr sb = opaque(nb);
      if (active) {
        if (ZS == 1 || half == 0)
          stencil_part<T, N, ZN, 0, PERIODIC>(u, G(a.V), cf, sb, ok, wg, un, tau, length);
        else
          stencil_part<T, N, ZN, (ZS == 2 ? ZN : 0), PERIODIC>(u, G(a.V), cf, sb, ok, wg, un, tau, length);
      }
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int zz = 0; zz < ZN; ++zz) u[(z0 + zz) * plane + nb.c] = un[zz];
    }
    __syncthreads();
    // ---- nonlocal part of the stage, scattered over each atom's sphere:
    // u_{s-1}(x_e) += (-i tau) exp(-i kappa.x_e) sum_p beta_p(x_e) E_p u_p.
    // Atoms of one colour have disjoint spheres, colours run in a fixed order.
    if (n_atoms > 0) {
      const double taud = a.dt / s;
      if (one_colour) {
        for (int at = wave; at < n_atoms; at += nwaves) {
          const int e0 = atom_start[at], e1 = atom_start[at + 1];
          {
            double2 E4[kMaxProj];
#pragma unroll
            for (int p = 0; p < kMaxProj; ++p) E4[p] = eu[at * kMaxProj + p];
            for (int e = e0 + lane; e < e1; e += 64) {
              const int idx = ent_idx[e];
              const double2 ph = phkA[e];
              const double pr = ph.x, pim = ph.y;
              double sr = 0.0, si = 0.0;
#pragma unroll
              for (int p = 0; p < kMaxProj; ++p) {
                const double b = ent_beta[(size_t)e * kMaxProj + p];
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
          // the same lanes read back the same points: no barrier needed
          if (s > 1) {
            double acc[2 * kMaxProj] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (int e = e0 + lane; e < e1; e += 64) {
              const T2 v = u[ent_idx[e]];
              const double2 ph = phkA[e];
              const double pr = ph.x, pim = ph.y;
              const double gr = pr * (double)v.x - pim * (double)v.y;
              const double gi = pr * (double)v.y + pim * (double)v.x;
#pragma unroll
              for (int p = 0; p < kMaxProj; ++p) {
                const double b = ent_beta[(size_t)e * kMaxProj + p];
                acc[2 * p] += b * gr;
                acc[2 * p + 1] += b * gi;
              }
            }
            const double tot = wave_sum8(acc, lane);
            const double im = __shfl_down(tot, 8, 64);
            if ((lane & 15) == 0) {
              const int p = lane >> 4;
              const double E = atom_E[at * kMaxProj + p] * a.dV;
              eu[at * kMaxProj + p] = make_double2(E * tot, E * im);
            }
          }
        }
        __syncthreads();
      } else {
        for (int cl = 0; cl < a.n_colors; ++cl) {
          for (int ii = color_start[cl] + wave; ii < color_start[cl + 1]; ii += nwaves) {
            const int at = color_atoms[ii];
            const int e0 = atom_start[at], e1 = atom_start[at + 1];
            double2 E4[kMaxProj];
#pragma unroll
            for (int p = 0; p < kMaxProj; ++p) E4[p] = eu[at * kMaxProj + p];
            for (int e = e0 + lane; e < e1; e += 64) {
              const int idx = ent_idx[e];
              const double2 ph = phkA[e];
              const double pr = ph.x, pim = ph.y;
              double sr = 0.0, si = 0.0;
#pragma unroll
              for (int p = 0; p < kMaxProj; ++p) {
                const double b = ent_beta[(size_t)e * kMaxProj + p];
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
        if (s > 1) project();
      }
    }
  }

  // ---- w_new to HBM, observables for the current
  double sv[4] = {0, 0, 0, 0};
  {
    const Nbr fb = opaque(nb);
    if (active) {
#pragma unroll
      for (int zz = 0; zz < ZN; ++zz) wg[(z0 + zz) * plane + fb.c] = u[(z0 + zz) * plane + fb.c];
      // whole columns, by the threads of the first column half: the summation
      // order is the same for either column split
      if (half == 0) observe_part<T, N, N, 0, PERIODIC>(u, a.dhc, fb, ok, sv);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) sv[i] = wave_sum(sv[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) red[wave * 8 + i] = sv[i];
  }
  __syncthreads();
  if (tid < 6) {
    double acc = 0;
    if (tid < 4)
      for (int wv = 0; wv < nwaves; ++wv) acc += red[wv * 8 + tid];
    G(a.obs)[(size_t)o * 8 + tid] = acc;  // slots 4, 5 (kinetic, local) stay 0 here
  }
  __syncthreads();

  // ---- nonlocal current and energy at t_{n+1}: moments (1, x, y, z) of the
  // projections with the phase of A_{n+1}; one wavefront per atom, two
  // moments per gather of the sphere values
  if (n_atoms > 0) {
    for (int at = wave; at < n_atoms; at += nwaves) {
      const int e0 = atom_start[at], e1 = atom_start[at + 1];
      // lane 32 mm + 8 p holds the real part of the pass's moment mm of
      // projector p and receives the imaginary part from 4 lanes up
      const int pl = (lane >> 3) & 3, mml = lane >> 5;
      const double E = atom_E[at * kMaxProj + pl];
      double ur = 0.0, ui = 0.0;
#pragma unroll 1
      for (int pass = 0; pass < 2; ++pass) {
        // value 8 mm + 2 p + (0 real, 1 imaginary) for moments m = 2 pass + mm
        double acc[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] = 0.0;
        for (int e = e0 + lane; e < e1; e += 64) {
          const T2 v = u[ent_idx[e]];
          const double2 p1 = phk[e], p2 = phAJ[e];
          const double pr = p1.x * p2.x - p1.y * p2.y, pim = p1.x * p2.y + p1.y * p2.x;
          const double gr = pr * (double)v.x - pim * (double)v.y;
          const double gi = pr * (double)v.y + pim * (double)v.x;
          const double m0 = pass == 0 ? 1.0 : ent_x[3 * (size_t)e + 1];
          const double m1 = ent_x[3 * (size_t)e + 2 * pass];
#pragma unroll
          for (int p = 0; p < kMaxProj; ++p) {
            const double b = ent_beta[(size_t)e * kMaxProj + p];
            const double br = b * gr, bi = b * gi;
            acc[2 * p] += m0 * br;
            acc[2 * p + 1] += m0 * bi;
            acc[8 + 2 * p] += m1 * br;
            acc[8 + 2 * p + 1] += m1 * bi;
          }
        }
        const double tot = wave_sum16(acc, lane) * a.dV;
        const double im = __shfl_down(tot, 4, 64);
        if (pass == 0) {
          ur = __shfl(tot, 8 * pl, 64);
          ui = __shfl(im, 8 * pl, 64);
        }
        // E_p |u_p|^2 for m = 0, 2 E_p Im(conj(v_p) u_p) for m = 1..3, summed over p
        const int m = 2 * pass + mml;
        double c = (m == 0) ? E * (ur * ur + ui * ui) : 2.0 * E * (tot * ui - im * ur);
        c += __shfl_xor(c, 8, 64);
        c += __shfl_xor(c, 16, 64);
        if ((lane & 31) == 0) ja[at * 4 + (m == 0 ? 3 : m - 1)] = c;
      }
    }
  }
  __syncthreads();
  if (tid < 4) {  // atoms summed in index order, whatever wavefront formed them
    double acc = 0;
    for (int at = 0; at < n_atoms; ++at) acc += ja[at * 4 + tid];
    G(a.jnl)[(size_t)o * 4 + tid] = acc;
  }
}

// one orbital per workgroup
template <typename T, int N, int ZS, bool PERIODIC, int MAXT>
__global__ __launch_bounds__(MAXT) void k_fused(FusedArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  fused_body<T, N, ZS, PERIODIC>(a, blockIdx.x, smem_raw);
}

// Persistent form for batches of cells with the same grid: a fixed grid of
// workgroups pulls (cell, orbital) items from a device queue in the given
// (largest-cell-first) order until the list is exhausted; every item is
// computed exactly as in k_fused, so the result does not depend on which
// workgroup takes it.
template <typename T, int N, int ZS, bool PERIODIC, int MAXT>
__global__ __launch_bounds__(MAXT, (MAXT <= 512 && sizeof(T) == 4) ? 4 : 1) void k_fused_persistent(const FusedArgs<T>* __restrict__ cells,
                                                           const int2* __restrict__ items, int n_items,
                                                           int* queue) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int next;
  if (threadIdx.x == 0) next = atomicAdd(queue, 1);
  __syncthreads();
  int it = __builtin_amdgcn_readfirstlane(next);
  __syncthreads();
  while (it < n_items) {
    // claim the following item now, so that the queue's round trip overlaps
    // this item's work (every item is still taken exactly once)
    int claim = 0;
    if (threadIdx.x == 0) claim = atomicAdd(queue, 1);
    // the cell and orbital are uniform: scalar registers, so that the
    // cell's arguments are read with scalar loads as kernel arguments are
    const int2 ci = items[it];
    const int cx = __builtin_amdgcn_readfirstlane(ci.x), orb = __builtin_amdgcn_readfirstlane(ci.y);
    fused_body<T, N, ZS, PERIODIC, true>(cells[cx], orb, smem_raw);
    __syncthreads();
    if (threadIdx.x == 0) next = claim;
    __syncthreads();
    it = __builtin_amdgcn_readfirstlane(next);
    __syncthreads();
  }
}

// per k-point coefficients of the step in the stage precision (from kappa at
// the step midpoint): kappa_mu d_m / h_mu and the diagonal
// -1/2 sum_mu c_0 / h_mu^2 + |kappa|^2 / 2
template <typename T>
__device__ __forceinline__ void fused_coef_k(const double* __restrict__ kappa, const double (&dh)[3][4], double cdiag,
                                             T* __restrict__ coef, int k) {
  const double kx = kappa[3 * k], ky = kappa[3 * k + 1], kz = kappa[3 * k + 2];
  T* c = coef + (size_t)k * kCoef;
  for (int m = 0; m < 4; ++m) {
    c[m] = (T)(kx * dh[0][m]);
    c[4 + m] = (T)(ky * dh[1][m]);
    c[8 + m] = (T)(kz * dh[2][m]);
  }
  c[12] = (T)(cdiag + 0.5 * (kx * kx + ky * ky + kz * kz));
  c[13] = c[14] = c[15] = (T)0;
}

template <typename T>
__global__ void k_fused_coef(const double* __restrict__ kappa, int n_k, FusedCoefIn in, T* __restrict__ coef) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_k) return;
  fused_coef_k<T>(kappa, in.dh, in.cdiag, coef, k);
}

// exp(i kappa . x_e) = exp(i k . x_e) exp(i A . x_e / c) for every k-point and
// sphere entry, once per step (each workgroup then reads one factor per entry)
__device__ __forceinline__ void fused_phase_t(const double2* __restrict__ phk, const double2* __restrict__ phA, int S,
                                              double2* __restrict__ out, size_t t) {
  const int e = (int)(t % S);
  const double2 p1 = phk[t], p2 = phA[e];
  out[t] = make_double2(p1.x * p2.x - p1.y * p2.y, p1.x * p2.y + p1.y * p2.x);
}

__global__ void k_fused_phase(const double2* __restrict__ phk, const double2* __restrict__ phA, int S, int n_k,
                              double2* __restrict__ out) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)n_k * S) return;
  fused_phase_t(phk, phA, S, out, t);
}

// the same two for the cells of a group (cell blockIdx.y)
template <typename T>
__global__ void k_fused_coef_group(const ParamCell* __restrict__ tab) {
  const ParamCell& c = tab[blockIdx.y];
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= c.n_k) return;
  fused_coef_k<T>(c.kappa, c.dh, c.cdiag, static_cast<T*>(c.coef), k);
}

__global__ void k_fused_phase_group(const ParamCell* __restrict__ tab) {
  const ParamCell& c = tab[blockIdx.y];
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c.S == 0 || t >= (size_t)c.n_k * c.S) return;
  fused_phase_t(c.phk, c.phA, c.S, c.phkA, t);
}

template <typename T>
hipError_t launch_fused_coef_group(const ParamCell* tab, int ncells, int max_nk, long max_phases, hipStream_t s) {
  hipLaunchKernelGGL((k_fused_coef_group<T>), dim3((unsigned)((max_nk + 63) / 64), ncells), dim3(64), 0, s, tab);
  if (max_phases > 0)
    hipLaunchKernelGGL(k_fused_phase_group, dim3((unsigned)((max_phases + 255) / 256), ncells), dim3(256), 0, s,
                       tab);
  return hipGetLastError();
}
template hipError_t launch_fused_coef_group<double>(const ParamCell*, int, int, long, hipStream_t);
template hipError_t launch_fused_coef_group<float>(const ParamCell*, int, int, long, hipStream_t);

template <typename T>
hipError_t launch_fused_coef(const FusedArgs<T>& a, hipStream_t s) {
  FusedCoefIn in;
  for (int i = 0; i < 3; ++i)
    for (int m = 0; m < 4; ++m) in.dh[i][m] = a.dh[i][m];
  in.cdiag = a.cdiag;
  const int nk = a.g.n_k;
  hipLaunchKernelGGL((k_fused_coef<T>), dim3((unsigned)((nk + 63) / 64)), dim3(64), 0, s, a.kappa, nk, in, a.coef);
  const size_t tot = (size_t)nk * a.nl.n_ent;
  if (tot > 0)
    hipLaunchKernelGGL(k_fused_phase, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, a.nl.phk, a.phA,
                       a.nl.n_ent, nk, a.phkA);
  return hipGetLastError();
}

template hipError_t launch_fused_coef<double>(const FusedArgs<double>&, hipStream_t);
template hipError_t launch_fused_coef<float>(const FusedArgs<float>&, hipStream_t);

// the per-k coefficient table alone (the per-stage kernels read it too)
template <typename T>
hipError_t launch_coef_table(const double* kappa, int n_k, const double dh[3][4], double cdiag, T* coef,
                             hipStream_t s) {
  FusedCoefIn in;
  for (int i = 0; i < 3; ++i)
    for (int m = 0; m < 4; ++m) in.dh[i][m] = dh[i][m];
  in.cdiag = cdiag;
  hipLaunchKernelGGL((k_fused_coef<T>), dim3((unsigned)((n_k + 63) / 64)), dim3(64), 0, s, kappa, n_k, in, coef);
  return hipGetLastError();
}
template hipError_t launch_coef_table<double>(const double*, int, const double[3][4], double, double*, hipStream_t);
template hipError_t launch_coef_table<float>(const double*, int, const double[3][4], double, float*, hipStream_t);

size_t fused_lds_bytes(const Geometry& g, int n_atoms, size_t elem) {
  const size_t N = (size_t)g.n1 * g.n2 * g.n3;
  return ((N * elem + 15) & ~(size_t)15) + (size_t)n_atoms * kMaxProj * sizeof(double2) + 16 * 8 * sizeof(double) +
         (size_t)n_atoms * 4 * sizeof(double);
}

bool fused_supported(const Geometry& g, int n_atoms, size_t elem) {
  const int n = g.n3;
  if (n != 12 && n != 16 && n != 20 && n != 24) return false;
  if (g.n1 != n || g.n2 != n) return false;
  return fused_lds_bytes(g, n_atoms, elem) <= 160 * 1024;
}

// Workgroup size: the column threads, rounded up to eight wavefronts so that
// the nonlocal phases (one wavefront per atom) run the eight atoms of a
// diamond cell side by side; the extra wavefronts idle through the stencil.
// Results do not depend on the count (inactive threads add exact zeros).
template <int N, int ZS>
constexpr int fused_threads() {
  return ZS * (((N * N + 63) / 64) * 64) < 512 ? 512 : ZS * (((N * N + 63) / 64) * 64);
}

// launch bound: 512, or the exact count above it (24^3: 576 threads, one
// workgroup per CU by LDS, so up to 168 registers per lane)
template <int N, int ZS>
constexpr int fused_bound() {
  return fused_threads<N, ZS>() <= 512 ? 512 : fused_threads<N, ZS>();
}

template <typename T, int N, int ZS>
static void launch_n(bool periodic, const FusedArgs<T>& a, size_t lds, hipStream_t s) {
  constexpr int threads = fused_threads<N, ZS>();
  constexpr int bound = fused_bound<N, ZS>();
  const dim3 grid((unsigned)((size_t)a.g.n_orb * a.g.n_k));
  if (periodic)
    hipLaunchKernelGGL((k_fused<T, N, ZS, true, bound>), grid, dim3(threads), lds, s, a);
  else
    hipLaunchKernelGGL((k_fused<T, N, ZS, false, bound>), grid, dim3(threads), lds, s, a);
}

template <typename T>
hipError_t launch_fused(const FusedArgs<T>& a, hipStream_t s) {
  using T2 = typename Vec2<T>::type;
  if (!fused_supported(a.g, a.nl.n_atoms, sizeof(T2))) return hipErrorInvalidValue;
  const size_t lds = fused_lds_bytes(a.g, a.nl.n_atoms, sizeof(T2));
  const bool per = a.g.periodic != 0;
  switch (a.g.n3) {
    case 12: launch_n<T, 12, 2>(per, a, lds, s); break;
    case 16: launch_n<T, 16, 2>(per, a, lds, s); break;
    case 20: launch_n<T, 20, 1>(per, a, lds, s); break;
    default: launch_n<T, 24, 1>(per, a, lds, s); break;
  }
  return hipGetLastError();
}

// Column split per grid size, fixed so that every path computes the same
// bits: measured on MI355X, splitting the 12^3 and 16^3 columns between two
// wavefronts is faster; at 20^3 the split spills registers and is slower, and
// at 24^3 (576 column threads) two halves would exceed 1024 threads.
int fused_column_split(int n) { return n <= 16 ? 2 : 1; }

template hipError_t launch_fused<double>(const FusedArgs<double>&, hipStream_t);
template hipError_t launch_fused<float>(const FusedArgs<float>&, hipStream_t);

template <typename T, int N, int ZS>
static void launch_pers_n(bool periodic, const FusedArgs<T>* cells, const int2* items, int n_items,
                          int* queue, int wgs, size_t lds, hipStream_t s) {
  constexpr int threads = fused_threads<N, ZS>();
  constexpr int bound = fused_bound<N, ZS>();
  if (periodic)
    hipLaunchKernelGGL((k_fused_persistent<T, N, ZS, true, bound>), dim3(wgs), dim3(threads), lds, s, cells,
                       items, n_items, queue);
  else
    hipLaunchKernelGGL((k_fused_persistent<T, N, ZS, false, bound>), dim3(wgs), dim3(threads), lds, s, cells,
                       items, n_items, queue);
}

template <typename T>
hipError_t launch_fused_persistent(int n, int zs, bool periodic, const FusedArgs<T>* cells, const int2* items,
                                   int n_items, int* queue, int wgs, size_t lds, hipStream_t s) {
  if (wgs < 1 || n_items < 1) return hipErrorInvalidValue;
  if (zs == 2) {
    switch (n) {
      case 12: launch_pers_n<T, 12, 2>(periodic, cells, items, n_items, queue, wgs, lds, s); break;
      case 16: launch_pers_n<T, 16, 2>(periodic, cells, items, n_items, queue, wgs, lds, s); break;
      case 20: launch_pers_n<T, 20, 2>(periodic, cells, items, n_items, queue, wgs, lds, s); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (n) {
      case 12: launch_pers_n<T, 12, 1>(periodic, cells, items, n_items, queue, wgs, lds, s); break;
      case 16: launch_pers_n<T, 16, 1>(periodic, cells, items, n_items, queue, wgs, lds, s); break;
      case 20: launch_pers_n<T, 20, 1>(periodic, cells, items, n_items, queue, wgs, lds, s); break;
      case 24: launch_pers_n<T, 24, 1>(periodic, cells, items, n_items, queue, wgs, lds, s); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

template hipError_t launch_fused_persistent<double>(int, int, bool, const FusedArgs<double>*, const int2*, int,
                                                    int*, int, size_t, hipStream_t);
template hipError_t launch_fused_persistent<float>(int, int, bool, const FusedArgs<float>*, const int2*, int,
                                                   int*, int, size_t, hipStream_t);

}  // namespace td
