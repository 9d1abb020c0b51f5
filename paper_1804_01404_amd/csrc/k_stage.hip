// Horner stage of the fourth-order Taylor step and the orbital observables.
//
// One stage computes u_{s-1} = w + (-i dt / s) h u_s for one orbital
// (Program Summary: truncated Taylor expansion of exp(-i dt h); Sec. 4.1,
// Eq. TDKS_solid for h). h is applied in the expanded form
//   h u = -1/2 Lap_h u - i kappa . grad_h u + (1/2 |kappa|^2 + V) u + V_NL u,
// with 9-point central differences along each axis.
//
// Work decomposition: one workgroup owns one orbital and one xy-tile and
// marches along z. Each thread owns one (x, y) column: the nine z-neighbours
// of the current plane live in a register queue, the x/y neighbours come
// from the current plane staged in LDS (double-buffered, one barrier per
// plane). Periodic cells whose plane fits one workgroup (n1 n2 <= 1024) use
// the whole plane as the tile and wrap x/y inside LDS; other grids use tiles
// with a 4-point halo loaded from HBM (wrap or zero).
//
// HBM traffic per orbital point and stage: read u_s once, read w once (not in
// the first stage, where u_4 = w), write u_{s-1} once.
#include <type_traits>
#include <utility>

#include "internal.h"

namespace td {

template <typename T2>
__device__ __forceinline__ T2 zero2() {
  T2 z;
  z.x = 0;
  z.y = 0;
  return z;
}

// v where c holds, else zero, selected per component: a select of the whole
// vector value can be compiled as a select between addresses, one of them a
// zero kept in private memory
template <typename T2>
__device__ __forceinline__ T2 keep_if(bool c, const T2& v) {
  T2 r;
  r.x = c ? v.x : 0;
  r.y = c ? v.y : 0;
  return r;
}

// p advanced by an unsigned 32-bit byte offset: with p uniform this is a
// scalar base plus a 32-bit lane offset, which the load instruction adds
// itself (no 64-bit address arithmetic per lane)
template <class X>
__device__ __forceinline__ X* at(X* p, unsigned bytes) {
  using C = typename std::conditional<std::is_const<X>::value, const char, char>::type;
  return reinterpret_cast<X*>(reinterpret_cast<C*>(p) + bytes);
}

__device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Loads and stores of data used once (w, and u_{s-1} of a stage) marked
// non-temporal, so that they do not push out of L2 the u lines that the
// neighbouring tiles read as halo.
typedef float f2v_t __attribute__((ext_vector_type(2)));
typedef double d2v_t __attribute__((ext_vector_type(2)));
template <class T2> struct NtVec;
template <> struct NtVec<float2> { using V = f2v_t; };
template <> struct NtVec<double2> { using V = d2v_t; };
// Copies through the native vector type: a copy of the 16-byte complex128
// struct into an array element is otherwise a memcpy that keeps the array in
// private memory.
template <class T2>
__device__ __forceinline__ T2 load2(const T2* p) {
  using V = typename NtVec<T2>::V;
  const V v = *reinterpret_cast<const V*>(p);
  T2 r;
  r.x = v.x;
  r.y = v.y;
  return r;
}
template <class T2>
__device__ __forceinline__ void store2(T2* p, const T2& a) {
  using V = typename NtVec<T2>::V;
  V v;
  v.x = a.x;
  v.y = a.y;
  *reinterpret_cast<V*>(p) = v;
}
template <class T2>
__device__ __forceinline__ T2 load_once(const T2* p) {
  using V = typename NtVec<T2>::V;
  const V v = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
  T2 r;
  r.x = v.x;
  r.y = v.y;
  return r;
}
template <class T2>
__device__ __forceinline__ void store_once(T2* p, const T2& a) {
  using V = typename NtVec<T2>::V;
  V v;
  v.x = a.x;
  v.y = a.y;
  __builtin_nontemporal_store(v, reinterpret_cast<V*>(p));
}

// The 4-point halo of a tiled workgroup's TX x TY tile (rows above and below,
// columns left and right; the stencil needs no corners): 8 (TX + TY) points
// per plane, dealt to the threads in turn, so a thread stages the same slots
// on every plane. Every thread loads all kHaloSlots slots on every plane (a
// fixed count of loads per plane lets the compiler wait for exactly the
// plane it needs); slots past the last point repeat it and are not staged
// (a per-lane test, so that the slot loop keeps constant indices).
struct HaloSlots {
  int lds[kHaloSlots];       // place in the staged plane
  unsigned off[kHaloSlots];  // in-plane offset of the source point (wrapped or clamped)
  bool own[kHaloSlots];      // a real slot of this thread (not a repeat of the last one)
  bool in[kHaloSlots];       // false outside an isolated grid: staged as zero
  bool stage[kHaloSlots];    // own and in: staged from the plane's load
};

__device__ __forceinline__ HaloSlots halo_slots(int tid, int B, int TX, int TY, int LW, int x0, int y0, int n1,
                                                int n2, bool periodic) {
  HaloSlots h;
  const int S = 8 * (TX + TY);
#pragma unroll
  for (int i = 0; i < kHaloSlots; ++i) {
    h.own[i] = tid + i * B < S;
    const int s = min(tid + i * B, S - 1);
    int lx, ly, x, y;
    if (s < 8 * TX) {  // four rows below, then four above: TX consecutive points each
      const int side = s / (4 * TX), j = (s / TX) % 4, c = s % TX;
      lx = c + 4;
      ly = side ? TY + 4 + j : j;
      x = x0 + c;
      y = side ? y0 + TY + j : y0 - 4 + j;
    } else {  // four columns left, then four right, by row
      const int r = s - 8 * TX;
      const int side = r / (4 * TY), row = (r / 4) % TY, j = r % 4;
      lx = side ? TX + 4 + j : j;
      ly = row + 4;
      x = side ? x0 + TX + j : x0 - 4 + j;
      y = y0 + row;
    }
    bool in = true;
    if (periodic) {
      x = (x + n1) % n1;
      y = (y + n2) % n2;
    } else {
      in = x >= 0 && x < n1 && y >= 0 && y < n2;
      x = min(max(x, 0), n1 - 1);
      y = min(max(y, 0), n2 - 1);
    }
    h.lds[i] = ly * LW + lx;
    h.off[i] = (unsigned)(y * n1 + x);
    h.in[i] = in;
    h.stage[i] = h.own[i] & in;
  }
  return h;
}

// The z loop in rounds of PF planes, plane z + S of a round using prefetch
// slot S (a compile-time index, so every slot stays in its own registers), then
// the last planes of an incomplete round. Every full round issues the same
// loads, which keeps the compiler's wait counts exact.
template <class F, int... S>
__device__ __forceinline__ void round_steps(F& f, int z, std::integer_sequence<int, S...>) {
  (f(z + S, std::integral_constant<int, S>{}), ...);
}
template <class F, int... S>
__device__ __forceinline__ void tail_steps(F& f, int z, int z1, std::integer_sequence<int, S...>) {
  ((z + S < z1 ? (f(z + S, std::integral_constant<int, S>{}), 0) : 0), ...);
}
template <int PF, class F>
__device__ __forceinline__ void run_planes(int z0, int z1, F& f) {
  int z = z0;
  for (; z + PF <= z1; z += PF) round_steps(f, z, std::make_integer_sequence<int, PF>{});
  if (z < z1) tail_steps(f, z, z1, std::make_integer_sequence<int, PF - 1>{});
}

// planes of u, w, V and the halo in flight ahead of the current one: two for
// complex FP32, one for complex128 (whose queue holds twice the registers)
template <typename T, int BC>
constexpr int stage_prefetch() {
  return sizeof(T) == 4 ? 2 : 1;
}

// Loads in the z loop are issued unconditionally at in-bounds plane indices
// (wrapped, or clamped past the ends of an isolated grid and of the slab) and
// zero is selected only where a value is consumed, planes later. A load
// under a branch, or a select right after it, makes the compiler wait for it
// on the spot (and a branch around a load whose alternative is a constant can
// become a flat load, which the LDS wait before the barrier also waits for):
// either undoes the prefetch.
template <typename T, int MODE, int BC>
__global__ __launch_bounds__(1024) void k_stage(StageArgs<T> a) {
  using T2 = typename Vec2<T>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T2* lds = reinterpret_cast<T2*>(smem_raw);

  const Geometry& g = a.g;
  const int n1 = g.n1, n2 = g.n2, n3 = g.n3;
  const int plane = n1 * n2;
  const size_t N = (size_t)plane * n3;
  const int ntiles = g.tiles_x * g.tiles_y;
  const int nz = g.zslabs;
  const int bid = g.xmap ? xcd_block((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
  const int o = bid / (ntiles * nz);
  const int rem = bid - o * ntiles * nz;
  const int tile = rem / nz;
  const int slab = rem - tile * nz;
  // planes z0 .. z1 - 1 of the column (the whole column unless split)
  const int zlen = (n3 + nz - 1) / nz;
  const int z0 = slab * zlen;
  const int z1 = min(n3, z0 + zlen);
  const int k = o / g.n_orb;
  const int TX = g.TX, TY = g.TY;
  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const bool active = ty < TY;
  const int x0 = (tile % g.tiles_x) * TX, y0 = (tile / g.tiles_x) * TY;
  const int gx = x0 + tx, gy = y0 + ty;

  const int LW = (BC == kPeriodicPlane) ? n1 : TX + 8;
  const int LH = (BC == kPeriodicPlane) ? n2 : TY + 8;
  const int lsz = LW * LH;
  const int lx = (BC == kPeriodicPlane) ? tx : tx + 4;
  const int ly = (BC == kPeriodicPlane) ? ty : ty + 4;
  const int lc = ly * LW + lx;

  // LDS places of the x/y neighbours: a table of wrapped places for a whole
  // periodic plane, lc +- m and lc +- m LW (uniform multiples, no vector
  // registers) for a tile with its halo
  int oxp[4], oxm[4], oyp[4], oym[4];
  if (BC == kPeriodicPlane) {
#pragma unroll
    for (int m = 1; m <= 4; ++m) {
      oxp[m - 1] = ly * LW + (tx + m) % n1;
      oxm[m - 1] = ly * LW + (tx - m + n1) % n1;
      oyp[m - 1] = ((ty + m) % n2) * LW + lx;
      oym[m - 1] = ((ty - m + n2) % n2) * LW + lx;
    }
  }
  auto XP = [&](int m) { return BC == kPeriodicPlane ? oxp[m] : lc + (m + 1); };
  auto XM = [&](int m) { return BC == kPeriodicPlane ? oxm[m] : lc - (m + 1); };
  auto YP = [&](int m) { return BC == kPeriodicPlane ? oyp[m] : lc + (m + 1) * LW; };
  auto YM = [&](int m) { return BC == kPeriodicPlane ? oym[m] : lc - (m + 1) * LW; };

  const size_t base = (size_t)o * N;
  // idle threads of the last wave read column 0 and store nothing; every
  // global access is a uniform plane pointer plus this unsigned lane offset
  const unsigned col = active ? (unsigned)(gy * n1 + gx) : 0u;
  const unsigned colb = col * (unsigned)sizeof(T2), colv = col * (unsigned)sizeof(T);
  const T2* __restrict__ src = a.in + base;
  const T2 z2 = zero2<T2>();
  const bool periodic = (BC != kIsolatedTile);
  // plane index of the column load for plane z: wrapped, or clamped (the
  // value is replaced by zero where it is used)
  auto zidx = [&](int z) -> int {
    if (periodic) {
      int zz = z % n3;
      return zz < 0 ? zz + n3 : zz;
    }
    return min(max(z, 0), n3 - 1);
  };
  auto zin = [&](int z) -> bool { return periodic || (z >= 0 && z < n3); };

  // per-step, per-k coefficients (uniform across the workgroup): the k-point's
  // table row is read with scalar loads and the weights come as stage-precision
  // kernel arguments, so none of them occupies vector registers
  const T* __restrict__ ck = a.coef + (size_t)k * kCoef;
  T cx[4], cy[4], cz[4], bx[4], by[4], bz[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    cx[m] = a.lapc[0][m];
    cy[m] = a.lapc[1][m];
    cz[m] = a.lapc[2][m];
    bx[m] = ck[m];
    by[m] = ck[4 + m];
    bz[m] = ck[8 + m];
  }
  const T tau = (T)a.tau;
  const T tau_re = (T)a.tau_re;
  // diagonal without V: kinetic |kappa|^2 / 2 and, in the length gauge, the
  // field's in-plane part E_x x + E_y y (the z part is added per plane)
  T dgx = ck[12], ez = 0;
  if (a.efield) {
    const double xr = (gx - 0.5 * (n1 - 1)) * g.h1;
    const double yr = (gy - 0.5 * (n2 - 1)) * g.h2;
    dgx += (T)(a.efield[0] * xr + a.efield[1] * yr);
    ez = (T)(a.efield[2] * g.h3);
  }
  const T zc = (T)(0.5 * (n3 - 1));

  HaloSlots hs{};
  if (BC != kPeriodicPlane) {
    hs = halo_slots(tid, (int)blockDim.x, TX, TY, LW, x0, y0, n1, n2, periodic);
#pragma unroll
    for (int i = 0; i < kHaloSlots; ++i) hs.off[i] *= (unsigned)sizeof(T2);  // bytes
    // halo points outside an isolated grid are zero on every plane: staged
    // once in both buffers and never written again
#pragma unroll
    for (int i = 0; i < kHaloSlots; ++i)
      if (hs.own[i] && !hs.in[i]) lds[hs.lds[i]] = lds[lsz + hs.lds[i]] = z2;
  }

  constexpr int PF = stage_prefetch<T, BC>();
  T2 q[9];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const T2 v = load2(at(src + (size_t)zidx(z0 + i - 4) * plane, colb));
    q[i] = keep_if(zin(z0 + i - 4), v);
  }
  // slot d holds the column of plane z + 4 and w, V and the halo of plane z
  // for the planes z = z0 + d (mod PF); the loop is unrolled by PF so that a
  // slot's registers keep their loads until they are used (a register
  // rotation would move, and so wait for, values still in flight)
  T2 nxt[PF], wr[PF], hv[PF][kHaloSlots];
  T vr[PF];
  auto fetch = [&](int d, int zp) __attribute__((always_inline)) {  // plane zp into slot d (clamped past the end)
    const size_t pd = (size_t)min(zp, n3 - 1) * plane;
    const T2* __restrict__ sp = src + pd;
    nxt[d] = load2(at(src + (size_t)zidx(zp + 4) * plane, colb));
    if (MODE != kFirst) wr[d] = load_once(at(a.w + base + pd, colb));
    vr[d] = *at(a.V + pd, colv);
#pragma unroll
    for (int i = 0; i < kHaloSlots; ++i)
      if (BC != kPeriodicPlane) hv[d][i] = load2(at(sp, hs.off[i]));
  };
  // slots issued in order (the first plane's wait counts on it)
#pragma unroll
  for (int d = 0; d < PF; ++d) {
    wr[d] = z2;
    fetch(d, z0 + d);
    __builtin_amdgcn_sched_barrier(0);
  }

  auto plane_step = [&](int z, auto slot) __attribute__((always_inline)) {
    constexpr int d = decltype(slot)::value;
    q[8] = keep_if(zin(z + 4), nxt[d]);
    const T2 wv = (MODE == kFirst) ? q[4] : wr[d];
    const T vv = vr[d];
    T2* buf = lds + (z & 1) * lsz;
    if (active) buf[lc] = q[4];
#pragma unroll
    for (int i = 0; i < kHaloSlots; ++i)
      if (BC != kPeriodicPlane && hs.stage[i]) store2(buf + hs.lds[i], hv[d][i]);
    fetch(d, z + PF);
    __syncthreads();

    if (active) {
      const T2 u = q[4];
      T dg = dgx + vv;
      if (a.efield) dg = fmat(ez, (T)z - zc, dg);
      // h u as fused multiply-adds into two accumulators (real, imaginary)
      T hr = dg * u.x;
      T hi = dg * u.y;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        T2 p = buf[XP(m)], n = buf[XM(m)];
        hr = fmat(cx[m], p.x + n.x, hr);
        hr = fmat(bx[m], p.y - n.y, hr);
        hi = fmat(cx[m], p.y + n.y, hi);
        hi = fmat(-bx[m], p.x - n.x, hi);
        p = buf[YP(m)];
        n = buf[YM(m)];
        hr = fmat(cy[m], p.x + n.x, hr);
        hr = fmat(by[m], p.y - n.y, hr);
        hi = fmat(cy[m], p.y + n.y, hi);
        hi = fmat(-by[m], p.x - n.x, hi);
        p = q[5 + m];
        n = q[3 - m];
        hr = fmat(cz[m], p.x + n.x, hr);
        hr = fmat(bz[m], p.y - n.y, hr);
        hi = fmat(cz[m], p.y + n.y, hi);
        hi = fmat(-bz[m], p.x - n.x, hi);
      }
      // u_{s-1} = w + (tau_re - i tau) h u_s
      T2 res;
      res.x = fmat(tau, hi, fmat(tau_re, hr, wv.x));
      res.y = fmat(-tau, hr, fmat(tau_re, hi, wv.y));
      store_once(at(a.out + base + (size_t)z * plane, colb), res);
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) q[i] = q[i + 1];
  };

  run_planes<PF>(z0, z1, plane_step);
}

// Nonlocal term of a stage, added to u_{s-1} after the local part:
//   u_{s-1}(x_e) += (x / s) sum_p beta_p(x_e) exp(-i kappa . x_e) E_p u_p
// for the sphere entries of one colour (atoms whose spheres share no grid
// point, so the entries of one launch touch distinct points); colours run in
// a fixed order. Eu holds E_p u_p (h^3 included) from the projection of u_s.
// One thread per (entry, k-point, block of ob orbitals), looping over the
// block's orbitals; every (entry, orbital) pair is a distinct point of a
// distinct orbital, so the blocks need no ordering among themselves.
template <typename T>
__global__ void k_nl_addback(StageArgs<T> a, const int* __restrict__ ents, int n_ents, int ob) {
  using T2 = typename Vec2<T>::type;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (t >= n_ents) return;
  const int e = ents[t];
  const int S = a.nl.n_ent;
  const int n_orb = a.g.n_orb;
  const size_t N = (size_t)a.g.n1 * a.g.n2 * a.g.n3;
  const int at = a.nl.ent_atom[e];
  const double2 p1 = a.nl.phk[(size_t)k * S + e];
  const double2 p2 = a.phA[e];
  const double pr = p1.x * p2.x - p1.y * p2.y;
  const double pim = p1.x * p2.y + p1.y * p2.x;
  const double* B = a.nl.ent_B + (size_t)e * kCols;
  double b[kMaxProj];
#pragma unroll
  for (int p = 0; p < kMaxProj; ++p) b[p] = B[p * kMoments];
  const int idx = a.nl.ent_idx[e];
  // the entry's table values serve the block's orbitals of this k-point
  const int j0 = blockIdx.z * ob, j1 = min(n_orb, j0 + ob);
  // kPipe orbitals at a time, every load before any store (the points of
  // different orbitals are distinct); past j1 the last orbital is loaded again
  // and not stored
  constexpr int kPipe = 4;
  for (int j = j0; j < j1; j += kPipe) {
    double2 eu[kPipe][kMaxProj];
    T2 v[kPipe];
    T2* dst[kPipe];
#pragma unroll
    for (int u = 0; u < kPipe; ++u) {
      const size_t o = (size_t)k * n_orb + min(j + u, j1 - 1);
      const double2* eo = a.Eu + (o * a.nl.n_atoms + at) * kMaxProj;
#pragma unroll
      for (int p = 0; p < kMaxProj; ++p) eu[u][p] = eo[p];
      dst[u] = a.out + o * N + idx;
      v[u] = *dst[u];
    }
#pragma unroll
    for (int u = 0; u < kPipe; ++u) {
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int p = 0; p < kMaxProj; ++p) {
        sr += b[p] * eu[u][p].x;
        si += b[p] * eu[u][p].y;
      }
      const double hr = pr * sr + pim * si, hi = pr * si - pim * sr;
      v[u].x += (T)(a.tau * hi + a.tau_re * hr);
      v[u].y += (T)(-a.tau * hr + a.tau_re * hi);
      if (j + u < j1) *dst[u] = v[u];
    }
  }
}

template <typename T>
hipError_t launch_nl_addback(const StageArgs<T>& a, const int* ents, int n_ents, int n_orb_tot, hipStream_t s) {
  if (n_ents <= 0) return hipSuccess;
  const int nk = n_orb_tot / a.g.n_orb;
  const int bx = (n_ents + 255) / 256;
  // orbitals per thread: all of them when there are enough workgroups,
  // fewer (down to 2) for small cells
  int ob = a.g.n_orb;
  while (ob > 2 && (long)bx * nk * ((a.g.n_orb + ob - 1) / ob) < 1024) ob = (ob + 1) / 2;
  const dim3 grid((unsigned)bx, (unsigned)nk, (unsigned)((a.g.n_orb + ob - 1) / ob));
  hipLaunchKernelGGL((k_nl_addback<T>), grid, dim3(256), 0, s, a, ents, n_ents, ob);
  return hipGetLastError();
}

template hipError_t launch_nl_addback<double>(const StageArgs<double>&, const int*, int, int, hipStream_t);
template hipError_t launch_nl_addback<float>(const StageArgs<float>&, const int*, int, int, hipStream_t);

// Per-orbital sums used by the current and the energy:
// norm = sum |w|^2, p_mu = sum Im(conj(w) d_mu w), kin = sum Re(conj(w)(-1/2 Lap w)),
// vloc = sum V_loc |w|^2 (the caller multiplies by h1 h2 h3); with EN false
// only norm and p (what each step's current needs), kin and vloc written as
// 0. The neighbour
// differences and their weighted sums d_mu w and -1/2 Lap w are formed in the
// orbital precision (exact differences of FP32 values up to one rounding, then
// FP32 weighted sums for complex FP32); the products with w and the running
// sums over the grid are FP64. complex128 is FP64 throughout.
template <typename T, int BC, bool EN>
__global__ __launch_bounds__(1024) void k_observe(ObserveArgs<T> a) {
  using T2 = typename Vec2<T>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // the plane is staged in the stage precision and widened on read (exact)
  T2* lds = reinterpret_cast<T2*>(smem_raw);
  __shared__ double red[16][6];

  const Geometry& g = a.g;
  const int n1 = g.n1, n2 = g.n2, n3 = g.n3;
  const int plane = n1 * n2;
  const size_t N = (size_t)plane * n3;
  const int ntiles = g.tiles_x * g.tiles_y;
  const int nz = g.zslabs;
  const int bid = g.xmap ? xcd_block((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
  const int o = bid / (ntiles * nz);
  const int rem = bid - o * ntiles * nz;
  const int tile = rem / nz;
  const int slab = rem - tile * nz;
  // planes z0 .. z1 - 1 of the column (the whole column unless split)
  const int zlen = (n3 + nz - 1) / nz;
  const int z0 = slab * zlen;
  const int z1 = min(n3, z0 + zlen);
  const int TX = g.TX, TY = g.TY;
  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const bool active = ty < TY;
  const int x0 = (tile % g.tiles_x) * TX, y0 = (tile / g.tiles_x) * TY;
  const int gx = x0 + tx, gy = y0 + ty;
  const int LW = (BC == kPeriodicPlane) ? n1 : TX + 8;
  const int LH = (BC == kPeriodicPlane) ? n2 : TY + 8;
  const int lsz = LW * LH;
  const int lx = (BC == kPeriodicPlane) ? tx : tx + 4;
  const int ly = (BC == kPeriodicPlane) ? ty : ty + 4;
  const int lc = ly * LW + lx;
  // LDS places of the x/y neighbours: a table of wrapped places for a whole
  // periodic plane, lc +- m and lc +- m LW (uniform multiples, no vector
  // registers) for a tile with its halo
  int oxp[4], oxm[4], oyp[4], oym[4];
  if (BC == kPeriodicPlane) {
#pragma unroll
    for (int m = 1; m <= 4; ++m) {
      oxp[m - 1] = ly * LW + (tx + m) % n1;
      oxm[m - 1] = ly * LW + (tx - m + n1) % n1;
      oyp[m - 1] = ((ty + m) % n2) * LW + lx;
      oym[m - 1] = ((ty - m + n2) % n2) * LW + lx;
    }
  }
  auto XP = [&](int m) { return BC == kPeriodicPlane ? oxp[m] : lc + (m + 1); };
  auto XM = [&](int m) { return BC == kPeriodicPlane ? oxm[m] : lc - (m + 1); };
  auto YP = [&](int m) { return BC == kPeriodicPlane ? oyp[m] : lc + (m + 1) * LW; };
  auto YM = [&](int m) { return BC == kPeriodicPlane ? oym[m] : lc - (m + 1) * LW; };
  const size_t base = (size_t)o * N;
  const unsigned col = active ? (unsigned)(gy * n1 + gx) : 0u;
  const unsigned colb = col * (unsigned)sizeof(T2), cold = col * (unsigned)sizeof(double);
  const T2* __restrict__ src = a.w + base;
  const bool periodic = (BC != kIsolatedTile);
  // differences and weighted sums in the stage precision, products and the
  // running sums in FP64 (the same arithmetic as before for complex128)
  const T2 zt = zero2<T2>();
  // branch-free prefetch as in k_stage: loads at wrapped or clamped plane
  // indices, zero selected where a value is used
  auto zidx = [&](int z) -> int {
    if (periodic) {
      int zz = z % n3;
      return zz < 0 ? zz + n3 : zz;
    }
    return min(max(z, 0), n3 - 1);
  };
  auto zin = [&](int z) -> bool { return periodic || (z >= 0 && z < n3); };
  // weights in the stage precision, from the kernel arguments (the FP64
  // values themselves for complex128)
  auto CL = [&](int mu, int m) -> T { return a.cl[mu][m]; };
  auto CD = [&](int mu, int m) -> T { return a.cd[mu][m]; };
  const T cdiag = (T)a.cdiag;

  HaloSlots hs{};
  if (BC != kPeriodicPlane) {
    hs = halo_slots(tid, (int)blockDim.x, TX, TY, LW, x0, y0, n1, n2, periodic);
#pragma unroll
    for (int i = 0; i < kHaloSlots; ++i) hs.off[i] *= (unsigned)sizeof(T2);  // bytes
#pragma unroll
    for (int i = 0; i < kHaloSlots; ++i)
      if (hs.own[i] && !hs.in[i]) lds[hs.lds[i]] = lds[lsz + hs.lds[i]] = zt;
  }

  constexpr int PF = stage_prefetch<T, BC>();
  double s_norm = 0, s_px = 0, s_py = 0, s_pz = 0, s_kin = 0, s_v = 0;
  T2 q[9];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const T2 v = load2(at(src + (size_t)zidx(z0 + i - 4) * plane, colb));
    q[i] = keep_if(zin(z0 + i - 4), v);
  }
  // slots as in k_stage: column of plane z + 4, V_loc and the halo of plane z
  T2 nxt[PF], hv[PF][kHaloSlots];
  double vl[PF];
  auto fetch = [&](int d, int zp) __attribute__((always_inline)) {
    const size_t pd = (size_t)min(zp, n3 - 1) * plane;
    const T2* __restrict__ sp = src + pd;
    nxt[d] = load2(at(src + (size_t)zidx(zp + 4) * plane, colb));
    if (EN) vl[d] = *at(a.Vloc + pd, cold);
#pragma unroll
    for (int i = 0; i < kHaloSlots; ++i)
      if (BC != kPeriodicPlane) hv[d][i] = load2(at(sp, hs.off[i]));
  };
#pragma unroll
  for (int d = 0; d < PF; ++d) {
    fetch(d, z0 + d);
    __builtin_amdgcn_sched_barrier(0);
  }

  auto plane_step = [&](int z, auto slot) __attribute__((always_inline)) {
    constexpr int d = decltype(slot)::value;
    q[8] = keep_if(zin(z + 4), nxt[d]);
    const double vz = EN ? vl[d] : 0.0;
    T2* buf = lds + (z & 1) * lsz;
    if (active) buf[lc] = q[4];
#pragma unroll
    for (int i = 0; i < kHaloSlots; ++i)
      if (BC != kPeriodicPlane && hs.stage[i]) store2(buf + hs.lds[i], hv[d][i]);
    fetch(d, z + PF);
    __syncthreads();
    if (active) {
      const T2 u = q[4];
      T lr = cdiag * u.x, li = cdiag * u.y;
      T dxr = 0, dxi = 0, dyr = 0, dyi = 0, dzr = 0, dzi = 0;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        T2 p = buf[XP(m)], n = buf[XM(m)];
        if (EN) {
          lr = fmat(CL(0, m), p.x + n.x, lr);
          li = fmat(CL(0, m), p.y + n.y, li);
        }
        dxr = fmat(CD(0, m), p.x - n.x, dxr);
        dxi = fmat(CD(0, m), p.y - n.y, dxi);
        p = buf[YP(m)];
        n = buf[YM(m)];
        if (EN) {
          lr = fmat(CL(1, m), p.x + n.x, lr);
          li = fmat(CL(1, m), p.y + n.y, li);
        }
        dyr = fmat(CD(1, m), p.x - n.x, dyr);
        dyi = fmat(CD(1, m), p.y - n.y, dyi);
        p = q[5 + m];
        n = q[3 - m];
        if (EN) {
          lr = fmat(CL(2, m), p.x + n.x, lr);
          li = fmat(CL(2, m), p.y + n.y, li);
        }
        dzr = fmat(CD(2, m), p.x - n.x, dzr);
        dzi = fmat(CD(2, m), p.y - n.y, dzi);
      }
      const double ux = (double)u.x, uy = (double)u.y;
      const double nn = fmat(ux, ux, uy * uy);
      s_norm += nn;
      s_px = fmat(ux, (double)dxi, fmat(-uy, (double)dxr, s_px));
      s_py = fmat(ux, (double)dyi, fmat(-uy, (double)dyr, s_py));
      s_pz = fmat(ux, (double)dzi, fmat(-uy, (double)dzr, s_pz));
      if (EN) {
        s_kin = fmat(ux, (double)lr, fmat(uy, (double)li, s_kin));
        s_v = fmat(vz, nn, s_v);
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) q[i] = q[i + 1];
  };

  run_planes<PF>(z0, z1, plane_step);
  double v[6] = {s_norm, s_px, s_py, s_pz, s_kin, s_v};
  constexpr int NS = EN ? 6 : 4;  // sums reduced (kin and vloc stay 0 without EN)
#pragma unroll
  for (int i = 0; i < NS; ++i) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_down(v[i], off, 64);
  }
  const int lane = tid & 63, wave = tid >> 6;
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < 6; ++i) red[wave][i] = v[i];
  }
  __syncthreads();
  if (tid < 6) {
    const int nw = (blockDim.x + 63) / 64;
    double s = 0;
    if (tid < NS)
      for (int w = 0; w < nw; ++w) s += red[w][tid];
    a.out[(((size_t)o * ntiles + tile) * nz + slab) * 8 + tid] = s;
  }
}

static int block_threads(const Geometry& g) { return ((g.TX * g.TY + 63) / 64) * 64; }
static size_t lds_elems(int bc, const Geometry& g) {
  return (bc == kPeriodicPlane) ? (size_t)2 * g.n1 * g.n2 : (size_t)2 * (g.TX + 8) * (g.TY + 8);
}

template <typename T, int MODE>
static hipError_t stage_bc(int bc, const StageArgs<T>& a, hipStream_t s) {
  using T2 = typename Vec2<T>::type;
  const dim3 grid((unsigned)((size_t)a.g.n_orb * a.g.n_k * a.g.tiles_x * a.g.tiles_y * a.g.zslabs));
  const dim3 block(block_threads(a.g));
  const size_t lds = lds_elems(bc, a.g) * sizeof(T2);
  switch (bc) {
    case kPeriodicPlane:
      hipLaunchKernelGGL((k_stage<T, MODE, kPeriodicPlane>), grid, block, lds, s, a);
      break;
    case kPeriodicTile:
      hipLaunchKernelGGL((k_stage<T, MODE, kPeriodicTile>), grid, block, lds, s, a);
      break;
    default:
      hipLaunchKernelGGL((k_stage<T, MODE, kIsolatedTile>), grid, block, lds, s, a);
      break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_stage(int mode, int bc, const StageArgs<T>& a, hipStream_t s) {
  if (mode == kFirst) return stage_bc<T, kFirst>(bc, a, s);
  if (mode == kMid) return stage_bc<T, kMid>(bc, a, s);
  return stage_bc<T, kLast>(bc, a, s);
}

template <typename T, bool EN>
static hipError_t observe_bc(int bc, const ObserveArgs<T>& a, hipStream_t s) {
  const dim3 grid((unsigned)((size_t)a.g.n_orb * a.g.n_k * a.g.tiles_x * a.g.tiles_y * a.g.zslabs));
  const dim3 block(block_threads(a.g));
  const size_t lds = lds_elems(bc, a.g) * sizeof(typename Vec2<T>::type);
  switch (bc) {
    case kPeriodicPlane:
      hipLaunchKernelGGL((k_observe<T, kPeriodicPlane, EN>), grid, block, lds, s, a);
      break;
    case kPeriodicTile:
      hipLaunchKernelGGL((k_observe<T, kPeriodicTile, EN>), grid, block, lds, s, a);
      break;
    default:
      hipLaunchKernelGGL((k_observe<T, kIsolatedTile, EN>), grid, block, lds, s, a);
      break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_observe(int bc, const ObserveArgs<T>& a, hipStream_t s) {
  return a.energy ? observe_bc<T, true>(bc, a, s) : observe_bc<T, false>(bc, a, s);
}

template hipError_t launch_stage<double>(int, int, const StageArgs<double>&, hipStream_t);
template hipError_t launch_stage<float>(int, int, const StageArgs<float>&, hipStream_t);
template hipError_t launch_observe<double>(int, const ObserveArgs<double>&, hipStream_t);
template hipError_t launch_observe<float>(int, const ObserveArgs<float>&, hipStream_t);

}  // namespace td
