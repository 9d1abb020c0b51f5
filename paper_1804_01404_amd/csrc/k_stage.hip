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
#include "internal.h"

namespace td {

template <typename T2>
__device__ __forceinline__ T2 zero2() {
  T2 z;
  z.x = 0;
  z.y = 0;
  return z;
}

// planes of u, w and V in flight ahead of the current one: two for complex
// FP32 on tiled grids, one otherwise (measured on 20^3 and 96^3 cells; a
// deeper queue costs complex128 more in registers than it gains)
template <typename T, int BC>
constexpr int stage_prefetch() {
  return (sizeof(T) == 4 && BC != kPeriodicPlane) ? 2 : 1;
}

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
  const int gx = (tile % g.tiles_x) * TX + tx;
  const int gy = (tile / g.tiles_x) * TY + ty;

  const int LW = (BC == kPeriodicPlane) ? n1 : TX + 8;
  const int LH = (BC == kPeriodicPlane) ? n2 : TY + 8;
  const int lsz = LW * LH;
  const int lx = (BC == kPeriodicPlane) ? tx : tx + 4;
  const int ly = (BC == kPeriodicPlane) ? ty : ty + 4;
  const int lc = ly * LW + lx;

  int oxp[4], oxm[4], oyp[4], oym[4];
#pragma unroll
  for (int m = 1; m <= 4; ++m) {
    if (BC == kPeriodicPlane) {
      oxp[m - 1] = ly * LW + (tx + m) % n1;
      oxm[m - 1] = ly * LW + (tx - m + n1) % n1;
      oyp[m - 1] = ((ty + m) % n2) * LW + lx;
      oym[m - 1] = ((ty - m + n2) % n2) * LW + lx;
    } else {
      oxp[m - 1] = lc + m;
      oxm[m - 1] = lc - m;
      oyp[m - 1] = lc + m * LW;
      oym[m - 1] = lc - m * LW;
    }
  }

  const size_t base = (size_t)o * N;
  const int col = gy * n1 + gx;
  const T2* __restrict__ src = a.in + base;
  const T2 z2 = zero2<T2>();
  const bool periodic = (BC != kIsolatedTile);

  auto load_col = [&](int z) -> T2 {
    if (!active) return z2;
    if (!periodic && (z < 0 || z >= n3)) return z2;
    int zz = z;
    if (periodic) {
      zz = z % n3;
      if (zz < 0) zz += n3;
    }
    return src[(size_t)zz * plane + col];
  };
  auto load_xy = [&](int x, int y, int z) -> T2 {
    if (periodic) {
      x = (x % n1 + n1) % n1;
      y = (y % n2 + n2) % n2;
    } else if (x < 0 || x >= n1 || y < 0 || y >= n2) {
      return z2;
    }
    return src[(size_t)z * plane + y * n1 + x];
  };

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
  const T diag_t = ck[12];
  const T tau = (T)a.tau;
  const T tau_re = (T)a.tau_re;
  T ext = 0, ez = 0;
  if (a.efield) {
    const double xr = (gx - 0.5 * (n1 - 1)) * g.h1;
    const double yr = (gy - 0.5 * (n2 - 1)) * g.h2;
    ext = (T)(a.efield[0] * xr + a.efield[1] * yr);
    ez = (T)(a.efield[2] * g.h3);
  }
  const T zc = (T)(0.5 * (n3 - 1));

  // u, w and V are fetched PF planes ahead of their use, so that a plane's
  // loads have that many barrier-separated iterations to arrive
  constexpr int PF = stage_prefetch<T, BC>();
  T2 q[9];
#pragma unroll
  for (int i = 0; i < 8; ++i) q[i] = load_col(z0 + i - 4);
  T2 nxt[PF];
#pragma unroll
  for (int d = 0; d < PF; ++d) nxt[d] = load_col(z0 + 4 + d);
  T2 wr[PF];
  T vr[PF];
#pragma unroll
  for (int d = 0; d < PF; ++d) {
    wr[d] = z2;
    vr[d] = 0;
    if (active && z0 + d < z1) {
      if (MODE != kFirst) wr[d] = a.w[base + (size_t)(z0 + d) * plane + col];
      vr[d] = a.V[(size_t)(z0 + d) * plane + col];
    }
  }

  // tile-edge threads also stage the x/y halo of their tile (4 points out,
  // wrapped or zero), one plane ahead like the column values
  const bool hxm = BC != kPeriodicPlane && active && tx < 4;
  const bool hxp = BC != kPeriodicPlane && active && tx >= TX - 4;
  const bool hym = BC != kPeriodicPlane && active && ty < 4;
  const bool hyp = BC != kPeriodicPlane && active && ty >= TY - 4;
  T2 hal[4] = {z2, z2, z2, z2};
  auto load_halo = [&](int z) {
    if (hxm) hal[0] = load_xy(gx - 4, gy, z);
    if (hxp) hal[1] = load_xy(gx + 4, gy, z);
    if (hym) hal[2] = load_xy(gx, gy - 4, z);
    if (hyp) hal[3] = load_xy(gx, gy + 4, z);
  };
  if (BC != kPeriodicPlane) load_halo(z0);

  for (int z = z0; z < z1; ++z) {
    q[8] = nxt[0];
    const size_t pz = (size_t)z * plane + col;
    T2 wv = (MODE == kFirst) ? q[4] : wr[0];
    const T vv = vr[0];
#pragma unroll
    for (int d = 0; d + 1 < PF; ++d) {
      nxt[d] = nxt[d + 1];
      wr[d] = wr[d + 1];
      vr[d] = vr[d + 1];
    }
    if (z + PF < z1) {
      nxt[PF - 1] = load_col(z + 4 + PF);
      if (active) {
        if (MODE != kFirst) wr[PF - 1] = a.w[base + pz + (size_t)PF * plane];
        vr[PF - 1] = a.V[pz + (size_t)PF * plane];
      }
    }

    T2* buf = lds + (z & 1) * lsz;
    if (active) {
      buf[lc] = q[4];
      if (BC != kPeriodicPlane) {
        // this plane's halo values, loaded one plane ahead
        if (hxm) buf[lc - 4] = hal[0];
        if (hxp) buf[lc + 4] = hal[1];
        if (hym) buf[lc - 4 * LW] = hal[2];
        if (hyp) buf[lc + 4 * LW] = hal[3];
        if (z + 1 < z1) load_halo(z + 1);
      }
    }
    __syncthreads();

    if (active) {
      const T2 u = q[4];
      T dg = diag_t + vv;
      if (a.efield) dg += ext + ez * ((T)z - zc);
      T hr = dg * u.x;
      T hi = dg * u.y;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        T2 p = buf[oxp[m]], n = buf[oxm[m]];
        hr += cx[m] * (p.x + n.x) + bx[m] * (p.y - n.y);
        hi += cx[m] * (p.y + n.y) - bx[m] * (p.x - n.x);
        p = buf[oyp[m]];
        n = buf[oym[m]];
        hr += cy[m] * (p.x + n.x) + by[m] * (p.y - n.y);
        hi += cy[m] * (p.y + n.y) - by[m] * (p.x - n.x);
        p = q[5 + m];
        n = q[3 - m];
        hr += cz[m] * (p.x + n.x) + bz[m] * (p.y - n.y);
        hi += cz[m] * (p.y + n.y) - bz[m] * (p.x - n.x);
      }
      T2 res;
      res.x = wv.x + tau * hi + tau_re * hr;
      res.y = wv.y - tau * hr + tau_re * hi;
      a.out[base + pz] = res;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) q[i] = q[i + 1];
  }
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
  for (int j = j0; j < j1; ++j) {
    const size_t o = (size_t)k * n_orb + j;
    const double2* eu = a.Eu + (o * a.nl.n_atoms + at) * kMaxProj;
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int p = 0; p < kMaxProj; ++p) {
      sr += b[p] * eu[p].x;
      si += b[p] * eu[p].y;
    }
    const double hr = pr * sr + pim * si, hi = pr * si - pim * sr;
    T2* dst = a.out + o * N + idx;
    T2 v = *dst;
    v.x += (T)(a.tau * hi + a.tau_re * hr);
    v.y += (T)(-a.tau * hr + a.tau_re * hi);
    *dst = v;
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
// vloc = sum V_loc |w|^2 (the caller multiplies by h1 h2 h3). The neighbour
// differences and their weighted sums d_mu w and -1/2 Lap w are formed in the
// orbital precision (exact differences of FP32 values up to one rounding, then
// FP32 weighted sums for complex FP32); the products with w and the running
// sums over the grid are FP64. complex128 is FP64 throughout.
template <typename T, int BC>
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
  const int gx = (tile % g.tiles_x) * TX + tx;
  const int gy = (tile / g.tiles_x) * TY + ty;
  const int LW = (BC == kPeriodicPlane) ? n1 : TX + 8;
  const int LH = (BC == kPeriodicPlane) ? n2 : TY + 8;
  const int lsz = LW * LH;
  const int lx = (BC == kPeriodicPlane) ? tx : tx + 4;
  const int ly = (BC == kPeriodicPlane) ? ty : ty + 4;
  const int lc = ly * LW + lx;
  int oxp[4], oxm[4], oyp[4], oym[4];
#pragma unroll
  for (int m = 1; m <= 4; ++m) {
    if (BC == kPeriodicPlane) {
      oxp[m - 1] = ly * LW + (tx + m) % n1;
      oxm[m - 1] = ly * LW + (tx - m + n1) % n1;
      oyp[m - 1] = ((ty + m) % n2) * LW + lx;
      oym[m - 1] = ((ty - m + n2) % n2) * LW + lx;
    } else {
      oxp[m - 1] = lc + m;
      oxm[m - 1] = lc - m;
      oyp[m - 1] = lc + m * LW;
      oym[m - 1] = lc - m * LW;
    }
  }
  const size_t base = (size_t)o * N;
  const int col = gy * n1 + gx;
  const T2* __restrict__ src = a.w + base;
  const bool periodic = (BC != kIsolatedTile);
  // differences and weighted sums in the stage precision, products and the
  // running sums in FP64 (the same arithmetic as before for complex128)
  const T2 zt = zero2<T2>();
  auto load_col = [&](int z) -> T2 {
    if (!active) return zt;
    if (!periodic && (z < 0 || z >= n3)) return zt;
    int zz = z;
    if (periodic) {
      zz = z % n3;
      if (zz < 0) zz += n3;
    }
    return src[(size_t)zz * plane + col];
  };
  auto load_xy = [&](int x, int y, int z) -> T2 {
    if (periodic) {
      x = (x % n1 + n1) % n1;
      y = (y % n2 + n2) % n2;
    } else if (x < 0 || x >= n1 || y < 0 || y >= n2) {
      return zt;
    }
    return src[(size_t)z * plane + y * n1 + x];
  };
  // weights: the FP64 kernel arguments themselves for complex128, a copy in
  // FP32 registers for complex FP32
  T cl[3][4], cd[3][4];
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int mu = 0; mu < 3; ++mu)
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        cl[mu][m] = (T)a.lap[mu][m + 1];
        cd[mu][m] = (T)a.dh[mu][m];
      }
  }
  auto CL = [&](int mu, int m) -> T {
    if constexpr (sizeof(T) == 8) return a.lap[mu][m + 1];
    else return cl[mu][m];
  };
  auto CD = [&](int mu, int m) -> T {
    if constexpr (sizeof(T) == 8) return a.dh[mu][m];
    else return cd[mu][m];
  };
  const T cdiag = (T)a.cdiag;

  double s_norm = 0, s_px = 0, s_py = 0, s_pz = 0, s_kin = 0, s_v = 0;
  T2 q[9];
#pragma unroll
  for (int i = 0; i < 8; ++i) q[i] = load_col(z0 + i - 4);
  T2 nxt = load_col(z0 + 4);  // the column one plane ahead, and V_loc
  double vl_nxt = active ? a.Vloc[(size_t)z0 * plane + col] : 0.0;
  for (int z = z0; z < z1; ++z) {
    q[8] = nxt;
    if (z + 1 < z1) nxt = load_col(z + 5);
    const double vl = vl_nxt;
    if (active && z + 1 < z1) vl_nxt = a.Vloc[(size_t)(z + 1) * plane + col];
    T2* buf = lds + (z & 1) * lsz;
    if (active) {
      buf[lc] = q[4];
      if (BC != kPeriodicPlane) {
        if (tx < 4) buf[lc - 4] = load_xy(gx - 4, gy, z);
        if (tx >= TX - 4) buf[lc + 4] = load_xy(gx + 4, gy, z);
        if (ty < 4) buf[lc - 4 * LW] = load_xy(gx, gy - 4, z);
        if (ty >= TY - 4) buf[lc + 4 * LW] = load_xy(gx, gy + 4, z);
      }
    }
    __syncthreads();
    if (active) {
      const T2 u = q[4];
      T lr = cdiag * u.x, li = cdiag * u.y;
      T dxr = 0, dxi = 0, dyr = 0, dyi = 0, dzr = 0, dzi = 0;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        T2 p = buf[oxp[m]], n = buf[oxm[m]];
        lr += CL(0, m) * (p.x + n.x);
        li += CL(0, m) * (p.y + n.y);
        dxr += CD(0, m) * (p.x - n.x);
        dxi += CD(0, m) * (p.y - n.y);
        p = buf[oyp[m]];
        n = buf[oym[m]];
        lr += CL(1, m) * (p.x + n.x);
        li += CL(1, m) * (p.y + n.y);
        dyr += CD(1, m) * (p.x - n.x);
        dyi += CD(1, m) * (p.y - n.y);
        p = q[5 + m];
        n = q[3 - m];
        lr += CL(2, m) * (p.x + n.x);
        li += CL(2, m) * (p.y + n.y);
        dzr += CD(2, m) * (p.x - n.x);
        dzi += CD(2, m) * (p.y - n.y);
      }
      const double ux = (double)u.x, uy = (double)u.y;
      const double nn = ux * ux + uy * uy;
      s_norm += nn;
      s_px += ux * (double)dxi - uy * (double)dxr;
      s_py += ux * (double)dyi - uy * (double)dyr;
      s_pz += ux * (double)dzi - uy * (double)dzr;
      s_kin += ux * (double)lr + uy * (double)li;
      s_v += vl * nn;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) q[i] = q[i + 1];
  }
  double v[6] = {s_norm, s_px, s_py, s_pz, s_kin, s_v};
#pragma unroll
  for (int i = 0; i < 6; ++i) {
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

template <typename T>
hipError_t launch_observe(int bc, const ObserveArgs<T>& a, hipStream_t s) {
  const dim3 grid((unsigned)((size_t)a.g.n_orb * a.g.n_k * a.g.tiles_x * a.g.tiles_y * a.g.zslabs));
  const dim3 block(block_threads(a.g));
  const size_t lds = lds_elems(bc, a.g) * sizeof(typename Vec2<T>::type);
  switch (bc) {
    case kPeriodicPlane:
      hipLaunchKernelGGL((k_observe<T, kPeriodicPlane>), grid, block, lds, s, a);
      break;
    case kPeriodicTile:
      hipLaunchKernelGGL((k_observe<T, kPeriodicTile>), grid, block, lds, s, a);
      break;
    default:
      hipLaunchKernelGGL((k_observe<T, kIsolatedTile>), grid, block, lds, s, a);
      break;
  }
  return hipGetLastError();
}

template hipError_t launch_stage<double>(int, int, const StageArgs<double>&, hipStream_t);
template hipError_t launch_stage<float>(int, int, const StageArgs<float>&, hipStream_t);
template hipError_t launch_observe<double>(int, const ObserveArgs<double>&, hipStream_t);
template hipError_t launch_observe<float>(int, const ObserveArgs<float>&, hipStream_t);

}  // namespace td
