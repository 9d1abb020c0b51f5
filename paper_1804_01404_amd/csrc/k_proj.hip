// Kleinman-Bylander projections on the matrix cores (Sec. 3.1, separable
// nonlocal pseudopotential; Sec. 4.1, phase exp(-i kappa.x) for gauge
// invariance):
//
//   u_{o,a,p}^{(m)} = h^3 sum_{e in sphere(a)} B[e][4p+m] exp(i kappa_k . x_e) t_o(idx_e)
//
// with B[e][4p+m] = beta_p(x_e) * (1, x, y, z)[m]. For one atom and a group of
// eight orbitals this is a real product D[16 x 16] = A[16 x K] B[K x 16]
// where row 2j/2j+1 of A holds the real/imaginary part of the phase-shifted
// gathered value of orbital j, K runs over the sphere entries in steps of 4,
// and column 4p+m of B is the moment m of projector p. One wavefront
// accumulates D with v_mfma_f64_16x16x4f64 (FP64 inputs: FP32 orbitals are
// upcast, so the inner products stay FP64 in the mixed-precision path).
//
// Lane layout of v_mfma_f64_16x16x4f64 (checked by a GPU unit test):
//   A: lane l holds A[l % 16][l / 16];  B: lane l holds B[l / 16][l % 16];
//   D: register r of lane l holds D[l / 16 + 4 r][l % 16], r = 0..3.
//
// Stage mode needs only m = 0, so it runs on the four-block FP64 MFMA
// v_mfma_f64_4x4x4f64 instead (k_project_eu): block b holds orbitals 2b and
// 2b + 1 of the group (rows: real and imaginary part of each), its four
// columns are the four projectors, and every product it forms is used.
// Lane layout of v_mfma_f64_4x4x4f64 (checked by a GPU unit test), with
// b = (l >> 2) & 3:
//   A: lane l holds A_b[l & 3][l >> 4];  B: lane l holds B_b[l >> 4][l & 3];
//   D: lane l holds D_b[l >> 4][l & 3].
// Moment mode writes, per orbital and atom, the nonlocal current
// sum_p 2 E_p Im(conj(v_p) u_p) (v = moments 1..3) and the nonlocal energy
// sum_p E_p |u_p|^2 into a partial table [orbital][atom][4]; k_moment_reduce
// then sums the atoms of each orbital in order. Both modes run one wavefront
// per (orbital group, atom).
#include "internal.h"

namespace td {

typedef double d4_t __attribute__((ext_vector_type(4)));

// SPLIT = 1: four (group, atom) items per workgroup, one per wavefront.
// SPLIT = 4 (few items: small cells, or few orbitals over many atoms): one
// item per workgroup, its sphere entries dealt out to the four wavefronts in
// turn, the four partial tiles summed in wavefront order through LDS, so a
// wavefront's serial loop over the sphere is a quarter as long.
template <typename T, int SPLIT>
__global__ __launch_bounds__(256) void k_project(ProjArgs<T> a) {
  using T2 = typename Vec2<T>::type;
  __shared__ double dpart[SPLIT > 1 ? SPLIT : 1][4][64];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int n_groups = (a.n_orb_tot + 7) / 8;
  const int n_atoms = a.nl.n_atoms;
  const int item = SPLIT > 1 ? (int)blockIdx.x : (int)blockIdx.x * 4 + wave;
  const int sub = SPLIT > 1 ? wave : 0;
  const int total = n_groups * n_atoms;
  if (item >= total) return;  // uniform over the wavefront (over the workgroup when split)
  const int grp = item / n_atoms;
  const int at0 = item - grp * n_atoms;
  const int at1 = at0 + 1;
  const int row = lane & 15;   // A row / B and D column
  const int kk = lane >> 4;    // A column / B row / D row block
  const int o_row = grp * 8 + (row >> 1);
  const int part = row & 1;
  const bool row_ok = o_row < a.n_orb_tot;
  const int k_row = row_ok ? o_row / a.n_orb : 0;
  const T2* __restrict__ urow = a.u + (size_t)(row_ok ? o_row : 0) * a.N;
  const double2* __restrict__ phk = a.nl.phk + (size_t)k_row * a.nl.n_ent;

  const int j = row;
  const int p = j >> 2, m = j & 3;
  double acc_moment[4] = {0.0, 0.0, 0.0, 0.0};  // moment mode: per owned orbital

  for (int at = at0; at < at1; ++at) {
    const int e0 = a.nl.atom_start[at], e1 = a.nl.atom_start[at + 1];
    d4_t acc = {0.0, 0.0, 0.0, 0.0};
    // kPipe k steps at a time, loads first (as in k_project_eu): steps past
    // the sphere load its last entry and use 0
    constexpr int kPipe = 4;
    const int step = 4 * SPLIT;
    for (int eb = e0 + 4 * sub; eb < e1; eb += step * kPipe) {
      bool ein[kPipe];
      int idx[kPipe];
      double bv[kPipe];
      double2 p1[kPipe], p2[kPipe];
#pragma unroll
      for (int u = 0; u < kPipe; ++u) {
        const int e = eb + step * u + kk;
        ein[u] = e < e1;
        const int ec = min(e, e1 - 1);
        bv[u] = a.nl.ent_B[(size_t)ec * kCols + j];
        idx[u] = a.nl.ent_idx[ec];
        p1[u] = phk[ec];
        p2[u] = a.phA[ec];
      }
      T2 uv[kPipe];
#pragma unroll
      for (int u = 0; u < kPipe; ++u) uv[u] = urow[idx[u]];
#pragma unroll
      for (int u = 0; u < kPipe; ++u) {
        const double pr = p1[u].x * p2[u].x - p1[u].y * p2[u].y;
        const double pim = p1[u].x * p2[u].y + p1[u].y * p2[u].x;
        const double ur = (double)uv[u].x, ui = (double)uv[u].y;
        const double avv = part ? (pr * ui + pim * ur) : (pr * ur - pim * ui);
        const double av = (ein[u] && row_ok) ? avv : 0.0;
        const double b = ein[u] ? bv[u] : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b, acc, 0, 0, 0);
      }
    }
    if (SPLIT > 1) {
#pragma unroll
      for (int r = 0; r < 4; ++r) dpart[wave][r][lane] = acc[r];
      __syncthreads();
      if (wave != 0) return;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double v = dpart[0][r][lane];
#pragma unroll
        for (int w = 1; w < SPLIT; ++w) v += dpart[w][r][lane];
        acc[r] = v;
      }
    }
    // acc[r] = D[kk + 4r][j]: orbital (kk >> 1) + 2r of the group, real part
    // for even kk, imaginary part for odd kk; the partner lane l ^ 16 holds
    // the other part of the same orbital.
    const double E = a.nl.atom_E[at * kMaxProj + p];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double mine = a.dV * acc[r];
      const double other = __shfl_xor(mine, 16, 64);
      const double ure = (kk & 1) ? other : mine;
      const double uim = (kk & 1) ? mine : other;
      const int o = grp * 8 + (kk >> 1) + 2 * r;
      if (!a.moments) {
        if (m == 0 && (kk & 1) == 0 && o < a.n_orb_tot)
          a.Eu[((size_t)o * n_atoms + at) * kMaxProj + p] = make_double2(E * ure, E * uim);
      } else {
        // u_p lives in the lane of column 4p (same row block): fetch it
        const int src = kk * 16 + 4 * p;
        const double u0r = __shfl(ure, src, 64);
        const double u0i = __shfl(uim, src, 64);
        if (m == 0)
          acc_moment[r] += E * (u0r * u0r + u0i * u0i);           // E_p |u_p|^2
        else
          acc_moment[r] += 2.0 * E * (ure * u0i - uim * u0r);     // 2 E_p Im(conj(v) u)
      }
    }
  }
  if (a.moments) {
    double* part = reinterpret_cast<double*>(a.Eu);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      // sum over p: lanes 4p+m of the same row block (xor over bits 2 and 3)
      double v = acc_moment[r];
      v += __shfl_xor(v, 4, 64);
      v += __shfl_xor(v, 8, 64);
      const int o = grp * 8 + (kk >> 1) + 2 * r;
      if (p == 0 && (kk & 1) == 0 && o < a.n_orb_tot) {
        const int slot = (m == 0) ? 3 : m - 1;
        part[((size_t)o * n_atoms + at0) * 4 + slot] = v;
      }
    }
  }
}

// Stage mode: E_p u_p of every (orbital, atom, projector) on the four-block
// MFMA. One wavefront per (group of eight orbitals, atom); SPLIT as in
// k_project.
template <typename T, int SPLIT, bool ADD>
__global__ __launch_bounds__(256) void k_project_eu(ProjArgs<T> a) {
  using T2 = typename Vec2<T>::type;
  __shared__ double dpart[SPLIT > 1 ? SPLIT : 1][64];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int n_groups = (a.n_orb_tot + 7) / 8;
  const int n_atoms = a.nl.n_atoms;
  const int item = SPLIT > 1 ? (int)blockIdx.x : (int)blockIdx.x * 4 + wave;
  const int sub = SPLIT > 1 ? wave : 0;
  if (item >= n_groups * n_atoms) return;  // uniform over the wavefront (the workgroup when split)
  const int grp = item / n_atoms;
  const int at = item - grp * n_atoms;
  const int blk = (lane >> 2) & 3;
  // A operand: row i = lane & 3 of block blk is orbital 2 blk + (i >> 1),
  // real (i even) or imaginary part; column k = lane >> 4 is entry eb + k
  const int i_a = lane & 3, k_op = lane >> 4;
  const int o_a = grp * 8 + 2 * blk + (i_a >> 1);
  const int part = i_a & 1;
  const bool row_ok = o_a < a.n_orb_tot;
  const int k_a = row_ok ? o_a / a.n_orb : 0;
  T2* __restrict__ urow = const_cast<T2*>(a.u) + (size_t)(row_ok ? o_a : 0) * a.N;
  const double2* __restrict__ phk = a.nl.phk + (size_t)k_a * a.nl.n_ent;
  // B operand: column j = lane & 3 is projector j (its m = 0 column), row k_op
  const int j_b = lane & 3;
  // the previous stage's E_p u_p of this lane's orbital and the wavefront's atom
  // ADD: a.Eu_prev is set and the previous stage's nonlocal term is added
  constexpr bool addback = ADD;
  double2 ep[kMaxProj];
#pragma unroll
  for (int p = 0; p < kMaxProj; ++p) {
    ep[p] = make_double2(0.0, 0.0);
    if (addback && row_ok) ep[p] = a.Eu_prev[((size_t)o_a * n_atoms + at) * kMaxProj + p];
  }

  const int e0 = a.nl.atom_start[at], e1 = a.nl.atom_start[at + 1];
  double acc = 0.0;
  // kPipe k steps at a time: their table and index loads are issued first,
  // then their gathers, then their products, so the gathers of a group are in
  // flight together. Steps past the sphere load its last entry and use 0 (the
  // products then add exact zeros). With the add-back, the points of a group
  // are distinct and the wavefront's own, so its loads may precede its stores.
  constexpr int kPipe = 4;
  const int step = 4 * SPLIT;
  for (int eb = e0 + 4 * sub; eb < e1; eb += step * kPipe) {
    bool ein[kPipe];
    int ec[kPipe], idx[kPipe];
    double bv[kPipe];
    double2 p1[kPipe], p2[kPipe];
#pragma unroll
    for (int u = 0; u < kPipe; ++u) {
      const int e = eb + step * u + k_op;
      ein[u] = e < e1;
      ec[u] = min(e, e1 - 1);
      bv[u] = a.nl.ent_B[(size_t)ec[u] * kCols + 4 * j_b];
      idx[u] = a.nl.ent_idx[ec[u]];
      p1[u] = phk[ec[u]];
      p2[u] = a.phA[ec[u]];
    }
    T2 uv[kPipe];
#pragma unroll
    for (int u = 0; u < kPipe; ++u) uv[u] = urow[idx[u]];
    double bt[kPipe][kMaxProj];
#pragma unroll
    for (int u = 0; u < kPipe; ++u)
#pragma unroll
      for (int p = 0; p < kMaxProj; ++p) bt[u][p] = addback ? a.ent_beta[(size_t)ec[u] * kMaxProj + p] : 0.0;
#pragma unroll
    for (int u = 0; u < kPipe; ++u) {
      const bool use = ein[u] && row_ok;
      const double pr = p1[u].x * p2[u].x - p1[u].y * p2[u].y;
      const double pim = p1[u].x * p2[u].y + p1[u].y * p2[u].x;
      T2 v = uv[u];
      if (addback) {
        // the previous stage's nonlocal term at this point, with the same
        // arithmetic as k_nl_addback (FP64 sum, one rounding to the stage
        // precision); with disjoint spheres this (orbital, point) belongs to
        // this wavefront alone, and the lane holding the real part writes it
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int p = 0; p < kMaxProj; ++p) {
          sr += bt[u][p] * ep[p].x;
          si += bt[u][p] * ep[p].y;
        }
        const double hr = pr * sr + pim * si, hi = pr * si - pim * sr;
        v.x += (T)(a.tau * hi + a.tau_re * hr);
        v.y += (T)(-a.tau * hr + a.tau_re * hi);
        if (use && part == 0) urow[idx[u]] = v;
      }
      const double ur = (double)v.x, ui = (double)v.y;
      const double avv = part ? (pr * ui + pim * ur) : (pr * ur - pim * ui);
      const double av = use ? avv : 0.0;
      const double b = ein[u] ? bv[u] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_4x4x4f64(av, b, acc, 0, 0, 0);
    }
  }
  if (SPLIT > 1) {
    dpart[wave][lane] = acc;
    __syncthreads();
    if (wave != 0) return;
    double v = dpart[0][lane];
#pragma unroll
    for (int w = 1; w < SPLIT; ++w) v += dpart[w][lane];
    acc = v;
  }
  // acc = D_blk[i][j], i = lane >> 4: orbital 2 blk + (i >> 1), real part for
  // even i; lane ^ 16 holds the other part of the same orbital and projector
  const double mine = a.dV * acc;
  const double other = __shfl_xor(mine, 16, 64);
  const int i_d = lane >> 4;
  const int o = grp * 8 + 2 * blk + (i_d >> 1);
  if ((i_d & 1) == 0 && o < a.n_orb_tot) {
    const double E = a.nl.atom_E[at * kMaxProj + j_b];
    a.Eu[((size_t)o * n_atoms + at) * kMaxProj + j_b] = make_double2(E * mine, E * other);
  }
}

// jnl[o][slot] = sum over atoms, in order, of the moment-mode partials
__global__ void k_moment_reduce(const double* __restrict__ part, int n_atoms, int n_orb_tot,
                                double* __restrict__ jnl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_orb_tot * 4) return;
  const int o = i >> 2, slot = i & 3;
  double s = 0.0;
  for (int at = 0; at < n_atoms; ++at) s += part[((size_t)o * n_atoms + at) * 4 + slot];
  jnl[i] = s;
}

// Moment mode uses Eu (free between the last stage and the next step's first
// projection) as its [orbital][atom][4] partial table.
template <typename T>
hipError_t launch_project(const ProjArgs<T>& a, hipStream_t s) {
  const int n_groups = (a.n_orb_tot + 7) / 8;
  const long total = (long)n_groups * a.nl.n_atoms;
  if (total == 0) return hipSuccess;
  // up to 64 items per CU: split each item over a workgroup, so that there
  // are enough wavefronts to hide the latency of the sphere gathers and each
  // serial chain is a quarter as long (the 96^3 cluster, 8 orbital groups x
  // 256 atoms: 0.075 -> 0.048 ms per projection; the 20^3 cell with 512
  // k-points on the per-stage path, 1024 groups x 8 atoms: 0.172 -> 0.140 ms)
  if (!a.moments) {
    const bool add = a.Eu_prev != nullptr;
    if (total < 16384) {
      if (add)
        hipLaunchKernelGGL((k_project_eu<T, 4, true>), dim3((unsigned)total), dim3(256), 0, s, a);
      else
        hipLaunchKernelGGL((k_project_eu<T, 4, false>), dim3((unsigned)total), dim3(256), 0, s, a);
    } else {
      const dim3 grid((unsigned)((total + 3) / 4));
      if (add)
        hipLaunchKernelGGL((k_project_eu<T, 1, true>), grid, dim3(256), 0, s, a);
      else
        hipLaunchKernelGGL((k_project_eu<T, 1, false>), grid, dim3(256), 0, s, a);
    }
    return hipGetLastError();
  }
  if (total < 16384)
    hipLaunchKernelGGL((k_project<T, 4>), dim3((unsigned)total), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_project<T, 1>), dim3((unsigned)((total + 3) / 4)), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !a.moments) return e;
  hipLaunchKernelGGL(k_moment_reduce, dim3((unsigned)((4 * a.n_orb_tot + 255) / 256)), dim3(256), 0, s,
                     reinterpret_cast<const double*>(a.Eu), a.nl.n_atoms, a.n_orb_tot, a.jnl);
  return hipGetLastError();
}

template hipError_t launch_project<double>(const ProjArgs<double>&, hipStream_t);
template hipError_t launch_project<float>(const ProjArgs<float>&, hipStream_t);

// ---------------------------------------------------------------------------
// Unit check of the MFMA lane layout: D = A B for A [16 x 4], B [4 x 16]
// given row-major on the device; used only by a test entry point.
__global__ void k_mfma_layout(const double* A, const double* B, double* D) {
  const int l = threadIdx.x;
  const double av = A[(l % 16) * 4 + l / 16];
  const double bv = B[(l / 16) * 16 + l % 16];
  d4_t acc = {0.0, 0.0, 0.0, 0.0};
  acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
  for (int r = 0; r < 4; ++r) D[(l / 16 + 4 * r) * 16 + l % 16] = acc[r];
}

// D_b = A_b B_b for the four 4 x 4 blocks of v_mfma_f64_4x4x4f64, A, B, D
// given as [4 blocks][4][4] row-major; used only by a test entry point.
__global__ void k_mfma44_layout(const double* A, const double* B, double* D) {
  const int l = threadIdx.x;
  const int b = (l >> 2) & 3;
  const double av = A[b * 16 + (l & 3) * 4 + (l >> 4)];
  const double bv = B[b * 16 + (l >> 4) * 4 + (l & 3)];
  const double d = __builtin_amdgcn_mfma_f64_4x4x4f64(av, bv, 0.0, 0, 0, 0);
  D[b * 16 + (l >> 4) * 4 + (l & 3)] = d;
}

}  // namespace td

extern "C" int tddft_test_mfma44_layout(const double* A, const double* B, double* D) {
  double *dA, *dB, *dD;
  if (hipMalloc(&dA, 64 * sizeof(double)) != hipSuccess) return 1;
  if (hipMalloc(&dB, 64 * sizeof(double)) != hipSuccess) return 1;
  if (hipMalloc(&dD, 64 * sizeof(double)) != hipSuccess) return 1;
  hipError_t e = hipMemcpy(dA, A, 64 * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(dB, B, 64 * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(td::k_mfma44_layout, dim3(1), dim3(64), 0, 0, dA, dB, dD);
    e = hipMemcpy(D, dD, 64 * sizeof(double), hipMemcpyDeviceToHost);
  }
  hipFree(dA);
  hipFree(dB);
  hipFree(dD);
  return e == hipSuccess ? 0 : 2;
}

extern "C" int tddft_test_mfma_layout(const double* A, const double* B, double* D) {
  double *dA, *dB, *dD;
  if (hipMalloc(&dA, 64 * sizeof(double)) != hipSuccess) return 1;
  if (hipMalloc(&dB, 64 * sizeof(double)) != hipSuccess) return 1;
  if (hipMalloc(&dD, 256 * sizeof(double)) != hipSuccess) return 1;
  hipMemcpy(dA, A, 64 * sizeof(double), hipMemcpyHostToDevice);
  hipMemcpy(dB, B, 64 * sizeof(double), hipMemcpyHostToDevice);
  hipLaunchKernelGGL(td::k_mfma_layout, dim3(1), dim3(64), 0, 0, dA, dB, dD);
  hipError_t e = hipMemcpy(D, dD, 256 * sizeof(double), hipMemcpyDeviceToHost);
  hipFree(dA);
  hipFree(dB);
  hipFree(dD);
  return e == hipSuccess ? 0 : 2;
}
