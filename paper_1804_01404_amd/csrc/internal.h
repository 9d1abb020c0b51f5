// Internal declarations shared by the kernels and the C ABI layer.
// Device layout (all in HBM, owned by the context):
//   W, U0, U1   orbitals and the two Horner stage buffers,
//               [n_k][n_orb][n3][n2][n1] of T2 (double2 or float2)
//   V           total Kohn-Sham potential [N] in double and in float
//   NL tables   sphere entries grouped by atom (see NLTables)
//   per-step    kappa [n_k][3], kappaJ [n_k][3], E [3], phA [S], phAJ [S]
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <algorithm>

namespace td {

constexpr double kC = 137.035999084;   // speed of light, atomic units
constexpr int kHalf = 4;               // stencil half width (9 points per axis)
constexpr int kMaxProj = 4;            // projectors per atom
constexpr int kMoments = 4;            // beta, x beta, y beta, z beta
constexpr int kCols = kMaxProj * kMoments;  // MFMA B-matrix columns (16)
// halo points a thread of a tiled stage or observe workgroup stages per plane
// at most: 8 (TX + TY) points over ceil64(TX TY) threads
constexpr int kHaloSlots = 3;
__host__ __device__ inline bool halo_fits(int TX, int TY) {
  return 8 * (TX + TY) <= kHaloSlots * ((TX * TY + 63) / 64) * 64;
}
constexpr int kCoef = 16;  // per k-point: kappa_mu d_m / h_mu for x, y, z (3 x 4), diagonal, padding

enum StageMode { kFirst = 0, kMid = 1, kLast = 2 };
enum BcKind { kPeriodicPlane = 0, kPeriodicTile = 1, kIsolatedTile = 2 };

// Nonlocal tables on the device. Entries e = 0..S-1 are grouped by atom:
// atom a owns entries [atom_start[a], atom_start[a+1]).
struct NLTables {
  int n_atoms = 0;
  int n_ent = 0;
  const int* atom_start = nullptr;   // [n_atoms + 1]
  const int* ent_idx = nullptr;      // [S] flat grid index
  const int* ent_atom = nullptr;     // [S]
  const double* ent_B = nullptr;     // [S][16]: column 4p+m = beta_p * (1, x, y, z)[m]
  const double* atom_E = nullptr;    // [n_atoms][4] KB energies (0 where absent)
  const int* pt_ptr = nullptr;       // [N + 1] per grid point: entries covering it
  const int* pt_ent = nullptr;       // [nnz]
  const double2* phk = nullptr;      // [n_k][S] exp(i k . x_e)
};

struct Geometry {
  int n1, n2, n3;
  double h1, h2, h3;
  int periodic;
  int n_orb, n_k;         // orbitals per k-point, k-points
  // tiling of the stage kernels: xy tiles, and z split into zslabs slabs when
  // there are too few (orbital, tile) workgroups to fill the chip
  int TX, TY, tiles_x, tiles_y;
  int zslabs;
  // 1: renumber workgroups so that each XCD (each with its own L2) gets a
  // contiguous range of (orbital, tile, slab) blocks; the result does not
  // depend on it
  int xmap;
};

// Workgroups are dealt to the eight XCDs in turn (XCD = id mod 8). With
// q = n / 8, the first 8 q ids are renumbered so that XCD x runs the logical
// blocks x q .. x q + q - 1 in order; the tail keeps its id (a bijection).
__device__ __forceinline__ int xcd_block(int b, int n) {
  const int q = n >> 3;
  if (b >= 8 * q) return b;
  return (b & 7) * q + (b >> 3);
}

template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

template <typename T>
struct StageArgs {
  using T2 = typename Vec2<T>::type;
  const T2* in;            // u_s (the first stage reads W here)
  const T2* w;             // W (Horner base), unused by the first stage
  T2* out;                 // u_{s-1}; the last stage writes W in place
  const T* V;              // total potential in the stage precision
  const double* kappa;     // [n_k][3] for this step
  const double* efield;    // [3] length gauge field, or nullptr
  const double2* Eu;       // [n_orb_tot][n_atoms][4] E_p u_p, or nullptr
  const double2* phA;      // [S] exp(i A.x/c) for this step
  NLTables nl;
  Geometry g;
  double lap[3][5];        // -1/2 c_m / h_mu^2
  double dh[3][4];         // d_m / h_mu
  double cdiag;            // sum_mu -1/2 c_0 / h_mu^2
  double tau;              // dt / s: u_{s-1} = w + (tau_re - i tau) h u_s
  double tau_re;           // 0 in real time; -tau_imag / s for imaginary time
  const T* coef;           // [n_k][kCoef] kappa_mu d_m / h_mu and the diagonal, stage precision
  T lapc[3][4];            // off-centre Laplacian weights -1/2 c_m / h_mu^2, stage precision
};

template <typename T>
struct ObserveArgs {
  using T2 = typename Vec2<T>::type;
  const T2* w;
  const double* Vloc;      // [N]
  Geometry g;
  double dh[3][4];
  double lap[3][5];
  double cdiag;
  double* out;             // [n_orb_tot][tiles][8]: norm, p_x, p_y, p_z, kin, vloc
  int energy;              // 0: norm and p only (kin, vloc written as 0), as each step needs
  // off-centre weights of lap and dh in the stage precision (kernel
  // arguments, so they stay in scalar registers); set by set_weights
  T cl[3][4], cd[3][4];
  void set_weights() {
    for (int mu = 0; mu < 3; ++mu)
      for (int m = 0; m < 4; ++m) {
        cl[mu][m] = (T)lap[mu][m + 1];
        cd[mu][m] = (T)dh[mu][m];
      }
  }
};

template <typename T>
struct ProjArgs {
  using T2 = typename Vec2<T>::type;
  const T2* u;             // [n_orb_tot][N]
  const double2* phA;      // [S]
  NLTables nl;
  int N;
  int n_orb, n_orb_tot;
  double dV;
  int moments;             // 0: stage projections -> Eu; 1: all 16 columns -> proj
  double2* Eu;             // [n_orb_tot][n_atoms][4]
  double* jnl;             // moments: [n_orb_tot][4]: nonlocal current (3) and energy
  // stage mode with disjoint spheres: the nonlocal term of the stage that
  // produced u, tau (-i tau + tau_re) sum_p beta_p exp(-i kappa.x) Eu_prev_p,
  // is first added to u at the sphere points (in place) and the sum projected;
  // Eu_prev = nullptr: u is complete
  const double2* Eu_prev;  // [n_orb_tot][n_atoms][4]
  const double* ent_beta;  // [S][4] beta_p
  double tau, tau_re;
};

template <typename T>
struct FusedArgs {
  using T2 = typename Vec2<T>::type;
  T2* w;                   // [n_orb_tot][N], updated in place
  const T* V;              // [N] total potential, stage precision
  const double* Vloc;      // [N]
  const double* kappa;     // [n_k][3] at the step midpoint
  const double2* phA;      // [S] exp(i A_mid . x / c)
  const double2* phAJ;     // [S] exp(i A_{n+1} . x / c)
  const double* efield;    // [3] length gauge or nullptr
  NLTables nl;
  const double* ent_beta;  // [S][4] beta_p (0 beyond n_proj)
  const double* ent_x;     // [S][3]
  int n_colors;            // atoms grouped so that spheres within a group are disjoint
  const int* color_start;  // [n_colors + 1] into color_atoms
  const int* color_atoms;  // [n_atoms]
  Geometry g;
  double lap[3][5];
  double dh[3][4];
  double cdiag;
  double dt, dV;
  double* obs;             // [n_orb_tot][8]
  double* jnl;             // [n_orb_tot][4]
  T* coef;                 // [n_k][kCoef] stencil coefficients of the step, stage precision
  double2* phkA;           // [n_k][S] exp(i kappa . x_e) at the step midpoint (set with coef)
  T lapc[3][4];            // off-centre Laplacian weights -1/2 c_m / h_mu^2, stage precision
  T dhc[3][4];             // first-derivative weights d_m / h_mu, stage precision
};

// Becke-Johnson / Tran-Blaha exchange (k_mgga.hip): grid and the plain
// 9-point derivative weights
struct MggaArgs {
  Geometry g;
  double d1[3][4];         // d_m / h_mu
  double d2[3][5];         // c_m / h_mu^2
};

// ---- launchers (defined in the .hip files) --------------------------------
template <typename T>
hipError_t launch_stage(int mode, int bc, const StageArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_nl_addback(const StageArgs<T>& a, const int* ents, int n_ents, int n_orb_tot, hipStream_t s);
template <typename T>
hipError_t launch_observe(int bc, const ObserveArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_project(const ProjArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_fused(const FusedArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_fused_coef(const FusedArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_coef_table(const double* kappa, int n_k, const double dh[3][4], double cdiag, T* coef,
                             hipStream_t s);
bool fused_supported(const Geometry& g, int n_atoms, size_t elem);
size_t fused_lds_bytes(const Geometry& g, int n_atoms, size_t elem);
int fused_column_split(int n);
template <typename T>
hipError_t launch_fused_persistent(int n, int zs, bool periodic, const FusedArgs<T>* cells, const int2* items,
                                   int n_items, int* queue, int wgs, size_t lds, hipStream_t s);

hipError_t launch_step_params(const double* A, const int* counter, int use_counter,
                              const double* kpt, int n_k, const double* ent_x, int S, int gauge,
                              double dt, double* kappa, double* kappaJ, double* efield, double2* phA,
                              double2* phAJ, double* Alast, hipStream_t s);

template <typename T>
hipError_t launch_rho_partial(const typename Vec2<T>::type* w, const double* kw, int n_orb, int n_k,
                              int N, int chunk, double* part, hipStream_t s);
hipError_t launch_rho_reduce(const double* part, int nchunks, int N, double* rho, hipStream_t s);

// rho (with n1..n3): the first pass reads the density into the M-box itself;
// K: the pass multiplies what it stores by K (the Poisson kernel)
hipError_t launch_fft_axis(double2* data, int M1, int M2, int M3, int axis, int sign, hipStream_t s,
                           const double* rho = nullptr, int n1 = 0, int n2 = 0, int n3 = 0,
                           const double* K = nullptr);
// a pass over part of the box: lines (i1 < l1, i2 < l2) — (y, z) for the x
// axis, (x, z) for y, (x, y) for z — reading elements below n_in (the rest is
// 0) and storing those below n_out; fused (z axis, with K): forward, times K,
// inverse in one pass
hipError_t launch_fft_lines(double2* data, int M1, int M2, int M3, int axis, int sign, hipStream_t s,
                            const double* rho, int n1, int n2, int n3, const double* K, int l1, int l2, int n_in,
                            int n_out, int fused);
// Per-cell arguments of the end of a step (current, density, Poisson, xc)
// when a group of same-shape cells runs it with one launch per kernel: the
// cell is a grid dimension and each cell's pointers come from this table.
struct TailCell {
  const void* w;          // orbitals [n_orb n_k][N], stage precision
  const double* kw;       // [n_k]
  int n_orb, n_k, nchunks;
  double* rho_out;        // the density pass's output: rho with one chunk, else rho_part
  double* rho_part;       // [nchunks][N]
  double* rho;            // [N]
  double2* fft;           // M-box
  const double* Kfft;     // Poisson kernel on the M-box
  double vh_scale;
  const double* Vloc;
  double* Vd;
  float* Vf;
  double* vh;
  double* exc;
  const double* obs;      // [n_orb n_k][tiles][8]
  const double* jnl;      // [n_orb n_k][4] or nullptr
  int use_nl;
  const double* kappaJ;
  double dV, volume;
  int* counter;
  double* Jtab;
  double* scalars;
  int* nanflag;
  double norm_tol;
};

// Per-cell arguments of the start of a fused step (field, kappa and phases,
// the stencil coefficients, the per-k sphere phases) for one launch per
// kernel over a group of cells.
struct ParamCell {
  const double* A;        // A table [..][3]
  const int* counter;
  const double* kpt;      // [n_k][3]
  int n_k, S, gauge;
  const double* ent_x;    // [S][3]
  double dt;
  double* kappa;
  double* kappaJ;
  double* efield;
  double2* phA;
  double2* phAJ;
  double* Alast;
  double dh[3][4];
  double cdiag;
  void* coef;             // [n_k][16] stage precision
  const double2* phk;     // [n_k][S]
  double2* phkA;          // [n_k][S]
};

// A batch's per-cell A and J tables moved with one copy each way: the cells'
// table pointers, counters and NaN flags.
struct IOCell {
  double* A;
  int* counter;
  const double* J;
  const int* nanflag;
};
// io[c] and the staged A tables (len doubles per cell): A tables to the cells,
// their step counters to 0
hipError_t launch_batch_tables_in(const IOCell* io, int ncells, const double* staged, int len, hipStream_t s);
// the cells' J tables (len doubles) and NaN flags to staged [ncells][len + 1]
hipError_t launch_batch_tables_out(const IOCell* io, int ncells, double* staged, int len, hipStream_t s);

hipError_t launch_step_params_group(const ParamCell* tab, int ncells, int max_S, hipStream_t s);
template <typename T>
hipError_t launch_fused_coef_group(const ParamCell* tab, int ncells, int max_nk, long max_phases, hipStream_t s);

template <typename T>
hipError_t launch_rho_partial_group(const TailCell* tab, int ncells, int N, int chunk, int max_chunks,
                                    hipStream_t s);
hipError_t launch_rho_reduce_group(const TailCell* tab, int ncells, int N, hipStream_t s);
// as launch_fft_lines for every cell of tab (same box and lines); use_rho /
// use_K: the pass reads the cell's rho / multiplies by its K
hipError_t launch_fft_lines_group(const TailCell* tab, int ncells, int M1, int M2, int M3, int axis, int sign,
                                  int use_rho, int n1, int n2, int n3, int use_K, int l1, int l2, int n_in,
                                  int n_out, int fused, hipStream_t s);
hipError_t launch_xc_group(const TailCell* tab, int ncells, int n1, int n2, int n3, int M1, int M2, int hartree,
                           int xc, hipStream_t s);
hipError_t launch_finish_group(const TailCell* tab, int ncells, int tiles, hipStream_t s);

hipError_t launch_xc_assemble(const double2* data, int n1, int n2, int n3, int M1, int M2, int M3,
                              double vh_scale, const double* rho, const double* Vloc, int hartree,
                              int xc, const double* vx_mgga, double* Vd, float* Vf, double* vh, double* exc,
                              hipStream_t s);
template <typename T>
hipError_t launch_rho_tau_partial(const typename Vec2<T>::type* w, const double* kw, const double* kappa,
                                  const MggaArgs& a, int chunk, double* part_rho, double* part_tau,
                                  hipStream_t s);
int rho_tau_chunk(const Geometry& g, int n_tot);
hipError_t launch_mgga_potential(const double* rho, const double* tau, const MggaArgs& a, int tb09, double dV,
                                 double volume, double* gpart, double* cval, double* vx, hipStream_t s);

hipError_t launch_finish(const double* obs, int tiles, const double* jnl, int use_nl,
                         const double* kw, const double* kappaJ, int n_orb, int n_k, double dV,
                         double volume, int* counter, int bump, double* Jtab, double* scalars,
                         int* nanflag, double norm_tol, hipStream_t s);

hipError_t launch_grid_sums(const double* rho, const double* rho0, const double* vh,
                            const double* exc, Geometry g, double* out, hipStream_t s);

template <typename T>
hipError_t launch_convert_in(const double2* src, typename Vec2<T>::type* dst, size_t n, hipStream_t s);
template <typename T>
hipError_t launch_convert_out(const typename Vec2<T>::type* src, double2* dst, size_t n, hipStream_t s);
template <typename T>
hipError_t launch_kick(typename Vec2<T>::type* w, Geometry g, double F0, int axis, size_t n_orb_tot,
                       hipStream_t s);
hipError_t launch_set_int(int* p, int v, hipStream_t s);
template <typename T>
hipError_t launch_gram(const typename Vec2<T>::type* w, int n_orb, int n_k, int N, double dV, double2* S,
                       hipStream_t s);
template <typename T>
hipError_t launch_overlap_weight(const typename Vec2<T>::type* ref, const typename Vec2<T>::type* w, int n_orb,
                                 int n_k, int N, double dV, double* Sk, hipStream_t s);
template <typename T>
hipError_t launch_apply_lower(const typename Vec2<T>::type* w, const double2* M, int n_orb, int n_k, int N,
                              typename Vec2<T>::type* out, hipStream_t s);
hipError_t launch_chol_inverse(double2* S, double2* M, int n, int n_k, int* bad, hipStream_t s);
hipError_t launch_real_part(const double2* src, double* dst, size_t n, hipStream_t s);
hipError_t launch_fill(double* p, double v, size_t n, hipStream_t s);
hipError_t launch_copy8(const void* src, void* dst, size_t bytes, hipStream_t s);
hipError_t launch_mid_potential(const double* Vn, double* Vd, float* Vf, size_t n, hipStream_t s);

// ---- spectra and work from time series (k_spectra.hip) ----------------------
constexpr int kSpecThreads = 256;    // frequencies per workgroup
constexpr int kSpecChunksMax = 64;   // sample chunks summed in a fixed order
int spec_chunks(int n_t);
// scratch: 1 + spec_chunks(n_t) * n_w double2 (the mean, then the chunk partials)
size_t spectrum_scratch_entries(int n_t, int n_w);
// kind 0: out = scale * Z as [n_w][2] and eps ([n_w][2], may be null);
// kind 1: out[j] = (2 w_j / pi) Im Z(w_j) * scale
hipError_t launch_spectrum(const double* x, int n_t, double dt, const double* om, int n_w, int kind, double scale,
                           int use_mask, int subtract_mean, double2* scratch, double* out, double* eps,
                           hipStream_t s);
hipError_t launch_work(const double* I, const double* A, int n_t, double dt, double volume, double* W, hipStream_t s);
// message of the last failed call that has no context (thread-local)
void set_stateless_error(const char* msg);
const char* stateless_error();

// ---- multiscale Maxwell (k_maxwell.hip) -----------------------------------
hipError_t launch_fdtd_step(const double* A_now, const double* A_prev, const double* I, double* A_new, int n,
                            double S2, double src, double q, const double inc[4], hipStream_t s);
hipError_t launch_ring_push(const double* A, int x0, int n_mat, float* ring, int W, int slot, double inv_scale,
                            hipStream_t s);
hipError_t launch_ring_windows(const float* ring, int n_mat, int W, int head, float* X, hipStream_t s);
hipError_t launch_scatter_current(const float* y, int x0, int n_mat, int n, double j_scale, double* I,
                                  hipStream_t s);
hipError_t launch_ms_gate(const double* A, int x0, int n_mat, double a_max, int* flag, hipStream_t s);
hipError_t launch_em_energy(const double* A_now, const double* A_prev, int n, double dx, double dt, double* out,
                            hipStream_t s);
hipError_t launch_ms_work_step(const double* A_new, const double* A_now, const double* I_now, const double* I_new,
                               int x0, int n_mat, double dx, double dt, double* W, hipStream_t s);
hipError_t launch_ms_work_history(const double* A, const double* I, int steps, int n_mat, double dx, double dt,
                                  double* W, hipStream_t s);

// ---- current surrogate (k_nn.hip) ------------------------------------------
struct NNShape {
  int W, H;
};
struct NNWork {  // per-batch activations and gradients, FP32
  float *h1, *h2, *y, *dy, *dz2, *dz1, *loss;
};
hipError_t nn_forward(const NNShape& sh, const float* theta, const float* X, int B, NNWork& wk, hipStream_t s);
hipError_t nn_backward(const NNShape& sh, const float* theta, const float* X, const float* target, int B,
                       NNWork& wk, float* grad, hipStream_t s);
hipError_t nn_adam(float* theta, float* m, float* v, const float* g, long n, float lr, float b1, float b2,
                   float eps, float c1, float c2, hipStream_t s);
hipError_t nn_gather(const float* seqA, const float* seqJ, int T, int W, const int* idx, int B, float* X,
                     float* target, hipStream_t s);
hipError_t nn_accumulate(const float* src, float* dst, hipStream_t s);
// least squares of the skip weights ws [W] and output bias b3 over trajectories
// A, Y [n_traj][T] (scaled, FP64); G [(W+1)^2] and b [W+1] are work arrays
hipError_t nn_fit_linear(const double* A, const double* Y, int n_traj, int T, int W, double lambda_rel, double* G,
                         double* b, float* ws, float* b3, int* ok, hipStream_t s);
hipError_t nn_zero(float* p, long n, hipStream_t s);

}  // namespace td
