// C ABI of the TDKS time step (declared in include/tddft.h).
//
// One step, enqueued on the context's stream and captured once as a hipGraph:
//   1. per-step parameters: kappa_k, sphere phases, length-gauge field (from
//      the A table indexed by a device step counter);
//   2. four Horner stages s = 4, 3, 2, 1, each preceded (when projectors are
//      present) by the MFMA projection of its input for the nonlocal add-back;
//   3. observables of the new orbitals (norms, momentum, kinetic and local
//      energy sums) and the moment projections for the nonlocal current;
//   4. density (two fixed-order passes), Hartree by FFT, LDA, new V;
//   5. current reduction into the device J table, counter + 1.
// The potential stays frozen at rho(t_n) during a step.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/tddft.h"
#include "internal.h"

using namespace td;

namespace {

const double kFdC[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};
const double kFdD[4] = {4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0};

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct tddft_ctx {
  tddft_config cfg{};
  std::vector<double> kpt, kw;
  std::string err;
  bool poisoned = false;
  bool potential_set = false;
  bool own_stream = false;
  hipStream_t stream = nullptr;
  int device = 0;

  Geometry g{};               // observe pass and shared sizes
  int bc = kPeriodicPlane;
  Geometry gs{};              // decomposition of the per-stage kernel (tuned)
  int sbc = kPeriodicPlane;
  std::string tune_note;      // JSON of the tuner's choice and measurements
  std::string tune_choice;    // the same without the candidate list
  size_t N = 0, n_orb_tot = 0;
  bool mixed = false;
  double dV = 0, volume = 0;
  double lap[3][5]{}, dh[3][4]{}, cdiag = 0;

  std::vector<DevBuf> owned;
  void *W = nullptr, *U0 = nullptr, *U1 = nullptr;
  double *Vd = nullptr, *Vloc = nullptr, *vh = nullptr, *exc = nullptr, *rho = nullptr, *rho0 = nullptr;
  float* Vf = nullptr;
  double* rho_part = nullptr;
  int rho_chunk = 64, rho_nchunks = 0;
  // BJ / TB09 exchange: kinetic energy density, its chunk partials, v_x,
  // per-block sums of |grad rho| / rho and (c, g)
  double *tau = nullptr, *tau_part = nullptr, *vx_mgga = nullptr, *gpart = nullptr, *cval = nullptr;
  double2* fft = nullptr;
  double* Kfft = nullptr;
  int M[3] = {0, 0, 0};
  double vh_scale = 0;
  double *kpt_d = nullptr, *kw_d = nullptr;

  // nonlocal
  NLTables nl{};
  double* ent_x = nullptr;
  double* ent_beta = nullptr;  // [S][4]
  int n_colors = 0;
  int *color_start = nullptr, *color_atoms = nullptr;
  std::vector<int> color_ent_start;  // host: entries of colour c are color_ents[start[c] .. start[c+1])
  int* color_ents = nullptr;         // [S] entry ids grouped by colour
  bool fused = false;          // whole step per orbital in LDS
  double2* Eu = nullptr;
  double2* Eu2 = nullptr;      // second E_p u_p buffer: stages alternate when the add-back rides in the projection
  double* jnl = nullptr;
  double nl_bound = 0;
  double vabs = 0;
  int max_overlap = 0;

  // per step
  double *kappa = nullptr, *kappaJ = nullptr, *efield = nullptr, *Alast = nullptr;
  double* coef = nullptr;  // [n_k][kCoef] in the stage precision (fused step)
  double2* phkA = nullptr;  // [n_k][S] combined projector phases of the step (fused step)
  double2* gram = nullptr;  // [2][n_k][n_orb][n_orb] overlap and its inverse factor (ground state)
  int* chol_bad = nullptr;  // set by the device Cholesky when a pivot is not positive
  void* Wsave = nullptr;    // predictor-corrector: the orbitals at t_n
  void* Wref = nullptr;     // reference (ground-state) orbitals for the excited-pair count
  double* Sk = nullptr;     // [n_k] occupied weight kept in the reference space
  double E_ref = 0.0;       // energy of the reference state (excitation energy)
  bool have_E_ref = false;
  double* Vsave = nullptr;  // predictor-corrector: V(t_n)
  double2 *phA = nullptr, *phAJ = nullptr;
  double* obs = nullptr;
  double *Atab = nullptr, *Jtab = nullptr;
  int cap_steps = 0;
  double* Aobs = nullptr;  // [2][3] for observation calls
  int *counter = nullptr, *nanflag = nullptr;
  double *scalars = nullptr, *sums = nullptr;
  double A_last[3] = {0, 0, 0};
  // per-axis largest |A| of the last table that passed the stability bound
  // (the bound grows with each; -1: none since the potential was set)
  double bound_amax[3] = {-1.0, -1.0, -1.0};

  hipGraphExec_t graph = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double last_ms = 0;
};

namespace {

tddft_status fail(tddft_ctx* c, tddft_status st, const std::string& msg) {
  if (c) {
    c->err = msg;
    if (st == TDDFT_EDEVICE || st == TDDFT_ENUMERIC) c->poisoned = true;
  }
  return st;
}

#define HIP_TRY(expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return fail(c, TDDFT_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));        \
  } while (0)

tddft_status dalloc(tddft_ctx* c, size_t bytes, void** out) {
  *out = nullptr;
  if (bytes == 0) bytes = 16;
  void* p = nullptr;
  if (c->cfg.dev_alloc) {
    p = c->cfg.dev_alloc(bytes, c->cfg.alloc_user);
    if (!p) return fail(c, TDDFT_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  } else {
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(c, TDDFT_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
  }
  c->owned.push_back({p, bytes});
  *out = p;
  return TDDFT_OK;
}

template <typename P>
tddft_status dalloc_t(tddft_ctx* c, size_t count, P** out) {
  void* p = nullptr;
  tddft_status st = dalloc(c, count * sizeof(P), &p);
  *out = static_cast<P*>(p);
  return st;
}

void dfree_all(tddft_ctx* c) {
  for (auto& b : c->owned) {
    if (c->cfg.dev_free)
      c->cfg.dev_free(b.p, c->cfg.alloc_user);
    else
      (void)hipFree(b.p);
  }
  c->owned.clear();
}

bool debug_sync(const tddft_ctx* c) { return (c->cfg.flags & TDDFT_FLAG_DEBUG_SYNC) != 0; }

tddft_status check_launch(tddft_ctx* c, hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(c, TDDFT_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  if (debug_sync(c)) {
    hipError_t s = hipStreamSynchronize(c->stream);
    if (s != hipSuccess) return fail(c, TDDFT_EDEVICE, std::string(what) + " (sync): " + hipGetErrorString(s));
  }
  return TDDFT_OK;
}

#define LAUNCH(expr, what)                                   \
  do {                                                       \
    tddft_status st_ = check_launch(c, (expr), what);        \
    if (st_ != TDDFT_OK) return st_;                         \
  } while (0)

// Largest divisor of n that is <= cap and >= 4 (or n itself when n <= cap).
int tile_dim(int n, int cap) {
  if (n <= cap) return n;
  for (int d = cap; d >= 4; --d)
    if (n % d == 0) return d;
  return -1;
}

bool fft_size_ok(int m) {
  for (int r : {2, 3, 5})
    while (m % r == 0) m /= r;
  return m == 1;
}

// Gauss-Legendre nodes and weights on [0, 1].
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    double dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = 0.5 * (1.0 - z);
    w[i] = 1.0 / ((1.0 - z * z) * dp * dp) * 2.0 * 0.5;
  }
}

// Mean of 1/|r| over the cell [-h1/2, h1/2] x ... : split the positive octant
// box into three pyramids with apex at the origin; in each, r = t (1, s, u)
// turns the singular integrand into the smooth 1 / sqrt(1 + s^2 + u^2).
double self_cell_inverse_r(double h1, double h2, double h3) {
  std::vector<double> x, w;
  gauss_legendre(48, x, w);
  const double a[3] = {0.5 * h1, 0.5 * h2, 0.5 * h3};
  double tot = 0.0;
  for (int ax = 0; ax < 3; ++ax) {
    const double p = a[ax], q = a[(ax + 1) % 3], r = a[(ax + 2) % 3];
    const double S = q / p, U = r / p;
    double I = 0.0;
    for (int i = 0; i < 48; ++i)
      for (int j = 0; j < 48; ++j) {
        const double s = S * x[i], u = U * x[j];
        I += w[i] * w[j] / std::sqrt(1.0 + s * s + u * u);
      }
    tot += 0.5 * p * p * I * S * U;
  }
  return 8.0 * tot / (h1 * h2 * h3);
}

template <typename T>
typename Vec2<T>::type* as2(void* p) {
  return static_cast<typename Vec2<T>::type*>(p);
}

// ---------------------------------------------------------------------------
// enqueue helpers

MggaArgs mgga_args(const tddft_ctx* c) {
  MggaArgs a{};
  a.g = c->g;
  std::memcpy(a.d1, c->dh, sizeof(a.d1));
  for (int mu = 0; mu < 3; ++mu)
    for (int m = 0; m < 5; ++m) a.d2[mu][m] = -2.0 * c->lap[mu][m];
  return a;
}

bool is_mgga(const tddft_ctx* c) { return c->cfg.xc == TDDFT_XC_TB09 || c->cfg.xc == TDDFT_XC_BJ; }

template <typename T>
tddft_status enqueue_density_potential(tddft_ctx* c) {
  const int N = (int)c->N;
  const bool mgga = is_mgga(c);
  // with a single chunk of orbitals the partial sums are the sums: write them
  // in place and skip the reduction (0 + x = x, the same bits)
  const bool one = c->rho_nchunks == 1;
  if (mgga) {
    // rho and the kinetic energy density with kappa at the orbitals' time
    LAUNCH(launch_rho_tau_partial<T>(as2<T>(c->W), c->kw_d, c->kappaJ, mgga_args(c), c->rho_chunk,
                                     one ? c->rho : c->rho_part, one ? c->tau : c->tau_part, c->stream),
           "rho_tau_partial");
    if (!one) LAUNCH(launch_rho_reduce(c->tau_part, c->rho_nchunks, N, c->tau, c->stream), "tau_reduce");
  } else {
    LAUNCH(launch_rho_partial<T>(as2<T>(c->W), c->kw_d, c->cfg.n_orb, c->cfg.n_k, N, c->rho_chunk,
                                 one ? c->rho : c->rho_part, c->stream),
           "rho_partial");
  }
  if (!one) LAUNCH(launch_rho_reduce(c->rho_part, c->rho_nchunks, N, c->rho, c->stream), "rho_reduce");
  if (!c->potential_set) return TDDFT_OK;
  if (c->cfg.hartree) {
    // rho fills the corner n1 x n2 x n3 of the M-box (all of it for a
    // periodic cell) and only that corner of the potential is read back, so
    // each pass transforms only the lines that hold data or are needed:
    // forward x over y < n2, z < n3 (packing rho into the box), forward y
    // over z < n3 (zero beyond y = n2), then along z the forward transform,
    // the kernel K and the inverse in one pass, storing z < n3, inverse y over
    // z < n3 storing y < n2, inverse x over y < n2, z < n3 storing x < n1
    const int M1 = c->M[0], M2 = c->M[1], M3 = c->M[2];
    const int n1 = c->g.n1, n2 = c->g.n2, n3 = c->g.n3;
    LAUNCH(launch_fft_lines(c->fft, M1, M2, M3, 0, -1, c->stream, c->rho, n1, n2, n3, nullptr, n2, n3, n1, M1, 0),
           "fft x");
    LAUNCH(launch_fft_lines(c->fft, M1, M2, M3, 1, -1, c->stream, nullptr, 0, 0, 0, nullptr, M1, n3, n2, M2, 0),
           "fft y");
    LAUNCH(launch_fft_lines(c->fft, M1, M2, M3, 2, -1, c->stream, nullptr, 0, 0, 0, c->Kfft, M1, M2, n3, n3, 1),
           "fft z, kernel, inverse z");
    LAUNCH(launch_fft_lines(c->fft, M1, M2, M3, 1, +1, c->stream, nullptr, 0, 0, 0, nullptr, M1, n3, M2, n2, 0),
           "inverse fft y");
    LAUNCH(launch_fft_lines(c->fft, M1, M2, M3, 0, +1, c->stream, nullptr, 0, 0, 0, nullptr, n2, n3, M1, n1, 0),
           "inverse fft x");
  }
  if (mgga)
    LAUNCH(launch_mgga_potential(c->rho, c->tau, mgga_args(c), c->cfg.xc == TDDFT_XC_TB09, c->dV, c->volume,
                                 c->gpart, c->cval, c->vx_mgga, c->stream),
           "mgga exchange");
  LAUNCH(launch_xc_assemble(c->fft, c->g.n1, c->g.n2, c->g.n3, c->M[0], c->M[1], c->M[2], c->vh_scale,
                            c->rho, c->Vloc, c->cfg.hartree, c->cfg.xc, c->vx_mgga, c->Vd, c->Vf, c->vh,
                            c->exc, c->stream),
         "xc_assemble");
  return TDDFT_OK;
}

template <typename T>
StageArgs<T> stage_args(tddft_ctx* c) {
  StageArgs<T> a{};
  a.V = nullptr;
  a.kappa = c->kappa;
  a.efield = (c->cfg.gauge == TDDFT_LENGTH) ? c->efield : nullptr;
  a.Eu = c->nl.n_atoms > 0 ? c->Eu : nullptr;
  a.phA = c->phA;
  a.nl = c->nl;
  a.g = c->gs;
  std::memcpy(a.lap, c->lap, sizeof(a.lap));
  std::memcpy(a.dh, c->dh, sizeof(a.dh));
  a.cdiag = c->cdiag;
  a.coef = reinterpret_cast<const T*>(c->coef);
  for (int mu = 0; mu < 3; ++mu)
    for (int m = 0; m < 4; ++m) a.lapc[mu][m] = (T)c->lap[mu][m + 1];
  return a;
}

template <typename T>
const T* vpot(tddft_ctx* c);
template <>
const double* vpot<double>(tddft_ctx* c) {
  return c->Vd;
}
template <>
const float* vpot<float>(tddft_ctx* c) {
  return c->Vf;
}

// tolerance of the norm watchdog (0: off)
double norm_tol(const tddft_ctx* c) { return (c->cfg.flags & TDDFT_FLAG_NORM_WATCHDOG) ? 1e-3 : 0.0; }

// observables of W with kappaJ / phAJ already set: obs, jnl, then finish
template <typename T>
tddft_status enqueue_observe(tddft_ctx* c, int bump) {
  ObserveArgs<T> oa{};
  oa.w = as2<T>(c->W);
  oa.Vloc = c->Vloc;
  oa.g = c->g;
  std::memcpy(oa.dh, c->dh, sizeof(oa.dh));
  std::memcpy(oa.lap, c->lap, sizeof(oa.lap));
  oa.set_weights();
  oa.cdiag = c->cdiag;
  oa.out = c->obs;
  oa.energy = bump ? 0 : 1;  // a step records the current; the energy is read on demand
  LAUNCH(launch_observe<T>(c->bc, oa, c->stream), "observe");
  const bool nl = c->nl.n_atoms > 0;
  if (nl) {
    ProjArgs<T> pa{};
    pa.u = as2<T>(c->W);
    pa.phA = c->phAJ;
    pa.nl = c->nl;
    pa.N = (int)c->N;
    pa.n_orb = c->cfg.n_orb;
    pa.n_orb_tot = (int)c->n_orb_tot;
    pa.dV = c->dV;
    pa.moments = 1;
    pa.Eu = c->Eu;
    pa.jnl = c->jnl;
    LAUNCH(launch_project<T>(pa, c->stream), "project moments");
  }
  LAUNCH(launch_finish(c->obs, c->g.tiles_x * c->g.tiles_y * c->g.zslabs, c->jnl, nl ? 1 : 0, c->kw_d, c->kappaJ,
                       c->cfg.n_orb, c->cfg.n_k, c->dV, c->volume, c->counter, bump, c->Jtab, c->scalars,
                       c->nanflag, norm_tol(c), c->stream),
         "finish");
  return TDDFT_OK;
}

template <typename T>
FusedArgs<T> fused_args(tddft_ctx* c);

// stencil coefficients of the step from the kappa just set (and, for the
// fused step, the combined projector phases)
tddft_status enqueue_coef(tddft_ctx* c) {
  if (!c->fused) {
    if (c->mixed)
      LAUNCH(launch_coef_table<float>(c->kappa, c->cfg.n_k, c->dh, c->cdiag, reinterpret_cast<float*>(c->coef),
                                      c->stream),
             "stage coefficients");
    else
      LAUNCH(launch_coef_table<double>(c->kappa, c->cfg.n_k, c->dh, c->cdiag, c->coef, c->stream),
             "stage coefficients");
    return TDDFT_OK;
  }
  if (c->mixed)
    LAUNCH(launch_fused_coef<float>(fused_args<float>(c), c->stream), "fused coefficients");
  else
    LAUNCH(launch_fused_coef<double>(fused_args<double>(c), c->stream), "fused coefficients");
  return TDDFT_OK;
}

tddft_status enqueue_params(tddft_ctx* c) {
  LAUNCH(launch_step_params(c->Atab, c->counter, 1, c->kpt_d, c->cfg.n_k, c->ent_x, c->nl.n_ent,
                            c->cfg.gauge, c->cfg.dt, c->kappa, c->kappaJ, c->efield, c->phA, c->phAJ,
                            c->Alast, c->stream),
         "step_params");
  return enqueue_coef(c);
}

template <typename T>
FusedArgs<T> fused_args(tddft_ctx* c) {
  FusedArgs<T> f{};
  f.w = as2<T>(c->W);
  f.V = vpot<T>(c);
  f.Vloc = c->Vloc;
  f.kappa = c->kappa;
  f.phA = c->phA;
  f.phAJ = c->phAJ;
  f.efield = (c->cfg.gauge == TDDFT_LENGTH) ? c->efield : nullptr;
  f.nl = c->nl;
  f.ent_beta = c->ent_beta;
  f.ent_x = c->ent_x;
  f.n_colors = c->n_colors;
  f.color_start = c->color_start;
  f.color_atoms = c->color_atoms;
  f.g = c->g;
  std::memcpy(f.lap, c->lap, sizeof(f.lap));
  std::memcpy(f.dh, c->dh, sizeof(f.dh));
  f.cdiag = c->cdiag;
  f.dt = c->cfg.dt;
  f.dV = c->dV;
  f.obs = c->obs;
  f.jnl = c->jnl;
  f.coef = reinterpret_cast<T*>(c->coef);
  f.phkA = c->phkA;
  for (int mu = 0; mu < 3; ++mu)
    for (int m = 0; m < 4; ++m) {
      f.lapc[mu][m] = (T)c->lap[mu][m + 1];
      f.dhc[mu][m] = (T)c->dh[mu][m];
    }
  return f;
}

// after the fused orbital update: current, density and the new potential
template <typename T>
tddft_status enqueue_fused_tail(tddft_ctx* c) {
  LAUNCH(launch_finish(c->obs, 1, c->jnl, c->nl.n_atoms > 0 ? 1 : 0, c->kw_d, c->kappaJ, c->cfg.n_orb,
                       c->cfg.n_k, c->dV, c->volume, c->counter, 1, c->Jtab, c->scalars, c->nanflag,
                       norm_tol(c), c->stream),
         "finish");
  return enqueue_density_potential<T>(c);
}

// one kernel per Horner stage, then observables, current, density, potential
// the four Horner stages with per-stage projections, W <- sum_m (x h)^m / m! W
// with x = -i dt (real time, Eq. 2) or x = -tau (imaginary time)
template <typename T>
tddft_status enqueue_taylor_stages(tddft_ctx* c, double dt, double tau_imag) {
  StageArgs<T> a = stage_args<T>(c);
  a.V = vpot<T>(c);
  void* bufs_in[4] = {c->W, c->U0, c->U1, c->U0};
  void* bufs_out[4] = {c->U0, c->U1, c->U0, c->W};
  // With disjoint spheres (one colour) the nonlocal term of stages 4, 3 and 2
  // is added by the next stage's projection, at the sphere points it gathers
  // anyway (same arithmetic, so the same bits as the add-back kernel); E_p u_p
  // then alternates between two buffers. The last stage keeps the add-back
  // kernel: its output goes to the observables.
  const bool nl = c->nl.n_atoms > 0;
  const bool ride = nl && c->n_colors == 1;
  double2* eu_buf[2] = {c->Eu, ride ? c->Eu2 : c->Eu};
  for (int i = 0; i < 4; ++i) {
    const int s = 4 - i;
    if (nl) {
      ProjArgs<T> pa{};
      pa.u = as2<T>(bufs_in[i]);
      pa.phA = c->phA;
      pa.nl = c->nl;
      pa.N = (int)c->N;
      pa.n_orb = c->cfg.n_orb;
      pa.n_orb_tot = (int)c->n_orb_tot;
      pa.dV = c->dV;
      pa.moments = 0;
      pa.Eu = eu_buf[i & 1];
      pa.jnl = c->jnl;
      if (ride && i > 0) {
        // u_s came from stage s + 1, whose projections are in the other buffer
        pa.Eu_prev = eu_buf[(i - 1) & 1];
        pa.ent_beta = c->ent_beta;
        pa.tau = dt / (s + 1);
        pa.tau_re = -tau_imag / (s + 1);
      }
      LAUNCH(launch_project<T>(pa, c->stream), "project");
    }
    a.in = as2<T>(bufs_in[i]);
    a.w = as2<T>(c->W);
    a.out = as2<T>(bufs_out[i]);
    a.tau = dt / s;  // u_{s-1} = w + (x / s) h u_s
    a.tau_re = -tau_imag / s;
    a.Eu = nl ? eu_buf[i & 1] : nullptr;
    const int mode = (s == 4) ? kFirst : (s == 1 ? kLast : kMid);
    LAUNCH(launch_stage<T>(mode, c->sbc, a, c->stream), "stage");
    // the nonlocal term of the stage, added over each colour's sphere entries
    if (ride && s > 1) continue;
    for (int cl = 0; cl < c->n_colors && nl; ++cl) {
      const int e0 = c->color_ent_start[cl], ne = c->color_ent_start[cl + 1] - e0;
      LAUNCH(launch_nl_addback<T>(a, c->color_ents + e0, ne, (int)c->n_orb_tot, c->stream), "nonlocal add-back");
    }
  }
  return TDDFT_OK;
}

template <typename T>
tddft_status enqueue_streaming_update(tddft_ctx* c) {
  tddft_status st = enqueue_taylor_stages<T>(c, c->cfg.dt, 0.0);
  if (st != TDDFT_OK) return st;
  st = enqueue_observe<T>(c, 1);
  if (st != TDDFT_OK) return st;
  return enqueue_density_potential<T>(c);
}

template <typename T>
tddft_status enqueue_step(tddft_ctx* c) {
  tddft_status st = enqueue_params(c);
  if (st != TDDFT_OK) return st;
  if (c->cfg.flags & TDDFT_FLAG_PREDICTOR_CORRECTOR) {
    // predictor: the step under V(t_n), then rho and V at t_{n+1}; the
    // corrector below restarts from the saved orbitals under the mean potential
    const size_t wbytes = c->n_orb_tot * c->N * sizeof(typename Vec2<T>::type);
    LAUNCH(launch_copy8(c->W, c->Wsave, wbytes, c->stream), "save orbitals");
    LAUNCH(launch_copy8(c->Vd, c->Vsave, c->N * sizeof(double), c->stream), "save potential");
    if (c->fused) {
      LAUNCH(launch_fused<T>(fused_args<T>(c), c->stream), "fused step (predictor)");
    } else {
      st = enqueue_taylor_stages<T>(c, c->cfg.dt, 0.0);
      if (st != TDDFT_OK) return st;
    }
    st = enqueue_density_potential<T>(c);
    if (st != TDDFT_OK) return st;
    LAUNCH(launch_mid_potential(c->Vsave, c->Vd, c->Vf, c->N, c->stream), "mid potential");
    LAUNCH(launch_copy8(c->Wsave, c->W, wbytes, c->stream), "restore orbitals");
  }
  if (c->fused) {
    LAUNCH(launch_fused<T>(fused_args<T>(c), c->stream), "fused step");
    return enqueue_fused_tail<T>(c);
  }
  return enqueue_streaming_update<T>(c);
}

tddft_status step_dispatch(tddft_ctx* c) { return c->mixed ? enqueue_step<float>(c) : enqueue_step<double>(c); }
tddft_status observe_dispatch(tddft_ctx* c) {
  return c->mixed ? enqueue_observe<float>(c, 0) : enqueue_observe<double>(c, 0);
}
tddft_status potential_dispatch(tddft_ctx* c) {
  return c->mixed ? enqueue_density_potential<float>(c) : enqueue_density_potential<double>(c);
}

// observation at the current time with the last A: set kappaJ/phAJ, run observe
tddft_status observe_now(tddft_ctx* c) {
  double Ab[6];
  for (int i = 0; i < 3; ++i) Ab[i] = Ab[3 + i] = c->A_last[i];
  HIP_TRY(hipMemcpyAsync(c->Aobs, Ab, sizeof(Ab), hipMemcpyHostToDevice, c->stream));
  LAUNCH(launch_step_params(c->Aobs, c->counter, 0, c->kpt_d, c->cfg.n_k, c->ent_x, c->nl.n_ent,
                            c->cfg.gauge, c->cfg.dt, c->kappa, c->kappaJ, c->efield, c->phA, c->phAJ,
                            c->Alast, c->stream),
         "step_params");
  tddft_status st = observe_dispatch(c);
  if (st != TDDFT_OK) return st;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return TDDFT_OK;
}

void invalidate_graph(tddft_ctx* c) {
  if (c->graph) {
    (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
  }
}

tddft_status upload_orbitals(tddft_ctx* c, const double* psi) {
  const size_t total = c->n_orb_tot * c->N;
  // stage through U0 (which is at least total * sizeof(T2)); for c128 copy straight into W
  if (!c->mixed) {
    HIP_TRY(hipMemcpyAsync(c->W, psi, total * sizeof(double2), hipMemcpyHostToDevice, c->stream));
  } else {
    // U0 and U1 together hold total double2 (each holds total float2)
    HIP_TRY(hipMemcpyAsync(c->U0, psi, total * sizeof(double2), hipMemcpyHostToDevice, c->stream));
    LAUNCH(launch_convert_in<float>(static_cast<const double2*>(c->U0), as2<float>(c->W), total, c->stream),
           "convert_in");
  }
  return TDDFT_OK;
}

// Upper bound of |lambda(h)| for the stability checks. The kinetic part
// (1/2)(-i grad + kappa)^2, kappa = k + A/c, is a sum over the axes of commuting
// one-axis operators whose symbol is f_i(theta) = K2(theta)/(2 h_i^2) +
// kappa_i K1(theta)/h_i + kappa_i^2/2, with K2(theta) = -c0 - 2 sum c_m cos(m theta)
// >= 0 and K1(theta) = 2 sum d_m sin(m theta) the symbols of the eighth-order
// second and first differences that discretise the kinetic term of Eq.
// TDKS_solid. On a periodic grid the one-axis eigenvalues are values of f_i,
// with zero boundaries they lie between its extremes (Hermitian Toeplitz), so |lambda_kin| <= sum_i max_theta |f_i| <=
// sum_i [max_theta (K2/(2 h_i^2) + |kappa_i| |K1|/h_i) + kappa_i^2/2]. The
// maximum is taken over the Bloch vectors of the context and, per axis, the
// largest |A_i| of the table (amax); it is sampled on a grid of theta and raised
// by the Lipschitz constant times half the grid spacing, so it stays an upper
// bound. The potential and the nonlocal term add |V|_max and the nonlocal norm
// bound.
const double kNoField[3] = {0.0, 0.0, 0.0};

double spectral_bound(const tddft_ctx* c, const double amax[3], double vmin, double vmax) {
  constexpr int kTheta = 4096;
  static const std::vector<double> k2tab = [] {
    std::vector<double> t(kTheta + 1);
    for (int j = 0; j <= kTheta; ++j) {
      const double th = M_PI * j / kTheta;
      double v = -kFdC[0];
      for (int m = 1; m <= 4; ++m) v -= 2.0 * kFdC[m] * std::cos(m * th);
      t[j] = v;
    }
    return t;
  }();
  static const std::vector<double> k1tab = [] {
    std::vector<double> t(kTheta + 1);
    for (int j = 0; j <= kTheta; ++j) {
      const double th = M_PI * j / kTheta;
      double v = 0.0;
      for (int m = 1; m <= 4; ++m) v += 2.0 * kFdD[m - 1] * std::sin(m * th);
      t[j] = std::fabs(v);
    }
    return t;
  }();
  double lip2 = 0.0, lip1 = 0.0;  // Lipschitz constants of K2 and |K1| in theta
  for (int m = 1; m <= 4; ++m) {
    lip2 += 2.0 * m * std::fabs(kFdC[m]);
    lip1 += 2.0 * m * std::fabs(kFdD[m - 1]);
  }
  const double h[3] = {c->g.h1, c->g.h2, c->g.h3};
  double lam = 0.0;
  for (int i = 0; i < 3; ++i) {
    double kap = 0.0;
    for (int k = 0; k < c->cfg.n_k; ++k) kap = std::max(kap, std::fabs(c->kpt[3 * k + i]) + amax[i] / kC);
    const double a2 = 0.5 / (h[i] * h[i]), a1 = kap / h[i];
    double g = 0.0;
    for (int j = 0; j <= kTheta; ++j) g = std::max(g, a2 * k2tab[j] + a1 * k1tab[j]);
    lam += g + (a2 * lip2 + a1 * lip1) * (0.5 * M_PI / kTheta) + 0.5 * kap * kap;
  }
  const double vabs = std::max(std::fabs(vmin), std::fabs(vmax));
  return lam + vabs + c->nl_bound;
}

template <typename T>
tddft_status launch_one(tddft_ctx* c, int which) {
  if (which == TDDFT_KERNEL_STAGE) {
    StageArgs<T> a = stage_args<T>(c);
    a.V = vpot<T>(c);
    a.in = as2<T>(c->U0);
    a.w = as2<T>(c->W);
    a.out = as2<T>(c->U1);
    a.tau = c->cfg.dt / 2;
    LAUNCH(launch_stage<T>(kMid, c->sbc, a, c->stream), "stage");
    for (int cl = 0; cl < c->n_colors && c->nl.n_atoms > 0; ++cl) {
      const int e0 = c->color_ent_start[cl], ne = c->color_ent_start[cl + 1] - e0;
      LAUNCH(launch_nl_addback<T>(a, c->color_ents + e0, ne, (int)c->n_orb_tot, c->stream), "nonlocal add-back");
    }
  } else if (which == TDDFT_KERNEL_PROJECT) {
    if (c->nl.n_atoms == 0) return TDDFT_OK;
    ProjArgs<T> pa{};
    pa.u = as2<T>(c->U0);
    pa.phA = c->phA;
    pa.nl = c->nl;
    pa.N = (int)c->N;
    pa.n_orb = c->cfg.n_orb;
    pa.n_orb_tot = (int)c->n_orb_tot;
    pa.dV = c->dV;
    pa.moments = 0;
    pa.Eu = c->Eu;
    pa.jnl = c->jnl;
    LAUNCH(launch_project<T>(pa, c->stream), "project");
  } else if (which == TDDFT_KERNEL_OBSERVE) {
    ObserveArgs<T> oa{};
    oa.w = as2<T>(c->W);
    oa.Vloc = c->Vloc;
    oa.g = c->g;
    std::memcpy(oa.dh, c->dh, sizeof(oa.dh));
    std::memcpy(oa.lap, c->lap, sizeof(oa.lap));
    oa.set_weights();
    oa.cdiag = c->cdiag;
    oa.out = c->obs;
    oa.energy = 0;  // the variant each step runs
    LAUNCH(launch_observe<T>(c->bc, oa, c->stream), "observe");
  } else if (which == TDDFT_KERNEL_FUSED) {
    LAUNCH(launch_fused<T>(fused_args<T>(c), c->stream), "fused step");
  } else if (is_mgga(c)) {
    LAUNCH(launch_rho_tau_partial<T>(as2<T>(c->W), c->kw_d, c->kappaJ, mgga_args(c), c->rho_chunk, c->rho_part,
                                     c->tau_part, c->stream),
           "rho_tau_partial");
  } else {
    LAUNCH(launch_rho_partial<T>(as2<T>(c->W), c->kw_d, c->cfg.n_orb, c->cfg.n_k, (int)c->N, c->rho_chunk,
                                 c->rho_part, c->stream),
           "rho_partial");
  }
  return TDDFT_OK;
}

// ---------------------------------------------------------------------------
// Tuner of the per-stage kernel's decomposition: xy tile shape (or the whole
// periodic plane), z slabs and the XCD renumbering. Every candidate computes
// each output point with the same arithmetic in the same order, so the choice
// changes no bit of the result; the observe pass keeps its own decomposition,
// so the reductions of the current do not depend on it either. Each
// candidate's middle stage is timed on the two stage buffers (scratch
// between steps); the fastest is kept per (device, grid, boundary, orbital
// count, precision) in a process-wide table, and in the JSON file named by the
// environment variable TDDFT_TUNE_CACHE when it is set.

struct StagePlan {
  int bc, TX, TY, zs, xmap;
  double ms;
};

std::mutex g_tune_mu;
std::map<std::string, StagePlan> g_tune;
bool g_tune_file_read = false;

// the numbers that follow "name": after position pos (the file is our own)
bool json_num(const std::string& t, size_t pos, size_t end, const char* name, double* v) {
  const std::string pat = std::string("\"") + name + "\":";
  const size_t i = t.find(pat, pos);
  if (i == std::string::npos || i > end) return false;
  char* stop = nullptr;
  *v = std::strtod(t.c_str() + i + pat.size(), &stop);
  return stop != t.c_str() + i + pat.size();
}

void tune_file_read_locked() {
  if (g_tune_file_read) return;
  g_tune_file_read = true;
  const char* path = std::getenv("TDDFT_TUNE_CACHE");
  if (!path || !*path) return;
  std::ifstream f(path);
  if (!f) return;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string t = ss.str();
  size_t pos = 0;
  while ((pos = t.find("\"stage/", pos)) != std::string::npos) {
    const size_t kend = t.find('"', pos + 1);
    const size_t oend = t.find('}', kend);
    if (kend == std::string::npos || oend == std::string::npos) break;
    const std::string key = t.substr(pos + 1, kend - pos - 1);
    double v[6];
    const char* names[6] = {"bc", "TX", "TY", "zs", "xmap", "ms"};
    bool ok = true;
    for (int i = 0; i < 6 && ok; ++i) ok = json_num(t, kend, oend, names[i], &v[i]);
    if (ok) g_tune[key] = StagePlan{(int)v[0], (int)v[1], (int)v[2], (int)v[3], (int)v[4], v[5]};
    pos = oend;
  }
}

void tune_file_write_locked() {
  const char* path = std::getenv("TDDFT_TUNE_CACHE");
  if (!path || !*path) return;
  std::string tmp = std::string(path) + ".tmp";
  std::ofstream f(tmp);
  if (!f) return;
  f << "{\n";
  size_t i = 0;
  for (const auto& kv : g_tune) {
    const StagePlan& p = kv.second;
    char line[512];
    std::snprintf(line, sizeof line, "  \"%s\": {\"bc\": %d, \"TX\": %d, \"TY\": %d, \"zs\": %d, \"xmap\": %d, \"ms\": %.6f}%s\n",
                  kv.first.c_str(), p.bc, p.TX, p.TY, p.zs, p.xmap, p.ms, ++i < g_tune.size() ? "," : "");
    f << line;
  }
  f << "}\n";
  f.close();
  if (f) std::rename(tmp.c_str(), path);
}

std::string tune_key(const tddft_ctx* c) {
  hipDeviceProp_t prop{};
  std::string arch = "gpu";
  if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) {
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
  }
  char buf[160];
  std::snprintf(buf, sizeof buf, "stage/%s/%dx%dx%d/%s/%zu/%s", arch.c_str(), c->g.n1, c->g.n2, c->g.n3,
                c->g.periodic ? "periodic" : "isolated", c->n_orb_tot, c->mixed ? "c64" : "c128");
  return buf;
}

// a decomposition for (bc, TX, TY, zs, xmap), or false if it does not fit
bool make_stage_geometry(const tddft_ctx* c, const StagePlan& p, Geometry* out) {
  Geometry g = c->g;
  if (p.bc == kPeriodicPlane) {
    if (!g.periodic || g.n1 * g.n2 > 1024 || p.TX != g.n1 || p.TY != g.n2) return false;
  } else {
    if (p.bc != (g.periodic ? kPeriodicTile : kIsolatedTile)) return false;
    if (p.TX < 4 || p.TY < 4 || g.n1 % p.TX || g.n2 % p.TY || p.TX * p.TY > 1024 || !halo_fits(p.TX, p.TY))
      return false;
  }
  if (p.zs < 1 || p.zs > g.n3) return false;
  const int zlen = (g.n3 + p.zs - 1) / p.zs;
  if ((p.zs - 1) * zlen >= g.n3) return false;  // every slab non-empty
  g.TX = p.TX;
  g.TY = p.TY;
  g.tiles_x = g.n1 / p.TX;
  g.tiles_y = g.n2 / p.TY;
  g.zslabs = p.zs;
  g.xmap = p.xmap;
  *out = g;
  return true;
}

std::vector<StagePlan> stage_candidates(const tddft_ctx* c) {
  const Geometry& g = c->g;
  std::vector<StagePlan> out;
  const int tbc = g.periodic ? kPeriodicTile : kIsolatedTile;
  std::vector<std::pair<int, int>> tiles;
  if (g.periodic && g.n1 * g.n2 <= 1024) tiles.push_back({-1, -1});  // the whole plane
  for (int tx : {g.n1, 64, 48, 32, 24, 20, 16, 12, 10, 8})
    for (int ty : {32, 24, 20, 16, 12, 10, 8, 6, 5, 4}) {
      if (tx > g.n1 || ty > g.n2 || g.n1 % tx || g.n2 % ty || tx < 4 || ty < 4) continue;
      if (tx * ty < 128 || tx * ty > 1024) continue;
      if (std::find(tiles.begin(), tiles.end(), std::make_pair(tx, ty)) == tiles.end()) tiles.push_back({tx, ty});
    }
  for (const auto& t : tiles) {
    const bool plane = t.first < 0;
    const int tx = plane ? g.n1 : t.first, ty = plane ? g.n2 : t.second;
    const long per_z = (long)c->n_orb_tot * (g.n1 / tx) * (g.n2 / ty);
    for (int zs : {1, 2, 4}) {
      if (zs > 1 && (per_z * zs > 8192 || g.n3 / zs < 8)) continue;  // slabs only for few workgroups
      for (int xm : {0, 1}) {
        if (plane && xm) continue;  // no halo shared between the workgroups of a plane
        StagePlan p{plane ? kPeriodicPlane : tbc, tx, ty, zs, xm, 0.0};
        Geometry tmp;
        if (make_stage_geometry(c, p, &tmp)) out.push_back(p);
      }
    }
  }
  return out;
}

template <typename T>
tddft_status time_stage(tddft_ctx* c, const StagePlan& p, int reps, double* ms) {
  Geometry gs;
  if (!make_stage_geometry(c, p, &gs)) return fail(c, TDDFT_EINVAL, "bad stage decomposition");
  StageArgs<T> a = stage_args<T>(c);
  a.g = gs;
  a.V = vpot<T>(c);
  a.in = as2<T>(c->U0);
  a.w = as2<T>(c->W);
  a.out = as2<T>(c->U1);
  a.tau = c->cfg.dt / 2;
  LAUNCH(launch_stage<T>(kMid, p.bc, a, c->stream), "stage (tuner warm-up)");
  HIP_TRY(hipEventRecord(c->ev0, c->stream));
  for (int r = 0; r < reps; ++r) LAUNCH(launch_stage<T>(kMid, p.bc, a, c->stream), "stage (tuner)");
  HIP_TRY(hipEventRecord(c->ev1, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  float t = 0;
  HIP_TRY(hipEventElapsedTime(&t, c->ev0, c->ev1));
  *ms = t / reps;
  return TDDFT_OK;
}

std::string plan_json(const StagePlan& p) {
  char buf[160];
  std::snprintf(buf, sizeof buf, "{\"bc\": %d, \"TX\": %d, \"TY\": %d, \"zs\": %d, \"xmap\": %d, \"ms\": %.5f}",
                p.bc, p.TX, p.TY, p.zs, p.xmap, p.ms);
  return buf;
}

// choose gs / sbc for the per-stage path (after the potential is set)
tddft_status tune_stage(tddft_ctx* c) {
  const std::string key = tune_key(c);
  StagePlan best{c->bc, c->g.TX, c->g.TY, c->g.zslabs, c->g.xmap, 0.0};
  std::string source = "default";
  std::string cands = "[]";
  if (!(c->cfg.flags & TDDFT_FLAG_NO_TUNE)) {
    bool cached = false;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      tune_file_read_locked();
      auto it = g_tune.find(key);
      Geometry tmp;
      if (it != g_tune.end() && make_stage_geometry(c, it->second, &tmp)) {
        best = it->second;
        cached = true;
      }
    }
    if (cached) {
      source = "cache";
    } else {
      // coefficient tables of the current A, as for a real step
      double Ab[6];
      for (int i = 0; i < 3; ++i) Ab[i] = Ab[3 + i] = c->A_last[i];
      HIP_TRY(hipMemcpyAsync(c->Aobs, Ab, sizeof(Ab), hipMemcpyHostToDevice, c->stream));
      LAUNCH(launch_step_params(c->Aobs, c->counter, 0, c->kpt_d, c->cfg.n_k, c->ent_x, c->nl.n_ent, c->cfg.gauge,
                                c->cfg.dt, c->kappa, c->kappaJ, c->efield, c->phA, c->phAJ, c->Alast, c->stream),
             "step_params");
      tddft_status st = enqueue_coef(c);
      if (st != TDDFT_OK) return st;
      const std::vector<StagePlan> cand = stage_candidates(c);
      cands = "[";
      best.ms = 1e300;
      for (size_t i = 0; i < cand.size(); ++i) {
        StagePlan p = cand[i];
        st = c->mixed ? time_stage<float>(c, p, 3, &p.ms) : time_stage<double>(c, p, 3, &p.ms);
        if (st != TDDFT_OK) return st;
        cands += (i ? ", " : "") + plan_json(p);
        if (p.ms < best.ms) best = p;
      }
      cands += "]";
      source = "tuned";
      if (cand.empty()) best = StagePlan{c->bc, c->g.TX, c->g.TY, c->g.zslabs, c->g.xmap, 0.0};
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune[key] = best;
      tune_file_write_locked();
    }
  }
  Geometry gs;
  if (!make_stage_geometry(c, best, &gs)) {
    gs = c->g;
    best = StagePlan{c->bc, c->g.TX, c->g.TY, c->g.zslabs, c->g.xmap, 0.0};
  }
  c->gs = gs;
  c->sbc = best.bc;
  c->tune_choice = "{\"key\": \"" + key + "\", \"source\": \"" + source + "\", \"stage\": " + plan_json(best) + "}";
  c->tune_note = c->tune_choice.substr(0, c->tune_choice.size() - 1) + ", \"candidates\": " + cands + "}";
  return TDDFT_OK;
}

// validation, table upload and counter reset shared by single-cell and batch runs
// upload: copy the A table and reset the step counter here (a batch moves
// its cells' tables with one copy instead)
tddft_status prepare_propagate(tddft_ctx* c, int32_t nsteps, const double* A, bool upload = true) {
  if (c->poisoned) return fail(c, TDDFT_ESTATE, "context poisoned: " + c->err);
  if (!c->potential_set) return fail(c, TDDFT_ESTATE, "propagate before set_potential");
  if (nsteps < 1 || !A) return fail(c, TDDFT_EINVAL, "bad propagate arguments");
  double amax[3] = {0.0, 0.0, 0.0};
  for (size_t i = 0; i < 3 * (size_t)(nsteps + 1); ++i) {
    if (!std::isfinite(A[i])) return fail(c, TDDFT_EINVAL, "A table not finite");
    amax[i % 3] = std::max(amax[i % 3], std::fabs(A[i]));
  }
  // a table within the per-axis maxima of one that passed passes too (the
  // bound grows with each)
  const bool known = amax[0] <= c->bound_amax[0] && amax[1] <= c->bound_amax[1] && amax[2] <= c->bound_amax[2];
  if (c->cfg.gauge == TDDFT_VELOCITY && !(c->cfg.flags & TDDFT_FLAG_ALLOW_UNSTABLE) && !known) {
    // the potential part was checked in set_potential; recheck the kinetic part with |A|
    const double lam = spectral_bound(c, amax, -c->vabs, c->vabs);
    if (std::fabs(c->cfg.dt) * lam > 2.0 * std::sqrt(2.0)) {
      char buf[200];
      std::snprintf(buf, sizeof buf,
                    "unstable for this A table: |dt| * lambda_max = %.4g > 2 sqrt 2 (lambda_max <= %.6g Ha)",
                    std::fabs(c->cfg.dt) * lam, lam);
      return fail(c, TDDFT_EUNSTABLE, buf);
    }
    for (int i = 0; i < 3; ++i) c->bound_amax[i] = amax[i];
  }
  if (nsteps > c->cap_steps) {
    invalidate_graph(c);
    HIP_TRY(hipStreamSynchronize(c->stream));
    int cap = std::max(nsteps, 2 * c->cap_steps);
    tddft_status st;
    if ((st = dalloc_t(c, 3 * (size_t)(cap + 1), &c->Atab)) || (st = dalloc_t(c, 3 * (size_t)cap, &c->Jtab)))
      return st;
    c->cap_steps = cap;
  }
  if (upload) {
    HIP_TRY(hipMemcpyAsync(c->Atab, A, 3 * sizeof(double) * (nsteps + 1), hipMemcpyHostToDevice, c->stream));
    LAUNCH(launch_set_int(c->counter, 0, c->stream), "counter reset");
  }
  return TDDFT_OK;
}

// J table to the host, NaN check, remember the last A
tddft_status collect_propagate(tddft_ctx* c, int32_t nsteps, const double* A, double* J_out) {
  if (J_out)
    HIP_TRY(hipMemcpyAsync(J_out, c->Jtab, 3 * sizeof(double) * nsteps, hipMemcpyDeviceToHost, c->stream));
  int flag = 0;
  HIP_TRY(hipMemcpyAsync(&flag, c->nanflag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (int i = 0; i < 3; ++i) c->A_last[i] = A[3 * (size_t)nsteps + i];
  if (flag & 1) return fail(c, TDDFT_ENUMERIC, "NaN or Inf in the orbital norms or current");
  if (flag & 2)
    return fail(c, TDDFT_ENUMERIC, "norm watchdog: an orbital norm left 1 by more than 1e-3 (unstable step?)");
  return TDDFT_OK;
}

template <typename T>
tddft_status orthonormalise(tddft_ctx* c) {
  const int n = c->cfg.n_orb, nk = c->cfg.n_k, N = (int)c->N;
  double2* dS = c->gram;
  double2* dM = dS + (size_t)nk * n * n;
  for (int pass = 0; pass < 2; ++pass) {
    LAUNCH(launch_gram<T>(as2<T>(c->W), n, nk, N, c->dV, dS, c->stream), "gram");
    LAUNCH(launch_chol_inverse(dS, dM, n, nk, c->chol_bad, c->stream), "cholesky inverse");
    LAUNCH(launch_apply_lower<T>(as2<T>(c->W), dM, n, nk, N, as2<T>(c->U0), c->stream), "apply L^-1");
    HIP_TRY(hipMemcpyAsync(c->W, c->U0, c->n_orb_tot * c->N * sizeof(typename Vec2<T>::type),
                           hipMemcpyDeviceToDevice, c->stream));
  }
  return TDDFT_OK;
}

template <typename T>
tddft_status ground_state_iteration(tddft_ctx* c, double tau) {
  tddft_status st = enqueue_taylor_stages<T>(c, 0.0, tau);
  if (st != TDDFT_OK) return st;
  st = orthonormalise<T>(c);
  if (st != TDDFT_OK) return st;
  return enqueue_density_potential<T>(c);
}

}  // namespace

// ===========================================================================

extern "C" {

uint32_t tddft_abi_version(void) { return TDDFT_ABI_VERSION; }

const char* tddft_last_error(const tddft_ctx* ctx) { return ctx ? ctx->err.c_str() : stateless_error(); }

void tddft_free(tddft_ctx* ctx) {
  if (!ctx) return;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  invalidate_graph(ctx);
  if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
  if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
  dfree_all(ctx);
  if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

tddft_status tddft_init(const tddft_config* cfg, const double* psi0, tddft_ctx** out) {
  if (!out) return TDDFT_EINVAL;
  *out = nullptr;
  if (!cfg || !psi0) return TDDFT_EINVAL;
  if (cfg->abi_version != TDDFT_ABI_VERSION || cfg->struct_size != sizeof(tddft_config)) return TDDFT_EINVAL;
  auto* c = new tddft_ctx();
  c->cfg = *cfg;
  auto bad = [&](const std::string& m) {
    tddft_status st = fail(c, TDDFT_EINVAL, m);
    tddft_free(c);
    return st;
  };
  for (int i = 0; i < 3; ++i) {
    if (cfg->n[i] < 8) return bad("grid dimension below 8");
    if (!(cfg->cell[i] > 0)) return bad("cell length must be positive");
  }
  if (cfg->boundary != TDDFT_PERIODIC && cfg->boundary != TDDFT_ISOLATED) return bad("boundary");
  if (cfg->n_orb < 1 || cfg->n_k < 1) return bad("n_orb and n_k must be >= 1");
  if (!cfg->kpt || !cfg->kw) return bad("kpt and kw are required");
  if (!(cfg->dt != 0.0) || !std::isfinite(cfg->dt)) return bad("dt must be finite and nonzero");
  if (cfg->precision != TDDFT_C128 && cfg->precision != TDDFT_MIXED) return bad("precision");
  if (cfg->gauge != TDDFT_VELOCITY && cfg->gauge != TDDFT_LENGTH) return bad("gauge");
  if (cfg->gauge == TDDFT_LENGTH && cfg->boundary != TDDFT_ISOLATED)
    return bad("length gauge needs an isolated box");
  if (cfg->xc != TDDFT_XC_NONE && cfg->xc != TDDFT_XC_PZ81 && cfg->xc != TDDFT_XC_TB09 && cfg->xc != TDDFT_XC_BJ)
    return bad("xc");
  if ((cfg->dev_alloc == nullptr) != (cfg->dev_free == nullptr)) return bad("dev_alloc and dev_free go together");
  c->kpt.assign(cfg->kpt, cfg->kpt + 3 * cfg->n_k);
  c->kw.assign(cfg->kw, cfg->kw + cfg->n_k);
  double ws = 0;
  for (double v : c->kw) {
    if (!std::isfinite(v) || v < 0) return bad("k weights must be finite and >= 0");
    ws += v;
  }
  if (std::fabs(ws - 1.0) > 1e-10) return bad("k weights must sum to 1");
  for (double v : c->kpt)
    if (!std::isfinite(v)) return bad("k-points must be finite");
  c->cfg.kpt = nullptr;
  c->cfg.kw = nullptr;

  Geometry& g = c->g;
  g.n1 = cfg->n[0];
  g.n2 = cfg->n[1];
  g.n3 = cfg->n[2];
  g.h1 = cfg->cell[0] / g.n1;
  g.h2 = cfg->cell[1] / g.n2;
  g.h3 = cfg->cell[2] / g.n3;
  g.periodic = cfg->boundary == TDDFT_PERIODIC;
  g.n_orb = cfg->n_orb;
  g.n_k = cfg->n_k;
  c->N = (size_t)g.n1 * g.n2 * g.n3;
  if (c->N > (size_t)INT32_MAX / 2) return bad("grid too large");
  c->n_orb_tot = (size_t)cfg->n_orb * cfg->n_k;
  c->mixed = cfg->precision == TDDFT_MIXED;
  c->dV = g.h1 * g.h2 * g.h3;
  c->volume = cfg->cell[0] * cfg->cell[1] * cfg->cell[2];
  if (g.periodic && g.n1 * g.n2 <= 1024) {
    c->bc = kPeriodicPlane;
    g.TX = g.n1;
    g.TY = g.n2;
  } else {
    c->bc = g.periodic ? kPeriodicTile : kIsolatedTile;
    // 256-thread tiles (32 x 8 on wide grids): several workgroups per CU
    // interleave their per-plane barriers (measured 0.64 -> 0.46 ms per
    // complex FP32 stage on a 96^3 cell); taller tiles where n2 has no fitting
    // divisor
    g.TX = tile_dim(g.n1, 32);
    g.TY = g.TX > 0 ? tile_dim(g.n2, std::max(4, 256 / g.TX)) : -1;
    if (g.TX > 0 && g.TY < 4) g.TY = tile_dim(g.n2, std::max(4, 1024 / g.TX));
    if (g.TX < 4 || g.TY < 4 || g.TX * g.TY > 1024 || !halo_fits(g.TX, g.TY))
      return bad("no workgroup tiling for this grid");
  }
  g.tiles_x = g.n1 / g.TX;
  g.tiles_y = g.n2 / g.TY;
  // tiles of one orbital on one XCD share their halo rows in its L2
  g.xmap = c->bc == kPeriodicPlane ? 0 : 1;
  // per-stage kernels of cells with few orbitals: split z into slabs of at
  // least 8 planes until there are about a thousand workgroups
  g.zslabs = 1;
  while (g.zslabs < 8 && (long)c->n_orb_tot * g.tiles_x * g.tiles_y * g.zslabs < 1024 &&
         g.n3 / (2 * g.zslabs) >= 8)
    g.zslabs *= 2;
  c->gs = g;  // the per-stage kernel starts from the same decomposition
  c->sbc = c->bc;
  const double h[3] = {g.h1, g.h2, g.h3};
  c->cdiag = 0;
  for (int mu = 0; mu < 3; ++mu) {
    for (int m = 0; m < 5; ++m) c->lap[mu][m] = -0.5 * kFdC[m] / (h[mu] * h[mu]);
    for (int m = 0; m < 4; ++m) c->dh[mu][m] = kFdD[m] / h[mu];
    c->cdiag += c->lap[mu][0];
  }
  if (cfg->hartree) {
    for (int i = 0; i < 3; ++i) {
      c->M[i] = g.periodic ? cfg->n[i] : 2 * cfg->n[i];
      if (!fft_size_ok(c->M[i])) return bad("FFT sizes must have prime factors 2, 3, 5 only");
    }
  } else {
    c->M[0] = g.n1;
    c->M[1] = g.n2;
    c->M[2] = g.n3;
  }

  if (cfg->stream) {
    c->stream = static_cast<hipStream_t>(cfg->stream);
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      tddft_status st = fail(c, TDDFT_EDEVICE, "hipStreamCreate failed");
      tddft_free(c);
      return st;
    }
    c->own_stream = true;
  }
  (void)hipGetDevice(&c->device);
  auto cleanup = [&](tddft_status st) {
    std::string m = c->err;
    tddft_free(c);
    (void)m;
    return st;
  };
  tddft_status st = TDDFT_OK;
  const size_t esz = c->mixed ? sizeof(float2) : sizeof(double2);
  const size_t total = c->n_orb_tot * c->N;
  // the two stage buffers are contiguous so that a c128 upload can be staged through them
  void* u01 = nullptr;
  if ((st = dalloc(c, total * esz, &c->W)) != TDDFT_OK) return cleanup(st);
  if ((st = dalloc(c, 2 * total * esz, &u01)) != TDDFT_OK) return cleanup(st);
  c->U0 = u01;
  c->U1 = static_cast<char*>(u01) + total * esz;
  if ((cfg->flags & TDDFT_FLAG_PREDICTOR_CORRECTOR) && (st = dalloc(c, total * esz, &c->Wsave)) != TDDFT_OK)
    return cleanup(st);
  const size_t N = c->N;
  if ((st = dalloc_t(c, N, &c->Vd)) || (st = dalloc_t(c, N, &c->Vf)) || (st = dalloc_t(c, N, &c->Vloc)) ||
      (st = dalloc_t(c, N, &c->vh)) || (st = dalloc_t(c, N, &c->exc)) || (st = dalloc_t(c, N, &c->rho)) ||
      (st = dalloc_t(c, N, &c->rho0)))
    return cleanup(st);
  c->rho_chunk = is_mgga(c) ? rho_tau_chunk(c->g, (int)c->n_orb_tot) : 64;
  c->rho_nchunks = (int)((c->n_orb_tot + c->rho_chunk - 1) / c->rho_chunk);
  if ((st = dalloc_t(c, (size_t)c->rho_nchunks * N, &c->rho_part))) return cleanup(st);
  if (is_mgga(c) && ((st = dalloc_t(c, (size_t)c->rho_nchunks * N, &c->tau_part)) || (st = dalloc_t(c, N, &c->tau)) ||
                     (st = dalloc_t(c, N, &c->vx_mgga)) || (st = dalloc_t(c, (N + 255) / 256, &c->gpart)) ||
                     (st = dalloc_t(c, 2, &c->cval))))
    return cleanup(st);
  const size_t Mt = (size_t)c->M[0] * c->M[1] * c->M[2];
  if ((st = dalloc_t(c, Mt, &c->fft)) || (st = dalloc_t(c, Mt, &c->Kfft))) return cleanup(st);
  if ((st = dalloc_t(c, 3 * (size_t)cfg->n_k, &c->kpt_d)) || (st = dalloc_t(c, (size_t)cfg->n_k, &c->kw_d)) ||
      (st = dalloc_t(c, 3 * (size_t)cfg->n_k, &c->kappa)) || (st = dalloc_t(c, 3 * (size_t)cfg->n_k, &c->kappaJ)) ||
      (st = dalloc_t(c, (size_t)kCoef * cfg->n_k, &c->coef)) ||
      (st = dalloc_t(c, (cfg->flags & TDDFT_FLAG_PREDICTOR_CORRECTOR) ? N : 1, &c->Vsave)) ||
      (st = dalloc_t(c, 3, &c->efield)) || (st = dalloc_t(c, 3, &c->Alast)) || (st = dalloc_t(c, 6, &c->Aobs)) ||
      (st = dalloc_t(c, 1, &c->counter)) || (st = dalloc_t(c, 1, &c->nanflag)) ||
      (st = dalloc_t(c, 8, &c->scalars)) || (st = dalloc_t(c, 8, &c->sums)) ||
      (st = dalloc_t(c, c->n_orb_tot * g.tiles_x * g.tiles_y * g.zslabs * 8, &c->obs)) ||
      (st = dalloc_t(c, c->n_orb_tot * 4, &c->jnl)) || (st = dalloc_t(c, 1, &c->phA)) ||
      (st = dalloc_t(c, 1, &c->phAJ)) || (st = dalloc_t(c, 3, &c->ent_x)))
    return cleanup(st);
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess)
    return cleanup(fail(c, TDDFT_EDEVICE, "hipEventCreate failed"));
  if (hipMemcpyAsync(c->kpt_d, c->kpt.data(), 3 * sizeof(double) * cfg->n_k, hipMemcpyHostToDevice, c->stream) ||
      hipMemcpyAsync(c->kw_d, c->kw.data(), sizeof(double) * cfg->n_k, hipMemcpyHostToDevice, c->stream))
    return cleanup(fail(c, TDDFT_EDEVICE, "upload of k-points failed"));
  if ((st = upload_orbitals(c, psi0)) != TDDFT_OK) return cleanup(st);
  if (launch_fill(c->Vloc, 0.0, N, c->stream) != hipSuccess || launch_fill(c->vh, 0.0, N, c->stream) != hipSuccess ||
      launch_fill(c->exc, 0.0, N, c->stream) != hipSuccess)
    return cleanup(fail(c, TDDFT_EDEVICE, "initial fill failed"));
  if (launch_set_int(c->nanflag, 0, c->stream) != hipSuccess)
    return cleanup(fail(c, TDDFT_EDEVICE, "flag reset failed"));
  {
    // kappa, kappaJ and the field at A = 0 until the first step sets them
    const double Az[6] = {0, 0, 0, 0, 0, 0};
    if (hipMemcpyAsync(c->Aobs, Az, sizeof(Az), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        launch_step_params(c->Aobs, c->counter, 0, c->kpt_d, cfg->n_k, c->ent_x, 0, cfg->gauge, cfg->dt, c->kappa,
                           c->kappaJ, c->efield, c->phA, c->phAJ, c->Alast, c->stream) != hipSuccess)
      return cleanup(fail(c, TDDFT_EDEVICE, "initial field parameters failed"));
  }
  if ((st = potential_dispatch(c)) != TDDFT_OK) return cleanup(st);
  if (hipMemcpyAsync(c->rho0, c->rho, N * sizeof(double), hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return cleanup(fail(c, TDDFT_EDEVICE, "initial density failed"));
  *out = c;
  return TDDFT_OK;
}

tddft_status tddft_set_potential(tddft_ctx* c, const double* v_loc, int32_t n_atoms, const tddft_atom* atoms) {
  if (!c) return TDDFT_EINVAL;
  if (c->poisoned) return fail(c, TDDFT_ESTATE, "context poisoned: " + c->err);
  if (!v_loc || n_atoms < 0 || (n_atoms > 0 && !atoms)) return fail(c, TDDFT_EINVAL, "bad potential arguments");
  const size_t N = c->N;
  double vmin = 1e300, vmax = -1e300;
  for (size_t i = 0; i < N; ++i) {
    if (!std::isfinite(v_loc[i])) return fail(c, TDDFT_EINVAL, "v_loc not finite");
    vmin = std::min(vmin, v_loc[i]);
    vmax = std::max(vmax, v_loc[i]);
  }
  // ---- nonlocal tables on the host
  std::vector<int> atom_start(1, 0), ent_idx, ent_atom;
  std::vector<double> ent_B, atom_E, ent_x;
  std::vector<int> cover(N, 0);
  double nl_bound = 0;
  for (int a = 0; a < n_atoms; ++a) {
    const tddft_atom& A = atoms[a];
    if (A.npts < 1 || A.n_proj < 1 || A.n_proj > kMaxProj || !A.idx || !A.x || !A.beta || !A.e_kb)
      return fail(c, TDDFT_EINVAL, "atom " + std::to_string(a) + ": bad projector table");
    double ebound = 0;
    for (int p = 0; p < kMaxProj; ++p) {
      const double E = p < A.n_proj ? A.e_kb[p] : 0.0;
      if (!std::isfinite(E)) return fail(c, TDDFT_EINVAL, "KB energy not finite");
      atom_E.push_back(E);
      ebound += std::fabs(E);
    }
    nl_bound = std::max(nl_bound, ebound);
    std::vector<char> seen(N, 0);
    for (int i = 0; i < A.npts; ++i) {
      const int idx = A.idx[i];
      if (idx < 0 || (size_t)idx >= N) return fail(c, TDDFT_EINVAL, "projector index out of range");
      if (seen[idx]) return fail(c, TDDFT_EINVAL, "duplicate projector index within an atom");
      seen[idx] = 1;
      cover[idx]++;
      ent_idx.push_back(idx);
      ent_atom.push_back(a);
      const double x[3] = {A.x[3 * i], A.x[3 * i + 1], A.x[3 * i + 2]};
      for (int d = 0; d < 3; ++d) {
        if (!std::isfinite(x[d])) return fail(c, TDDFT_EINVAL, "projector offset not finite");
        ent_x.push_back(x[d]);
      }
      for (int p = 0; p < kMaxProj; ++p) {
        const double b = p < A.n_proj ? A.beta[(size_t)p * A.npts + i] : 0.0;
        if (!std::isfinite(b)) return fail(c, TDDFT_EINVAL, "projector value not finite");
        ent_B.push_back(b);
        ent_B.push_back(b * x[0]);
        ent_B.push_back(b * x[1]);
        ent_B.push_back(b * x[2]);
      }
    }
    atom_start.push_back((int)ent_idx.size());
  }
  const int S = (int)ent_idx.size();
  int max_overlap = 0;
  std::vector<int> pt_ptr(N + 1, 0);
  for (size_t p = 0; p < N; ++p) {
    pt_ptr[p + 1] = pt_ptr[p] + cover[p];
    max_overlap = std::max(max_overlap, cover[p]);
  }
  std::vector<int> pt_ent(std::max(S, 1)), fillpos(pt_ptr.begin(), pt_ptr.end() - 1);
  for (int e = 0; e < S; ++e) pt_ent[fillpos[ent_idx[e]]++] = e;
  c->nl_bound = nl_bound * std::max(1, max_overlap);
  // greedy colouring: atoms sharing a grid point get different colours
  std::vector<int> color(n_atoms, -1);
  int n_colors = 0;
  {
    for (int a = 0; a < n_atoms; ++a) {
      std::vector<char> used(n_colors + 1, 0);
      for (int e = atom_start[a]; e < atom_start[a + 1]; ++e) {
        const int p = ent_idx[e];
        for (int t = pt_ptr[p]; t < pt_ptr[p + 1]; ++t) {
          const int b = ent_atom[pt_ent[t]];
          if (b != a && color[b] >= 0) used[color[b]] = 1;
        }
      }
      int cl = 0;
      while (cl < n_colors && used[cl]) ++cl;
      color[a] = cl;
      n_colors = std::max(n_colors, cl + 1);
    }
  }
  std::vector<int> color_start(n_colors + 1, 0), color_atoms;
  for (int cl = 0; cl < n_colors; ++cl) {
    for (int a = 0; a < n_atoms; ++a)
      if (color[a] == cl) color_atoms.push_back(a);
    color_start[cl + 1] = (int)color_atoms.size();
  }
  std::vector<int> color_ent_start(n_colors + 1, 0), color_ents;
  for (int cl = 0; cl < n_colors; ++cl) {
    for (int i = color_start[cl]; i < color_start[cl + 1]; ++i)
      for (int e = atom_start[color_atoms[i]]; e < atom_start[color_atoms[i] + 1]; ++e) color_ents.push_back(e);
    color_ent_start[cl + 1] = (int)color_ents.size();
  }
  c->max_overlap = max_overlap;
  // exp(i k . x_e)
  std::vector<double2> phk((size_t)c->cfg.n_k * std::max(S, 1));
  for (int k = 0; k < c->cfg.n_k; ++k)
    for (int e = 0; e < S; ++e) {
      const double arg = c->kpt[3 * k] * ent_x[3 * e] + c->kpt[3 * k + 1] * ent_x[3 * e + 1] +
                         c->kpt[3 * k + 2] * ent_x[3 * e + 2];
      phk[(size_t)k * S + e] = make_double2(std::cos(arg), std::sin(arg));
    }
  // stability: |lambda| dt <= 2 sqrt 2 for the truncated fourth-order Taylor step
  c->vabs = std::max(std::fabs(vmin), std::fabs(vmax));
  for (int i = 0; i < 3; ++i) c->bound_amax[i] = -1.0;
  const double lam = spectral_bound(c, kNoField, vmin, vmax);
  if (std::fabs(c->cfg.dt) * lam > 2.0 * std::sqrt(2.0) && !(c->cfg.flags & TDDFT_FLAG_ALLOW_UNSTABLE)) {
    char buf[200];
    std::snprintf(buf, sizeof buf, "unstable: |dt| * lambda_max = %.4g > 2 sqrt 2 (lambda_max <= %.6g Ha)",
                  std::fabs(c->cfg.dt) * lam, lam);
    return fail(c, TDDFT_EUNSTABLE, buf);
  }
  // ---- device copies (replace any previous tables)
  invalidate_graph(c);
  HIP_TRY(hipStreamSynchronize(c->stream));
  tddft_status st;
  int *d_atom_start, *d_ent_idx, *d_ent_atom, *d_pt_ptr, *d_pt_ent;
  double *d_ent_B, *d_atom_E, *d_ent_x, *d_ent_beta;
  double2 *d_phk, *d_phA, *d_phAJ, *d_Eu, *d_Eu2;
  double* d_jnl;
  const int nA = std::max(n_atoms, 1);
  const int Sx = std::max(S, 1);
  if ((st = dalloc_t(c, atom_start.size(), &d_atom_start)) || (st = dalloc_t(c, Sx, &d_ent_idx)) ||
      (st = dalloc_t(c, Sx, &d_ent_atom)) || (st = dalloc_t(c, N + 1, &d_pt_ptr)) ||
      (st = dalloc_t(c, pt_ent.size(), &d_pt_ent)) || (st = dalloc_t(c, (size_t)Sx * kCols, &d_ent_B)) ||
      (st = dalloc_t(c, (size_t)nA * kMaxProj, &d_atom_E)) || (st = dalloc_t(c, (size_t)Sx * 3, &d_ent_x)) ||
      (st = dalloc_t(c, (size_t)Sx * kMaxProj, &d_ent_beta)) ||
      (st = dalloc_t(c, (size_t)n_colors + 1, &c->color_start)) || (st = dalloc_t(c, (size_t)nA, &c->color_atoms)) ||
      (st = dalloc_t(c, (size_t)Sx, &c->color_ents)) ||
      (st = dalloc_t(c, phk.size(), &d_phk)) || (st = dalloc_t(c, Sx, &d_phA)) ||
      (st = dalloc_t(c, Sx, &d_phAJ)) ||
      (st = dalloc_t(c, c->n_orb_tot * nA * kMaxProj, &d_Eu)) ||
      (st = dalloc_t(c, c->n_orb_tot * nA * kMaxProj, &d_Eu2)) || (st = dalloc_t(c, c->n_orb_tot * 4, &d_jnl)))
    return st;
  auto up = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
    if (bytes == 0) return hipSuccess;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream);
  };
  HIP_TRY(up(d_atom_start, atom_start.data(), atom_start.size() * sizeof(int)));
  HIP_TRY(up(d_ent_idx, ent_idx.data(), S * sizeof(int)));
  HIP_TRY(up(d_ent_atom, ent_atom.data(), S * sizeof(int)));
  HIP_TRY(up(d_pt_ptr, pt_ptr.data(), (N + 1) * sizeof(int)));
  HIP_TRY(up(d_pt_ent, pt_ent.data(), S * sizeof(int)));
  HIP_TRY(up(d_ent_B, ent_B.data(), ent_B.size() * sizeof(double)));
  HIP_TRY(up(d_atom_E, atom_E.data(), atom_E.size() * sizeof(double)));
  HIP_TRY(up(d_ent_x, ent_x.data(), ent_x.size() * sizeof(double)));
  std::vector<double> ent_beta((size_t)S * kMaxProj);
  for (int e = 0; e < S; ++e)
    for (int p = 0; p < kMaxProj; ++p) ent_beta[(size_t)e * kMaxProj + p] = ent_B[(size_t)e * kCols + p * kMoments];
  HIP_TRY(up(d_ent_beta, ent_beta.data(), ent_beta.size() * sizeof(double)));
  HIP_TRY(up(c->color_start, color_start.data(), color_start.size() * sizeof(int)));
  HIP_TRY(up(c->color_atoms, color_atoms.data(), color_atoms.size() * sizeof(int)));
  HIP_TRY(up(c->color_ents, color_ents.data(), color_ents.size() * sizeof(int)));
  c->color_ent_start = color_ent_start;
  c->n_colors = n_colors;
  HIP_TRY(up(d_phk, phk.data(), (size_t)c->cfg.n_k * S * sizeof(double2)));
  HIP_TRY(up(c->Vloc, v_loc, N * sizeof(double)));
  c->nl.n_atoms = n_atoms;
  c->nl.n_ent = S;
  c->nl.atom_start = d_atom_start;
  c->nl.ent_idx = d_ent_idx;
  c->nl.ent_atom = d_ent_atom;
  c->nl.ent_B = d_ent_B;
  c->nl.atom_E = d_atom_E;
  c->nl.pt_ptr = d_pt_ptr;
  c->nl.pt_ent = d_pt_ent;
  c->nl.phk = d_phk;
  c->ent_x = d_ent_x;
  c->ent_beta = d_ent_beta;
  c->fused = !(c->cfg.flags & TDDFT_FLAG_STREAMING) &&
             fused_supported(c->g, n_atoms, c->mixed ? sizeof(float2) : sizeof(double2));
  if (c->fused && (st = dalloc_t(c, (size_t)c->cfg.n_k * Sx, &c->phkA)) != TDDFT_OK) return st;
  c->phA = d_phA;
  c->phAJ = d_phAJ;
  c->Eu = d_Eu;
  c->Eu2 = d_Eu2;
  c->jnl = d_jnl;
  // ---- Hartree kernel in Fourier space
  if (c->cfg.hartree) {
    const size_t Mt = (size_t)c->M[0] * c->M[1] * c->M[2];
    const Geometry& g = c->g;
    if (g.periodic) {
      std::vector<double> K(Mt);
      for (int z = 0; z < c->M[2]; ++z)
        for (int y = 0; y < c->M[1]; ++y)
          for (int x = 0; x < c->M[0]; ++x) {
            const int mi[3] = {x, y, z};
            double G2 = 0;
            for (int d = 0; d < 3; ++d) {
              int m = mi[d];
              if (m > c->M[d] / 2) m -= c->M[d];
              if (2 * m == c->M[d]) m = -m;  // Nyquist: same |G|
              const double G = 2.0 * M_PI * m / c->cfg.cell[d];
              G2 += G * G;
            }
            K[((size_t)z * c->M[1] + y) * c->M[0] + x] = G2 > 0 ? 4.0 * M_PI / G2 : 0.0;
          }
      HIP_TRY(up(c->Kfft, K.data(), Mt * sizeof(double)));
      c->vh_scale = 1.0 / (double)Mt;
    } else {
      // g on the doubled box: 1/|d| for d != 0 and the cell average of 1/r at 0
      const double g0 = self_cell_inverse_r(g.h1, g.h2, g.h3);
      std::vector<double2> gk(Mt);
      for (int z = 0; z < c->M[2]; ++z)
        for (int y = 0; y < c->M[1]; ++y)
          for (int x = 0; x < c->M[0]; ++x) {
            const int ii[3] = {x, y, z};
            double r2 = 0;
            for (int d = 0; d < 3; ++d) {
              const int n = c->cfg.n[d];
              const int off = ii[d] < n ? ii[d] : ii[d] - 2 * n;
              const double hh = c->cfg.cell[d] / n;
              r2 += (off * hh) * (off * hh);
            }
            gk[((size_t)z * c->M[1] + y) * c->M[0] + x] = make_double2(r2 > 0 ? 1.0 / std::sqrt(r2) : g0, 0.0);
          }
      HIP_TRY(up(c->fft, gk.data(), Mt * sizeof(double2)));
      for (int ax = 0; ax < 3; ++ax)
        LAUNCH(launch_fft_axis(c->fft, c->M[0], c->M[1], c->M[2], ax, -1, c->stream), "fft kernel");
      LAUNCH(launch_real_part(c->fft, c->Kfft, Mt, c->stream), "fft kernel real part");
      c->vh_scale = c->dV / (double)Mt;
    }
  }
  c->potential_set = true;
  st = potential_dispatch(c);
  if (st != TDDFT_OK) return st;
  if (!c->fused) {
    st = tune_stage(c);
    if (st != TDDFT_OK) return st;
  } else {
    c->tune_note = "{\"path\": \"fused\"}";
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  return TDDFT_OK;
}

tddft_status tddft_propagate(tddft_ctx* c, int32_t nsteps, const double* A, double* J_out) {
  if (!c) return TDDFT_EINVAL;
  if (nsteps == 0 && !c->poisoned && c->potential_set) return TDDFT_OK;
  tddft_status st = prepare_propagate(c, nsteps, A);
  if (st != TDDFT_OK) return st;
  const bool use_graph = !(c->cfg.flags & (TDDFT_FLAG_NO_GRAPH | TDDFT_FLAG_DEBUG_SYNC));
  if (use_graph && !c->graph) {
    hipGraph_t gr;
    HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    st = step_dispatch(c);
    hipError_t e = hipStreamEndCapture(c->stream, &gr);
    if (st != TDDFT_OK) return st;
    if (e != hipSuccess) return fail(c, TDDFT_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&c->graph, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) return fail(c, TDDFT_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  }
  HIP_TRY(hipEventRecord(c->ev0, c->stream));
  for (int n = 0; n < nsteps; ++n) {
    if (use_graph) {
      HIP_TRY(hipGraphLaunch(c->graph, c->stream));
    } else {
      st = step_dispatch(c);
      if (st != TDDFT_OK) return st;
    }
  }
  HIP_TRY(hipEventRecord(c->ev1, c->stream));
  st = collect_propagate(c, nsteps, A, J_out);
  if (st != TDDFT_OK) return st;
  float ms = 0;
  HIP_TRY(hipEventElapsedTime(&ms, c->ev0, c->ev1));
  c->last_ms = ms / nsteps;
  return TDDFT_OK;
}

tddft_status tddft_density_current(tddft_ctx* c, double* rho, double* J) {
  if (!c) return TDDFT_EINVAL;
  if (c->poisoned) return fail(c, TDDFT_ESTATE, "context poisoned: " + c->err);
  if (rho) {
    HIP_TRY(hipMemcpyAsync(rho, c->rho, c->N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
  }
  if (J) {
    tddft_status st = observe_now(c);
    if (st != TDDFT_OK) return st;
    HIP_TRY(hipMemcpy(J, c->scalars, 3 * sizeof(double), hipMemcpyDeviceToHost));
  }
  return TDDFT_OK;
}

tddft_status tddft_get_orbitals(tddft_ctx* c, double* psi) {
  if (!c || !psi) return c ? fail(c, TDDFT_EINVAL, "null psi") : TDDFT_EINVAL;
  if (c->poisoned) return fail(c, TDDFT_ESTATE, "context poisoned: " + c->err);
  const size_t total = c->n_orb_tot * c->N;
  if (!c->mixed) {
    HIP_TRY(hipMemcpyAsync(psi, c->W, total * sizeof(double2), hipMemcpyDeviceToHost, c->stream));
  } else {
    LAUNCH(launch_convert_out<float>(as2<float>(c->W), static_cast<double2*>(c->U0), total, c->stream),
           "convert_out");
    HIP_TRY(hipMemcpyAsync(psi, c->U0, total * sizeof(double2), hipMemcpyDeviceToHost, c->stream));
  }
  HIP_TRY(hipStreamSynchronize(c->stream));
  return TDDFT_OK;
}

tddft_status tddft_set_orbitals(tddft_ctx* c, const double* psi) {
  if (!c || !psi) return c ? fail(c, TDDFT_EINVAL, "null psi") : TDDFT_EINVAL;
  if (c->poisoned) return fail(c, TDDFT_ESTATE, "context poisoned: " + c->err);
  tddft_status st = upload_orbitals(c, psi);
  if (st != TDDFT_OK) return st;
  st = potential_dispatch(c);
  if (st != TDDFT_OK) return st;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return TDDFT_OK;
}

tddft_status tddft_energy(tddft_ctx* c, double* E) {
  if (!c || !E) return c ? fail(c, TDDFT_EINVAL, "null E") : TDDFT_EINVAL;
  if (c->poisoned) return fail(c, TDDFT_ESTATE, "context poisoned: " + c->err);
  if (!c->potential_set) return fail(c, TDDFT_ESTATE, "energy before set_potential");
  tddft_status st = observe_now(c);
  if (st != TDDFT_OK) return st;
  LAUNCH(launch_grid_sums(c->rho, c->rho0, c->vh, c->exc, c->g, c->sums, c->stream), "grid_sums");
  double sc[8], gs[8];
  HIP_TRY(hipMemcpyAsync(sc, c->scalars, sizeof(sc), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipMemcpyAsync(gs, c->sums, sizeof(gs), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  *E = sc[3] + (c->cfg.hartree ? gs[0] : 0.0) + (c->cfg.xc ? gs[1] : 0.0);
  return TDDFT_OK;
}

tddft_status tddft_xc_parameter(tddft_ctx* c, double* cpar) {
  if (!c || !cpar) return c ? fail(c, TDDFT_EINVAL, "null c") : TDDFT_EINVAL;
  if (c->poisoned) return fail(c, TDDFT_ESTATE, "context poisoned: " + c->err);
  if (!is_mgga(c)) return fail(c, TDDFT_ESTATE, "the mixing parameter belongs to the BJ / TB09 exchange");
  if (!c->potential_set) return fail(c, TDDFT_ESTATE, "xc_parameter before set_potential");
  double v[2];
  HIP_TRY(hipMemcpyAsync(v, c->cval, sizeof(v), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  *cpar = v[0];
  return TDDFT_OK;
}

tddft_status tddft_norms(tddft_ctx* c, double* norms) {
  if (!c || !norms) return c ? fail(c, TDDFT_EINVAL, "null norms") : TDDFT_EINVAL;
  if (c->poisoned) return fail(c, TDDFT_ESTATE, "context poisoned: " + c->err);
  tddft_status st = observe_now(c);
  if (st != TDDFT_OK) return st;
  const int tiles = c->g.tiles_x * c->g.tiles_y * c->g.zslabs;
  std::vector<double> obs(c->n_orb_tot * tiles * 8);
  HIP_TRY(hipMemcpy(obs.data(), c->obs, obs.size() * sizeof(double), hipMemcpyDeviceToHost));
  for (size_t o = 0; o < c->n_orb_tot; ++o) {
    double s = 0;
    for (int t = 0; t < tiles; ++t) s += obs[(o * tiles + t) * 8];
    norms[o] = s * c->dV;
  }
  return TDDFT_OK;
}

tddft_status tddft_dipole(tddft_ctx* c, double d[3]) {
  if (!c || !d) return c ? fail(c, TDDFT_EINVAL, "null d") : TDDFT_EINVAL;
  if (c->poisoned) return fail(c, TDDFT_ESTATE, "context poisoned: " + c->err);
  LAUNCH(launch_grid_sums(c->rho, c->rho0, c->vh, c->exc, c->g, c->sums, c->stream), "grid_sums");
  double gs[8];
  HIP_TRY(hipMemcpyAsync(gs, c->sums, sizeof(gs), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (int i = 0; i < 3; ++i) d[i] = gs[2 + i];
  return TDDFT_OK;
}

tddft_status tddft_kick(tddft_ctx* c, double F0, int32_t axis) {
  if (!c) return TDDFT_EINVAL;
  if (c->poisoned) return fail(c, TDDFT_ESTATE, "context poisoned: " + c->err);
  if (c->g.periodic) return fail(c, TDDFT_EINVAL, "kick needs an isolated box (periodic: use the A table)");
  if (axis < 0 || axis > 2 || !std::isfinite(F0)) return fail(c, TDDFT_EINVAL, "bad kick arguments");
  if (c->mixed)
    LAUNCH(launch_kick<float>(as2<float>(c->W), c->g, F0, axis, c->n_orb_tot, c->stream), "kick");
  else
    LAUNCH(launch_kick<double>(as2<double>(c->W), c->g, F0, axis, c->n_orb_tot, c->stream), "kick");
  tddft_status st = potential_dispatch(c);
  if (st != TDDFT_OK) return st;
  HIP_TRY(hipStreamSynchronize(c->stream));
  return TDDFT_OK;
}

tddft_status tddft_time_kernel(tddft_ctx* c, int32_t which, int32_t reps, double* ms) {
  if (!c || !ms) return TDDFT_EINVAL;
  if (c->poisoned) return fail(c, TDDFT_ESTATE, "context poisoned: " + c->err);
  if (!c->potential_set) return fail(c, TDDFT_ESTATE, "time_kernel before set_potential");
  if (reps < 1 || which < 0 || which > TDDFT_KERNEL_FUSED) return fail(c, TDDFT_EINVAL, "bad kernel or reps");
  if (which == TDDFT_KERNEL_FUSED && !c->fused)
    return fail(c, TDDFT_EINVAL, "this context takes the per-stage kernels, not the fused step");
  const size_t wbytes = c->n_orb_tot * c->N * (c->mixed ? sizeof(float2) : sizeof(double2));
  if (which == TDDFT_KERNEL_FUSED)
    HIP_TRY(hipMemcpyAsync(c->U0, c->W, wbytes, hipMemcpyDeviceToDevice, c->stream));
  double Ab[6];
  for (int i = 0; i < 3; ++i) Ab[i] = Ab[3 + i] = c->A_last[i];
  HIP_TRY(hipMemcpyAsync(c->Aobs, Ab, sizeof(Ab), hipMemcpyHostToDevice, c->stream));
  LAUNCH(launch_step_params(c->Aobs, c->counter, 0, c->kpt_d, c->cfg.n_k, c->ent_x, c->nl.n_ent,
                            c->cfg.gauge, c->cfg.dt, c->kappa, c->kappaJ, c->efield, c->phA, c->phAJ,
                            c->Alast, c->stream),
         "step_params");
  tddft_status st = enqueue_coef(c);
  if (st != TDDFT_OK) return st;
  st = c->mixed ? launch_one<float>(c, which) : launch_one<double>(c, which);  // warm-up
  if (st != TDDFT_OK) return st;
  HIP_TRY(hipEventRecord(c->ev0, c->stream));
  for (int r = 0; r < reps; ++r) {
    st = c->mixed ? launch_one<float>(c, which) : launch_one<double>(c, which);
    if (st != TDDFT_OK) return st;
  }
  HIP_TRY(hipEventRecord(c->ev1, c->stream));
  if (which == TDDFT_KERNEL_FUSED)
    HIP_TRY(hipMemcpyAsync(c->W, c->U0, wbytes, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  float t = 0;
  HIP_TRY(hipEventElapsedTime(&t, c->ev0, c->ev1));
  *ms = t / reps;
  return TDDFT_OK;
}

tddft_status tddft_ground_state(tddft_ctx* c, int32_t n_iter, double tau, double* energies) {
  if (!c) return TDDFT_EINVAL;
  if (c->poisoned) return fail(c, TDDFT_ESTATE, "context poisoned: " + c->err);
  if (!c->potential_set) return fail(c, TDDFT_ESTATE, "ground_state before set_potential");
  if (n_iter < 0 || !(tau > 0.0) || !std::isfinite(tau)) return fail(c, TDDFT_EINVAL, "bad ground-state arguments");
  const double lam = spectral_bound(c, kNoField, -c->vabs, c->vabs);
  // P4(-x) = 1 - x + x^2/2 - x^3/6 + x^4/24 decreases monotonically only up to
  // x = 1.596 (where P4'(-x) = 0); beyond it high modes are damped less than
  // lower ones and the iteration can settle on the wrong subspace
  if (tau * lam > 1.59)
    return fail(c, TDDFT_EUNSTABLE, "tau * lambda_max > 1.59: the damping polynomial is not monotone there");
  const int n = c->cfg.n_orb;
  if (!c->gram) {
    tddft_status st = dalloc_t(c, (size_t)2 * c->cfg.n_k * n * n, &c->gram);
    if (st != TDDFT_OK) return st;
    if ((st = dalloc_t(c, 1, &c->chol_bad)) != TDDFT_OK) return st;
  }
  LAUNCH(launch_set_int(c->chol_bad, 0, c->stream), "flag reset");
  invalidate_graph(c);
  for (int i = 0; i < 3; ++i) c->A_last[i] = 0.0;
  double Ab[6] = {0, 0, 0, 0, 0, 0};
  HIP_TRY(hipMemcpyAsync(c->Aobs, Ab, sizeof(Ab), hipMemcpyHostToDevice, c->stream));
  for (int it = 0; it < n_iter; ++it) {
    LAUNCH(launch_step_params(c->Aobs, c->counter, 0, c->kpt_d, c->cfg.n_k, c->ent_x, c->nl.n_ent,
                              c->cfg.gauge, c->cfg.dt, c->kappa, c->kappaJ, c->efield, c->phA, c->phAJ,
                              c->Alast, c->stream),
           "step_params");
    tddft_status st = enqueue_coef(c);
    if (st != TDDFT_OK) return st;
    st = c->mixed ? ground_state_iteration<float>(c, tau) : ground_state_iteration<double>(c, tau);
    if (st != TDDFT_OK) return st;
    if (energies) {
      st = tddft_energy(c, &energies[it]);
      if (st != TDDFT_OK) return st;
    }
  }
  HIP_TRY(hipMemcpyAsync(c->rho0, c->rho, c->N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  int bad = 0;
  HIP_TRY(hipMemcpyAsync(&bad, c->chol_bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  if (bad) return fail(c, TDDFT_ENUMERIC, "orbitals became linearly dependent");
  return TDDFT_OK;
}

tddft_status tddft_set_reference(tddft_ctx* c) {
  if (!c) return TDDFT_EINVAL;
  if (c->poisoned) return fail(c, TDDFT_ESTATE, "context poisoned: " + c->err);
  if (c->cfg.n_orb > 64) return fail(c, TDDFT_EINVAL, "the excited-pair count supports at most 64 orbitals");
  const size_t wbytes = c->n_orb_tot * c->N * (c->mixed ? sizeof(float2) : sizeof(double2));
  tddft_status st;
  if (!c->Wref && (st = dalloc(c, wbytes, &c->Wref)) != TDDFT_OK) return st;
  if (!c->Sk && (st = dalloc_t(c, (size_t)c->cfg.n_k, &c->Sk)) != TDDFT_OK) return st;
  LAUNCH(launch_copy8(c->W, c->Wref, wbytes, c->stream), "copy reference");
  HIP_TRY(hipStreamSynchronize(c->stream));
  // the energy of the reference state, for the excitation energy (only where
  // the potential comes from an energy functional)
  c->have_E_ref = false;
  if (c->potential_set && !is_mgga(c)) {
    st = tddft_energy(c, &c->E_ref);
    if (st != TDDFT_OK) return st;
    c->have_E_ref = true;
  }
  return TDDFT_OK;
}

tddft_status tddft_excitation_energy(tddft_ctx* c, double* E_ex) {
  if (!c || !E_ex) return c ? fail(c, TDDFT_EINVAL, "null E_ex") : TDDFT_EINVAL;
  if (c->poisoned) return fail(c, TDDFT_ESTATE, "context poisoned: " + c->err);
  if (!c->have_E_ref)
    return fail(c, TDDFT_ESTATE,
                is_mgga(c) ? "the BJ / TB09 potentials have no energy functional: use tddft_work on the current"
                           : "excitation_energy before set_reference (with the potential set)");
  double E = 0.0;
  tddft_status st = tddft_energy(c, &E);
  if (st != TDDFT_OK) return st;
  *E_ex = E - c->E_ref;
  return TDDFT_OK;
}

tddft_status tddft_excited_electrons(tddft_ctx* c, double* n_ex) {
  if (!c || !n_ex) return c ? fail(c, TDDFT_EINVAL, "null n_ex") : TDDFT_EINVAL;
  if (c->poisoned) return fail(c, TDDFT_ESTATE, "context poisoned: " + c->err);
  if (!c->Wref) return fail(c, TDDFT_ESTATE, "excited_electrons before set_reference");
  const int nk = c->cfg.n_k, n = c->cfg.n_orb;
  if (c->mixed)
    LAUNCH(launch_overlap_weight<float>(as2<float>(c->Wref), as2<float>(c->W), n, nk, (int)c->N, c->dV, c->Sk,
                                        c->stream),
           "overlap weight");
  else
    LAUNCH(launch_overlap_weight<double>(as2<double>(c->Wref), as2<double>(c->W), n, nk, (int)c->N, c->dV, c->Sk,
                                         c->stream),
           "overlap weight");
  std::vector<double> S(nk);
  HIP_TRY(hipMemcpyAsync(S.data(), c->Sk, nk * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  double total = 0.0;
  for (int k = 0; k < nk; ++k) total += c->kw[k] * 2.0 * ((double)n - S[k]);
  *n_ex = total / c->volume;
  return TDDFT_OK;
}

tddft_status tddft_report(tddft_ctx* c, char* buf, size_t len) {
  if (!c || !buf || len == 0) return c ? fail(c, TDDFT_EINVAL, "null buffer") : TDDFT_EINVAL;
  const std::string r = c->tune_note.empty() ? std::string("{}") : c->tune_note;
  std::snprintf(buf, len, "%s", r.c_str());
  return r.size() < len ? TDDFT_OK : fail(c, TDDFT_EINVAL, "report buffer too small");
}

tddft_status tddft_last_timing(tddft_ctx* c, double* ms) {
  if (!c || !ms) return TDDFT_EINVAL;
  *ms = c->last_ms;
  return TDDFT_OK;
}

}  // extern "C"

// ===========================================================================
// Batches of cells

namespace {

struct BatchGroup {
  int n = 0;
  bool periodic = true;
  std::vector<int> cells;      // cell indices, largest first
  void* d_args = nullptr;      // FusedArgs<T>[cells.size()]
  int2* d_items = nullptr;
  int n_items = 0;
  int* d_queue = nullptr;
  size_t lds = 0;
  int zs = 1, wgs = 0;
  std::vector<std::pair<int, int>> cand;  // (zs, workgroups)
  std::vector<double> cand_ms;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  // the end of the step (current, density, Poisson, xc) as one launch per
  // kernel over the group's cells, when they all take the same kernels
  bool tail_ok = false;
  int max_chunks = 1;
  TailCell* d_tail = nullptr;
  // the start of the step (field, kappa, phases, coefficients) for all cells
  ParamCell* d_par = nullptr;
  int max_S = 0, max_nk = 0;
  long max_phases = 0;
};

}  // namespace

struct tddft_batch {
  std::vector<tddft_ctx*> cells;
  std::string err;
  bool poisoned = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool mixed = false;
  uint32_t flags = 0;
  int n_cu = 256;
  bool planned = false;
  int tune_next = 0;           // next candidate index while tuning
  std::vector<BatchGroup> groups;
  std::vector<std::vector<int>> lanes;  // per-stage cells per forked stream
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> side_done;
  hipEvent_t fork = nullptr, ev0 = nullptr, ev1 = nullptr;
  hipGraphExec_t graph = nullptr;
  double last_ms = 0;
  std::vector<void*> allocs;
  // one staging area each way for the cells' A and J tables: the IOCell
  // table, then [cells][3 (n + 1)] A values, or [cells][3 n + 1] J values and flags
  double* d_stage = nullptr;
  double* h_stage = nullptr;  // pinned
  size_t stage_cap = 0;       // doubles
};

namespace {

tddft_status bfail(tddft_batch* b, tddft_status st, const std::string& m) {
  if (b) {
    b->err = m;
    if (st == TDDFT_EDEVICE || st == TDDFT_ENUMERIC) b->poisoned = true;
  }
  return st;
}

#define BHIP(expr)                                                                          \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return bfail(b, TDDFT_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

tddft_status bcell(tddft_batch* b, tddft_status st, int i) {
  if (st == TDDFT_OK) return st;
  return bfail(b, st, "cell " + std::to_string(i) + ": " + b->cells[i]->err);
}

template <typename T>
tddft_status batch_plan(tddft_batch* b) {
  const int nc = (int)b->cells.size();
  std::vector<int> streaming;
  for (int i = 0; i < nc; ++i) {
    tddft_ctx* c = b->cells[i];
    if (!c->fused) {
      streaming.push_back(i);
      continue;
    }
    BatchGroup* g = nullptr;
    for (auto& gg : b->groups)
      if (gg.n == c->g.n3 && gg.periodic == (c->g.periodic != 0)) g = &gg;
    if (!g) {
      b->groups.emplace_back();
      g = &b->groups.back();
      g->n = c->g.n3;
      g->periodic = c->g.periodic != 0;
    }
    g->cells.push_back(i);
  }
  // work of one orbital item: grid points plus sphere entries (nonlocal part)
  auto cost = [&](int i) { return (double)b->cells[i]->N + 4.0 * b->cells[i]->nl.n_ent; };
  for (auto& g : b->groups) {
    std::stable_sort(g.cells.begin(), g.cells.end(), [&](int x, int y) { return cost(x) > cost(y); });
    std::vector<FusedArgs<T>> args;
    std::vector<int2> items;
    for (size_t j = 0; j < g.cells.size(); ++j) {
      tddft_ctx* c = b->cells[g.cells[j]];
      args.push_back(fused_args<T>(c));
      g.lds = std::max(g.lds, fused_lds_bytes(c->g, c->nl.n_atoms, sizeof(typename Vec2<T>::type)));
      for (size_t o = 0; o < c->n_orb_tot; ++o) items.push_back(make_int2((int)j, (int)o));
    }
    g.n_items = (int)items.size();
    void* p;
    BHIP(hipMalloc(&p, args.size() * sizeof(FusedArgs<T>)));
    b->allocs.push_back(p);
    g.d_args = p;
    BHIP(hipMalloc(&p, items.size() * sizeof(int2)));
    b->allocs.push_back(p);
    g.d_items = static_cast<int2*>(p);
    BHIP(hipMalloc(&p, sizeof(int)));
    b->allocs.push_back(p);
    g.d_queue = static_cast<int*>(p);
    BHIP(hipMemcpyAsync(g.d_args, args.data(), args.size() * sizeof(FusedArgs<T>), hipMemcpyHostToDevice, b->stream));
    BHIP(hipMemcpyAsync(g.d_items, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream));
    // the tuner only sizes the persistent grid: the column split is fixed per
    // grid size, so no tuning decision changes a single bit of the result
    g.zs = fused_column_split(g.n);
    for (int per_cu : {1, 2, 3, 4}) g.cand.push_back({g.zs, per_cu * b->n_cu});
    g.wgs = b->n_cu;
    BHIP(hipEventCreate(&g.e0));
    BHIP(hipEventCreate(&g.e1));
    // one tail launch per kernel for the whole group when every cell runs
    // the same tail kernels (LDA or no xc, the same Hartree switch and box)
    const tddft_ctx* c0 = b->cells[g.cells[0]];
    g.tail_ok = true;
    for (int i : g.cells) {
      const tddft_ctx* c = b->cells[i];
      g.max_chunks = std::max(g.max_chunks, c->rho_nchunks);
      if (is_mgga(c) || c->cfg.hartree != c0->cfg.hartree || c->cfg.xc != c0->cfg.xc ||
          c->rho_chunk != c0->rho_chunk || c->N != c0->N || c->M[0] != c0->M[0] || c->M[1] != c0->M[1] ||
          c->M[2] != c0->M[2])
        g.tail_ok = false;
    }
    if (g.tail_ok) {
      BHIP(hipMalloc(&p, g.cells.size() * sizeof(TailCell)));
      b->allocs.push_back(p);
      g.d_tail = static_cast<TailCell*>(p);
    }
    for (int i : g.cells) {
      const tddft_ctx* c = b->cells[i];
      g.max_S = std::max(g.max_S, c->nl.n_ent);
      g.max_nk = std::max(g.max_nk, c->cfg.n_k);
      g.max_phases = std::max(g.max_phases, (long)c->cfg.n_k * c->nl.n_ent);
    }
    BHIP(hipMalloc(&p, g.cells.size() * sizeof(ParamCell)));
    b->allocs.push_back(p);
    g.d_par = static_cast<ParamCell*>(p);
  }
  // per-stage cells: longest-processing-time-first over up to four streams
  const int L = std::min<int>(4, (int)streaming.size());
  b->lanes.assign(L, {});
  std::vector<double> load(L, 0.0);
  std::stable_sort(streaming.begin(), streaming.end(), [&](int x, int y) {
    return (double)b->cells[x]->N * b->cells[x]->n_orb_tot > (double)b->cells[y]->N * b->cells[y]->n_orb_tot;
  });
  for (int i : streaming) {
    const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    b->lanes[l].push_back(i);
    load[l] += (double)b->cells[i]->N * b->cells[i]->n_orb_tot;
  }
  const int nside = (int)b->groups.size() + L;
  for (int i = 0; i < nside; ++i) {
    hipStream_t s;
    hipEvent_t e;
    BHIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    BHIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    b->side.push_back(s);
    b->side_done.push_back(e);
  }
  BHIP(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
  BHIP(hipStreamSynchronize(b->stream));
  b->planned = true;
  b->tune_next = (b->flags & TDDFT_FLAG_NO_TUNE) ? -1 : -2;  // -2: one unrecorded warm-up step first
  return TDDFT_OK;
}

// the group tail tables from the cells' current buffers (a cell's A and J
// tables move when a longer run needs more room)
tddft_status batch_tail_upload(tddft_batch* b) {
  for (auto& g : b->groups) {
    std::vector<ParamCell> par(g.cells.size());
    for (size_t j = 0; j < g.cells.size(); ++j) {
      tddft_ctx* c = b->cells[g.cells[j]];
      ParamCell& q = par[j];
      q.A = c->Atab;
      q.counter = c->counter;
      q.kpt = c->kpt_d;
      q.n_k = c->cfg.n_k;
      q.S = c->nl.n_ent;
      q.gauge = c->cfg.gauge;
      q.ent_x = c->ent_x;
      q.dt = c->cfg.dt;
      q.kappa = c->kappa;
      q.kappaJ = c->kappaJ;
      q.efield = c->efield;
      q.phA = c->phA;
      q.phAJ = c->phAJ;
      q.Alast = c->Alast;
      std::memcpy(q.dh, c->dh, sizeof(q.dh));
      q.cdiag = c->cdiag;
      q.coef = c->coef;
      q.phk = c->nl.phk;
      q.phkA = c->phkA;
    }
    BHIP(hipMemcpyAsync(g.d_par, par.data(), par.size() * sizeof(ParamCell), hipMemcpyHostToDevice, b->stream));
    BHIP(hipStreamSynchronize(b->stream));
    if (!g.tail_ok) continue;
    std::vector<TailCell> tab(g.cells.size());
    for (size_t j = 0; j < g.cells.size(); ++j) {
      tddft_ctx* c = b->cells[g.cells[j]];
      TailCell& t = tab[j];
      t.w = c->W;
      t.kw = c->kw_d;
      t.n_orb = c->cfg.n_orb;
      t.n_k = c->cfg.n_k;
      t.nchunks = c->rho_nchunks;
      t.rho_out = c->rho_nchunks == 1 ? c->rho : c->rho_part;
      t.rho_part = c->rho_part;
      t.rho = c->rho;
      t.fft = c->fft;
      t.Kfft = c->Kfft;
      t.vh_scale = c->vh_scale;
      t.Vloc = c->Vloc;
      t.Vd = c->Vd;
      t.Vf = c->Vf;
      t.vh = c->vh;
      t.exc = c->exc;
      t.obs = c->obs;
      t.jnl = c->jnl;
      t.use_nl = c->nl.n_atoms > 0 ? 1 : 0;
      t.kappaJ = c->kappaJ;
      t.dV = c->dV;
      t.volume = c->volume;
      t.counter = c->counter;
      t.Jtab = c->Jtab;
      t.scalars = c->scalars;
      t.nanflag = c->nanflag;
      t.norm_tol = norm_tol(c);
    }
    BHIP(hipMemcpyAsync(g.d_tail, tab.data(), tab.size() * sizeof(TailCell), hipMemcpyHostToDevice, b->stream));
    BHIP(hipStreamSynchronize(b->stream));
  }
  return TDDFT_OK;
}

// the end of the step for every cell of a group, one launch per kernel: the
// same kernels and order as enqueue_fused_tail applied to each cell
template <typename T>
tddft_status enqueue_group_tail(tddft_batch* b, const BatchGroup& g, hipStream_t s) {
  const tddft_ctx* c0 = b->cells[g.cells[0]];
  const int nc = (int)g.cells.size();
  const int N = (int)c0->N;
  BHIP(launch_finish_group(g.d_tail, nc, 1, s));
  BHIP(launch_rho_partial_group<T>(g.d_tail, nc, N, c0->rho_chunk, g.max_chunks, s));
  if (g.max_chunks > 1) BHIP(launch_rho_reduce_group(g.d_tail, nc, N, s));
  const int M1 = c0->M[0], M2 = c0->M[1], M3 = c0->M[2];
  const int n1 = c0->g.n1, n2 = c0->g.n2, n3 = c0->g.n3;
  if (c0->cfg.hartree) {
    BHIP(launch_fft_lines_group(g.d_tail, nc, M1, M2, M3, 0, -1, 1, n1, n2, n3, 0, n2, n3, n1, M1, 0, s));
    BHIP(launch_fft_lines_group(g.d_tail, nc, M1, M2, M3, 1, -1, 0, n1, n2, n3, 0, M1, n3, n2, M2, 0, s));
    BHIP(launch_fft_lines_group(g.d_tail, nc, M1, M2, M3, 2, -1, 0, n1, n2, n3, 1, M1, M2, n3, n3, 1, s));
    BHIP(launch_fft_lines_group(g.d_tail, nc, M1, M2, M3, 1, +1, 0, n1, n2, n3, 0, M1, n3, M2, n2, 0, s));
    BHIP(launch_fft_lines_group(g.d_tail, nc, M1, M2, M3, 0, +1, 0, n1, n2, n3, 0, n2, n3, M1, n1, 0, s));
  }
  BHIP(launch_xc_group(g.d_tail, nc, n1, n2, n3, M1, M2, c0->cfg.hartree, c0->cfg.xc, s));
  return TDDFT_OK;
}

// One batch step. timing: bracket each group's persistent launch with events.
template <typename T>
tddft_status batch_step(tddft_batch* b, bool timing) {
  // the start of the step: one launch per kernel for each fused group, per
  // cell for the per-stage lanes (the same kernels and arithmetic either way)
  for (auto& g : b->groups) {
    const int nc = (int)g.cells.size();
    BHIP(launch_step_params_group(g.d_par, nc, g.max_S, b->stream));
    BHIP(launch_fused_coef_group<T>(g.d_par, nc, g.max_nk, g.max_phases, b->stream));
  }
  for (auto& lane : b->lanes)
    for (int i : lane) {
      tddft_ctx* c = b->cells[i];
      c->stream = b->stream;
      tddft_status st = enqueue_params(c);
      if (st != TDDFT_OK) return bcell(b, st, i);
    }
  BHIP(hipEventRecord(b->fork, b->stream));
  int si = 0;
  for (auto& g : b->groups) {
    hipStream_t s = b->side[si];
    BHIP(hipStreamWaitEvent(s, b->fork, 0));
    BHIP(launch_set_int(g.d_queue, 0, s));
    if (timing) BHIP(hipEventRecord(g.e0, s));
    BHIP(launch_fused_persistent<T>(g.n, g.zs, g.periodic, static_cast<const FusedArgs<T>*>(g.d_args), g.d_items,
                                    g.n_items, g.d_queue, g.wgs, g.lds, s));
    if (timing) BHIP(hipEventRecord(g.e1, s));
    if (g.tail_ok) {
      tddft_status st = enqueue_group_tail<T>(b, g, s);
      if (st != TDDFT_OK) return st;
    } else {
      for (int i : g.cells) {
        tddft_ctx* c = b->cells[i];
        c->stream = s;
        tddft_status st = enqueue_fused_tail<T>(c);
        c->stream = b->stream;
        if (st != TDDFT_OK) return bcell(b, st, i);
      }
    }
    BHIP(hipEventRecord(b->side_done[si], s));
    ++si;
  }
  for (auto& lane : b->lanes) {
    hipStream_t s = b->side[si];
    BHIP(hipStreamWaitEvent(s, b->fork, 0));
    for (int i : lane) {
      tddft_ctx* c = b->cells[i];
      c->stream = s;
      tddft_status st = enqueue_streaming_update<T>(c);
      c->stream = b->stream;
      if (st != TDDFT_OK) return bcell(b, st, i);
    }
    BHIP(hipEventRecord(b->side_done[si], s));
    ++si;
  }
  for (int i = 0; i < si; ++i) BHIP(hipStreamWaitEvent(b->stream, b->side_done[i], 0));
  return TDDFT_OK;
}

template <typename T>
tddft_status batch_propagate(tddft_batch* b, int32_t nsteps) {
  if (!b->planned) {
    tddft_status st = batch_plan<T>(b);
    if (st != TDDFT_OK) return st;
  }
  {
    tddft_status st = batch_tail_upload(b);
    if (st != TDDFT_OK) return st;
  }
  int done = 0;
  if (b->tune_next == -2) {  // warm-up step (first launches load code objects)
    tddft_status st = batch_step<T>(b, false);
    if (st != TDDFT_OK) return st;
    b->tune_next = 0;
    ++done;
  }
  // online tuning: each candidate runs one real step (identical results)
  while (b->tune_next >= 0 && done < nsteps) {
    size_t maxc = 0;
    for (auto& g : b->groups) maxc = std::max(maxc, g.cand.size());
    if ((size_t)b->tune_next >= maxc) {
      for (auto& g : b->groups) {
        size_t best = 0;
        for (size_t i = 1; i < g.cand_ms.size(); ++i)
          if (g.cand_ms[i] < g.cand_ms[best]) best = i;
        if (!g.cand_ms.empty()) {
          g.zs = g.cand[best].first;
          g.wgs = g.cand[best].second;
        }
      }
      b->tune_next = -1;
      break;
    }
    for (auto& g : b->groups) {
      const size_t ci = std::min((size_t)b->tune_next, g.cand.size() - 1);
      g.zs = g.cand[ci].first;
      g.wgs = g.cand[ci].second;
    }
    tddft_status st = batch_step<T>(b, true);
    if (st != TDDFT_OK) return st;
    BHIP(hipStreamSynchronize(b->stream));
    for (auto& g : b->groups) {
      if ((size_t)b->tune_next < g.cand.size()) {
        float ms = 0;
        BHIP(hipEventElapsedTime(&ms, g.e0, g.e1));
        g.cand_ms.push_back(ms);
      }
    }
    ++b->tune_next;
    ++done;
  }
  if (done >= nsteps) return TDDFT_OK;
  const bool use_graph = !(b->flags & (TDDFT_FLAG_NO_GRAPH | TDDFT_FLAG_DEBUG_SYNC));
  if (use_graph && !b->graph) {
    hipGraph_t gr;
    BHIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    tddft_status st = batch_step<T>(b, false);
    hipError_t e = hipStreamEndCapture(b->stream, &gr);
    if (st != TDDFT_OK) return st;
    if (e != hipSuccess) return bfail(b, TDDFT_EDEVICE, std::string("batch graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&b->graph, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) return bfail(b, TDDFT_EDEVICE, std::string("batch graph: ") + hipGetErrorString(e));
  }
  BHIP(hipEventRecord(b->ev0, b->stream));
  for (int n = done; n < nsteps; ++n) {
    if (use_graph) {
      BHIP(hipGraphLaunch(b->graph, b->stream));
    } else {
      tddft_status st = batch_step<T>(b, false);
      if (st != TDDFT_OK) return st;
    }
  }
  BHIP(hipEventRecord(b->ev1, b->stream));
  BHIP(hipStreamSynchronize(b->stream));
  float ms = 0;
  BHIP(hipEventElapsedTime(&ms, b->ev0, b->ev1));
  b->last_ms = ms / (nsteps - done);
  return TDDFT_OK;
}

}  // namespace

extern "C" {

tddft_status tddft_batch_create(int32_t n_cells, const tddft_config* cfgs, const double* const* psi0,
                                tddft_batch** out) {
  if (!out) return TDDFT_EINVAL;
  *out = nullptr;
  if (n_cells < 1 || !cfgs || !psi0) return TDDFT_EINVAL;
  if (cfgs[0].flags & TDDFT_FLAG_PREDICTOR_CORRECTOR) return TDDFT_EINVAL;  // single contexts only
  auto* b = new tddft_batch();
  b->mixed = cfgs[0].precision == TDDFT_MIXED;
  b->flags = cfgs[0].flags;
  if (cfgs[0].stream) {
    b->stream = static_cast<hipStream_t>(cfgs[0].stream);
  } else if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
    delete b;
    return TDDFT_EDEVICE;
  } else {
    b->own_stream = true;
  }
  int dev = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&b->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  for (int i = 0; i < n_cells; ++i) {
    tddft_config cf = cfgs[i];
    cf.precision = cfgs[0].precision;
    cf.stream = b->stream;
    cf.flags = cfgs[0].flags;
    tddft_ctx* c = nullptr;
    tddft_status st = tddft_init(&cf, psi0[i], &c);
    if (st != TDDFT_OK) {
      tddft_batch_free(b);
      return st;
    }
    b->cells.push_back(c);
  }
  if (hipEventCreate(&b->ev0) != hipSuccess || hipEventCreate(&b->ev1) != hipSuccess) {
    tddft_batch_free(b);
    return TDDFT_EDEVICE;
  }
  *out = b;
  return TDDFT_OK;
}

tddft_status tddft_batch_set_potential(tddft_batch* b, int32_t cell, const double* v_loc, int32_t n_atoms,
                                       const tddft_atom* atoms) {
  if (!b) return TDDFT_EINVAL;
  if (b->poisoned) return bfail(b, TDDFT_ESTATE, "batch poisoned: " + b->err);
  if (cell < 0 || cell >= (int)b->cells.size()) return bfail(b, TDDFT_EINVAL, "cell out of range");
  if (b->planned) return bfail(b, TDDFT_ESTATE, "potentials are fixed once the batch has propagated");
  return bcell(b, tddft_set_potential(b->cells[cell], v_loc, n_atoms, atoms), cell);
}

tddft_status tddft_batch_propagate(tddft_batch* b, int32_t nsteps, const double* const* A, double* const* J_out) {
  if (!b) return TDDFT_EINVAL;
  if (b->poisoned) return bfail(b, TDDFT_ESTATE, "batch poisoned: " + b->err);
  if (nsteps < 0 || (nsteps > 0 && !A)) return bfail(b, TDDFT_EINVAL, "bad propagate arguments");
  if (nsteps == 0) return TDDFT_OK;
  const int nc = (int)b->cells.size();
  for (int i = 0; i < nc; ++i) {
    tddft_ctx* c = b->cells[i];
    c->stream = b->stream;
    const bool had = c->cap_steps >= nsteps;
    tddft_status st = prepare_propagate(c, nsteps, A[i], false);
    if (st != TDDFT_OK) return bcell(b, st, i);
    if (!had && b->graph) {  // a cell's A/J tables moved: the captured step must be rebuilt
      (void)hipGraphExecDestroy(b->graph);
      b->graph = nullptr;
    }
  }
  // the A tables of every cell with one copy: the IOCell table and the tables
  // staged in pinned memory, scattered on the device (counters reset there)
  const size_t io_d = (nc * sizeof(IOCell) + sizeof(double) - 1) / sizeof(double);
  const size_t len_in = 3 * (size_t)(nsteps + 1), len_out = 3 * (size_t)nsteps + 1;
  const size_t need = io_d + (size_t)nc * std::max(len_in, len_out);
  if (need > b->stage_cap) {
    const size_t cap = std::max(need, 2 * b->stage_cap);
    BHIP(hipStreamSynchronize(b->stream));
    if (b->d_stage) (void)hipFree(b->d_stage);
    if (b->h_stage) (void)hipHostFree(b->h_stage);
    b->d_stage = nullptr;
    b->h_stage = nullptr;
    b->stage_cap = 0;
    BHIP(hipMalloc(&b->d_stage, cap * sizeof(double)));
    BHIP(hipHostMalloc(&b->h_stage, cap * sizeof(double)));
    b->stage_cap = cap;
  }
  IOCell* hio = reinterpret_cast<IOCell*>(b->h_stage);
  for (int i = 0; i < nc; ++i) {
    tddft_ctx* c = b->cells[i];
    hio[i] = IOCell{c->Atab, c->counter, c->Jtab, c->nanflag};
    std::memcpy(b->h_stage + io_d + (size_t)i * len_in, A[i], len_in * sizeof(double));
  }
  const IOCell* dio = reinterpret_cast<const IOCell*>(b->d_stage);
  BHIP(hipMemcpyAsync(b->d_stage, b->h_stage, (io_d + (size_t)nc * len_in) * sizeof(double), hipMemcpyHostToDevice,
                      b->stream));
  BHIP(launch_batch_tables_in(dio, nc, b->d_stage + io_d, (int)len_in, b->stream));
  tddft_status st = b->mixed ? batch_propagate<float>(b, nsteps) : batch_propagate<double>(b, nsteps);
  if (st != TDDFT_OK) return st;
  // the J tables and NaN flags back with one copy and one wait
  BHIP(launch_batch_tables_out(dio, nc, b->d_stage + io_d, (int)(len_out - 1), b->stream));
  BHIP(hipMemcpyAsync(b->h_stage + io_d, b->d_stage + io_d, (size_t)nc * len_out * sizeof(double),
                      hipMemcpyDeviceToHost, b->stream));
  BHIP(hipStreamSynchronize(b->stream));
  for (int i = 0; i < nc; ++i) {
    tddft_ctx* c = b->cells[i];
    const double* out = b->h_stage + io_d + (size_t)i * len_out;
    if (J_out && J_out[i]) std::memcpy(J_out[i], out, (len_out - 1) * sizeof(double));
    for (int k = 0; k < 3; ++k) c->A_last[k] = A[i][3 * (size_t)nsteps + k];
    c->last_ms = b->last_ms;
    const int flag = (int)out[len_out - 1];
    if (flag & 1) return bcell(b, fail(c, TDDFT_ENUMERIC, "NaN or Inf in the orbital norms or current"), i);
    if (flag & 2)
      return bcell(b, fail(c, TDDFT_ENUMERIC, "norm watchdog: an orbital norm left 1 by more than 1e-3 (unstable step?)"),
                   i);
  }
  return TDDFT_OK;
}

tddft_ctx* tddft_batch_cell(tddft_batch* b, int32_t cell) {
  if (!b || cell < 0 || cell >= (int)b->cells.size()) return nullptr;
  return b->cells[cell];
}

tddft_status tddft_batch_last_timing(tddft_batch* b, double* ms) {
  if (!b || !ms) return TDDFT_EINVAL;
  *ms = b->last_ms;
  return TDDFT_OK;
}

tddft_status tddft_batch_report(tddft_batch* b, char* buf, size_t len) {
  if (!b || !buf || len == 0) return TDDFT_EINVAL;
  std::string r = "{\"groups\": [";
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    const auto& g = b->groups[gi];
    char tmp[256];
    std::snprintf(tmp, sizeof tmp,
                  "%s{\"n\": %d, \"cells\": %zu, \"items\": %d, \"zs\": %d, \"workgroups\": %d, "
                  "\"grouped_tail\": %s, \"tuned_ms\": [",
                  gi ? ", " : "", g.n, g.cells.size(), g.n_items, g.zs, g.wgs, g.tail_ok ? "true" : "false");
    r += tmp;
    for (size_t i = 0; i < g.cand_ms.size(); ++i) {
      std::snprintf(tmp, sizeof tmp, "%s[%d, %d, %.4f]", i ? ", " : "", g.cand[i].first, g.cand[i].second,
                    g.cand_ms[i]);
      r += tmp;
    }
    r += "]}";
  }
  r += "], \"per_stage_cells\": [";
  bool first = true;
  for (const auto& lane : b->lanes)
    for (int i : lane) {
      r += (first ? "" : ", ") + std::to_string(i);
      first = false;
    }
  // the per-stage decomposition chosen for each cell shape
  r += "], \"per_stage_tiles\": {";
  std::vector<std::string> seen;
  for (const auto& lane : b->lanes)
    for (int i : lane) {
      const tddft_ctx* c = b->cells[i];
      const size_t k0 = c->tune_choice.find("\"key\": \"");
      if (k0 == std::string::npos) continue;
      const size_t k1 = c->tune_choice.find('"', k0 + 8);
      const std::string key = c->tune_choice.substr(k0 + 8, k1 - k0 - 8);
      if (std::find(seen.begin(), seen.end(), key) != seen.end()) continue;
      seen.push_back(key);
      r += (seen.size() > 1 ? ", \"" : "\"") + key + "\": " + c->tune_choice;
    }
  r += "}}";
  std::snprintf(buf, len, "%s", r.c_str());
  return r.size() < len ? TDDFT_OK : TDDFT_EINVAL;
}

const char* tddft_batch_last_error(const tddft_batch* b) { return b ? b->err.c_str() : "null batch"; }

void tddft_batch_free(tddft_batch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  for (auto* c : b->cells) {
    c->stream = b->stream;
    tddft_free(c);
  }
  for (auto& g : b->groups) {
    if (g.e0) (void)hipEventDestroy(g.e0);
    if (g.e1) (void)hipEventDestroy(g.e1);
  }
  for (auto s : b->side) (void)hipStreamDestroy(s);
  for (auto e : b->side_done) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
  for (void* p : b->allocs) (void)hipFree(p);
  if (b->d_stage) (void)hipFree(b->d_stage);
  if (b->h_stage) (void)hipHostFree(b->h_stage);
  if (b->own_stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

}  // extern "C"
