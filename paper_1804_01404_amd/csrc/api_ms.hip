// C ABI of the learned current surrogate and of the multiscale light
// propagation (Sec. 5, Eqs. Maxwell_ms and TDKS_ms). The cells of the medium
// are a batch of ordinary contexts (tddft_batch_*); the wave equation, the
// surrogate's windows and its network run in the kernels of k_maxwell.hip
// and k_nn.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "internal.h"
#include "tddft.h"

using namespace td;

// ===========================================================================
// surrogate network

struct tddft_nn {
  tddft_nn_config cfg{};
  NNShape sh{};
  long np = 0;
  float *theta = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
  int t_adam = 0;
  bool has_grad = false;
  hipStream_t stream = nullptr;
  int cap = 0;  // batch capacity of the workspace
  float *X = nullptr, *target = nullptr;
  int* idx = nullptr;
  NNWork wk{};
  std::string err;
};

namespace {

tddft_status nn_fail(tddft_nn* n, tddft_status st, const std::string& msg) {
  if (n) n->err = msg;
  return st;
}

#define NHIP(expr)                                                                         \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return nn_fail(n, TDDFT_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename P>
hipError_t nalloc(P** p, size_t count) {
  return hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(count, 1) * sizeof(P));
}

void nn_release_work(tddft_nn* n) {
  for (float* p : {n->X, n->target, n->wk.h1, n->wk.h2, n->wk.y, n->wk.dy, n->wk.dz2, n->wk.dz1, n->wk.loss})
    if (p) (void)hipFree(p);
  if (n->idx) (void)hipFree(n->idx);
  n->X = n->target = nullptr;
  n->idx = nullptr;
  n->wk = NNWork{};
  n->cap = 0;
}

tddft_status nn_reserve(tddft_nn* n, int B) {
  if (B <= n->cap) return TDDFT_OK;
  nn_release_work(n);
  const size_t W = n->sh.W, H = n->sh.H;
  if (nalloc(&n->X, (size_t)B * W) || nalloc(&n->target, B) || nalloc(&n->idx, B) ||
      nalloc(&n->wk.h1, (size_t)B * H) || nalloc(&n->wk.h2, (size_t)B * H) || nalloc(&n->wk.y, B) ||
      nalloc(&n->wk.dy, B) || nalloc(&n->wk.dz2, (size_t)B * H) || nalloc(&n->wk.dz1, (size_t)B * H) ||
      nalloc(&n->wk.loss, 1)) {
    nn_release_work(n);
    return nn_fail(n, TDDFT_ENOMEM, "device allocation failed (network workspace)");
  }
  n->cap = B;
  return TDDFT_OK;
}

tddft_status nn_adam_now(tddft_nn* n, float lr = -1.0f) {
  n->t_adam += 1;
  const double c1 = 1.0 - std::pow((double)n->cfg.beta1, n->t_adam);
  const double c2 = 1.0 - std::pow((double)n->cfg.beta2, n->t_adam);
  NHIP(nn_adam(n->theta, n->m, n->v, n->grad, n->np, lr > 0.0f ? lr : n->cfg.lr, n->cfg.beta1, n->cfg.beta2,
               n->cfg.eps, (float)c1, (float)c2, n->stream));
  return TDDFT_OK;
}

}  // namespace

extern "C" {

int64_t tddft_nn_num_params(int32_t W, int32_t H) {
  return (int64_t)H * W + H + (int64_t)H * H + H + H + 1 + W;
}

tddft_status tddft_nn_create(const tddft_nn_config* cfg, const float* params, tddft_nn** out) {
  if (!out) return TDDFT_EINVAL;
  *out = nullptr;
  if (!cfg || !params) return TDDFT_EINVAL;
  if (cfg->window < 1 || cfg->window > 4096 || cfg->hidden < 1 || cfg->hidden > 1024) return TDDFT_EINVAL;
  if (!(cfg->a_scale != 0.0) || !(cfg->j_scale != 0.0) || !std::isfinite(cfg->a_scale) ||
      !std::isfinite(cfg->j_scale))
    return TDDFT_EINVAL;
  if (!(cfg->lr > 0.0f) || !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) || !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) ||
      !(cfg->eps > 0.0f))
    return TDDFT_EINVAL;
  tddft_nn* n = new tddft_nn();
  n->cfg = *cfg;
  n->sh.W = cfg->window;
  n->sh.H = cfg->hidden;
  n->np = (long)tddft_nn_num_params(cfg->window, cfg->hidden);
  if (hipStreamCreate(&n->stream) != hipSuccess || nalloc(&n->theta, n->np) || nalloc(&n->m, n->np) ||
      nalloc(&n->v, n->np) || nalloc(&n->grad, n->np)) {
    tddft_nn_free(n);
    return TDDFT_ENOMEM;
  }
  if (tddft_nn_set_params(n, params) != TDDFT_OK) {
    tddft_nn_free(n);
    return TDDFT_EDEVICE;
  }
  *out = n;
  return TDDFT_OK;
}

tddft_status tddft_nn_set_params(tddft_nn* n, const float* params) {
  if (!n || !params) return n ? nn_fail(n, TDDFT_EINVAL, "null params") : TDDFT_EINVAL;
  NHIP(hipMemcpyAsync(n->theta, params, n->np * sizeof(float), hipMemcpyHostToDevice, n->stream));
  NHIP(hipMemsetAsync(n->m, 0, n->np * sizeof(float), n->stream));
  NHIP(hipMemsetAsync(n->v, 0, n->np * sizeof(float), n->stream));
  NHIP(hipStreamSynchronize(n->stream));
  n->t_adam = 0;
  n->has_grad = false;
  return TDDFT_OK;
}

tddft_status tddft_nn_get_params(tddft_nn* n, float* params) {
  if (!n || !params) return n ? nn_fail(n, TDDFT_EINVAL, "null params") : TDDFT_EINVAL;
  NHIP(hipMemcpyAsync(params, n->theta, n->np * sizeof(float), hipMemcpyDeviceToHost, n->stream));
  NHIP(hipStreamSynchronize(n->stream));
  return TDDFT_OK;
}

tddft_status tddft_nn_forward(tddft_nn* n, int32_t B, const float* x, float* y) {
  if (!n || !x || !y || B < 1) return n ? nn_fail(n, TDDFT_EINVAL, "bad forward arguments") : TDDFT_EINVAL;
  tddft_status st = nn_reserve(n, B);
  if (st != TDDFT_OK) return st;
  NHIP(hipMemcpyAsync(n->X, x, (size_t)B * n->sh.W * sizeof(float), hipMemcpyHostToDevice, n->stream));
  NHIP(nn_forward(n->sh, n->theta, n->X, B, n->wk, n->stream));
  NHIP(hipMemcpyAsync(y, n->wk.y, (size_t)B * sizeof(float), hipMemcpyDeviceToHost, n->stream));
  NHIP(hipStreamSynchronize(n->stream));
  return TDDFT_OK;
}

tddft_status tddft_nn_loss_grad(tddft_nn* n, int32_t B, const float* x, const float* target, float* loss,
                                float* grad) {
  if (!n || !x || !target || B < 1) return n ? nn_fail(n, TDDFT_EINVAL, "bad loss_grad arguments") : TDDFT_EINVAL;
  tddft_status st = nn_reserve(n, B);
  if (st != TDDFT_OK) return st;
  NHIP(hipMemcpyAsync(n->X, x, (size_t)B * n->sh.W * sizeof(float), hipMemcpyHostToDevice, n->stream));
  NHIP(hipMemcpyAsync(n->target, target, (size_t)B * sizeof(float), hipMemcpyHostToDevice, n->stream));
  NHIP(nn_forward(n->sh, n->theta, n->X, B, n->wk, n->stream));
  NHIP(nn_backward(n->sh, n->theta, n->X, n->target, B, n->wk, n->grad, n->stream));
  if (loss) NHIP(hipMemcpyAsync(loss, n->wk.loss, sizeof(float), hipMemcpyDeviceToHost, n->stream));
  if (grad) NHIP(hipMemcpyAsync(grad, n->grad, n->np * sizeof(float), hipMemcpyDeviceToHost, n->stream));
  NHIP(hipStreamSynchronize(n->stream));
  n->has_grad = true;
  return TDDFT_OK;
}

tddft_status tddft_nn_adam_step(tddft_nn* n) {
  if (!n) return TDDFT_EINVAL;
  if (!n->has_grad) return nn_fail(n, TDDFT_ESTATE, "adam_step before loss_grad");
  tddft_status st = nn_adam_now(n);
  if (st != TDDFT_OK) return st;
  NHIP(hipStreamSynchronize(n->stream));
  return TDDFT_OK;
}

tddft_status tddft_nn_train(tddft_nn* n, int32_t n_traj, int32_t T, const double* A, const double* J,
                            int32_t epochs, int32_t batch, uint64_t seed, float* loss_per_epoch) {
  return tddft_nn_train_ex(n, n_traj, T, A, J, epochs, batch, seed, 0u, loss_per_epoch);
}

tddft_status tddft_nn_fit_linear(tddft_nn* n, int32_t n_traj, int32_t T, const double* A, const double* J,
                                 double a_fit, double lambda_rel) {
  if (!n || !A || !J || n_traj < 1 || T < 1 || !(a_fit > 0.0) || !(lambda_rel >= 0.0) || !std::isfinite(lambda_rel))
    return n ? nn_fail(n, TDDFT_EINVAL, "bad fit_linear arguments") : TDDFT_EINVAL;
  const int W = n->sh.W, H = n->sh.H;
  // trajectories whose largest |A| is within a_fit, scaled as the network sees them
  std::vector<double> hA, hY;
  int used = 0;
  for (int k = 0; k < n_traj; ++k) {
    double amax = 0.0;
    for (int t = 0; t < T; ++t) {
      const double a = A[(size_t)k * T + t], j = J[(size_t)k * T + t];
      if (!std::isfinite(a) || !std::isfinite(j)) return nn_fail(n, TDDFT_EINVAL, "trajectories not finite");
      amax = std::max(amax, std::fabs(a));
    }
    if (amax > a_fit) continue;
    for (int t = 0; t < T; ++t) {
      hA.push_back(A[(size_t)k * T + t] / n->cfg.a_scale);
      hY.push_back(J[(size_t)k * T + t] / n->cfg.j_scale);
    }
    ++used;
  }
  if ((long)used * T < W + 1) return nn_fail(n, TDDFT_EINVAL, "too few samples within a_fit for the linear fit");
  const int nn1 = W + 1;
  double *dA = nullptr, *dY = nullptr, *dG = nullptr, *db = nullptr;
  int* dok = nullptr;
  auto cleanup = [&](tddft_status st) {
    for (double* p : {dA, dY, dG, db})
      if (p) (void)hipFree(p);
    if (dok) (void)hipFree(dok);
    return st;
  };
  if (nalloc(&dA, hA.size()) || nalloc(&dY, hY.size()) || nalloc(&dG, (size_t)nn1 * nn1) || nalloc(&db, nn1) ||
      nalloc(&dok, 1))
    return cleanup(nn_fail(n, TDDFT_ENOMEM, "device allocation failed (linear fit)"));
#define FHIP(expr)                                                                                       do {                                                                                                     hipError_t e_ = (expr);                                                                                if (e_ != hipSuccess) return cleanup(nn_fail(n, TDDFT_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)));   } while (0)
  FHIP(hipMemcpyAsync(dA, hA.data(), hA.size() * sizeof(double), hipMemcpyHostToDevice, n->stream));
  FHIP(hipMemcpyAsync(dY, hY.data(), hY.size() * sizeof(double), hipMemcpyHostToDevice, n->stream));
  // layout: ... w3 [H] at offset H W + H + H H + H, b3 right after, ws last
  const long off_w3 = (long)H * W + H + (long)H * H + H;
  float* w3 = n->theta + off_w3;
  float* b3 = w3 + H;
  float* ws = b3 + 1;
  FHIP(nn_fit_linear(dA, dY, used, T, W, lambda_rel, dG, db, ws, b3, dok, n->stream));
  // the hidden layers start from zero output weight: the network is the fit
  FHIP(nn_zero(w3, H, n->stream));
  FHIP(nn_zero(n->m, n->np, n->stream));
  FHIP(nn_zero(n->v, n->np, n->stream));
  int ok = 0;
  FHIP(hipMemcpyAsync(&ok, dok, sizeof(int), hipMemcpyDeviceToHost, n->stream));
  FHIP(hipStreamSynchronize(n->stream));
#undef FHIP
  n->t_adam = 0;
  n->has_grad = false;
  if (!ok) return cleanup(nn_fail(n, TDDFT_ENUMERIC, "linear fit: the normal equations are not positive definite"));
  return cleanup(TDDFT_OK);
}

tddft_status tddft_nn_train_ex(tddft_nn* n, int32_t n_traj, int32_t T, const double* A, const double* J,
                               int32_t epochs, int32_t batch, uint64_t seed, uint32_t flags, float* loss_per_epoch) {
  if (!n || !A || !J || n_traj < 1 || T < 1 || epochs < 0 || batch < 1 ||
      (flags & ~(uint32_t)(TDDFT_NN_COSINE_LR | TDDFT_NN_FREEZE_LINEAR)))
    return n ? nn_fail(n, TDDFT_EINVAL, "bad train arguments") : TDDFT_EINVAL;
  const long S = (long)n_traj * T;
  if (S > (1L << 30)) return nn_fail(n, TDDFT_EINVAL, "too many samples");
  const int B = (int)std::min<long>(batch, S);
  tddft_status st = nn_reserve(n, B);
  if (st != TDDFT_OK) return st;
  std::vector<float> hA(S), hJ(S);
  for (long i = 0; i < S; ++i) {
    hA[i] = (float)(A[i] / n->cfg.a_scale);
    hJ[i] = (float)(J[i] / n->cfg.j_scale);
  }
  float *dA = nullptr, *dJ = nullptr, *dloss = nullptr;
  int* dperm = nullptr;
  auto cleanup = [&](tddft_status s) {
    if (dA) (void)hipFree(dA);
    if (dJ) (void)hipFree(dJ);
    if (dloss) (void)hipFree(dloss);
    if (dperm) (void)hipFree(dperm);
    return s;
  };
  if (nalloc(&dA, S) || nalloc(&dJ, S) || nalloc(&dperm, S) || nalloc(&dloss, std::max(epochs, 1)))
    return cleanup(nn_fail(n, TDDFT_ENOMEM, "device allocation failed (training set)"));
#define THIP(expr)                                                                                     \
  do {                                                                                                 \
    hipError_t e_ = (expr);                                                                            \
    if (e_ != hipSuccess) return cleanup(nn_fail(n, TDDFT_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_))); \
  } while (0)
  THIP(hipMemcpyAsync(dA, hA.data(), S * sizeof(float), hipMemcpyHostToDevice, n->stream));
  THIP(hipMemcpyAsync(dJ, hJ.data(), S * sizeof(float), hipMemcpyHostToDevice, n->stream));
  THIP(hipMemsetAsync(dloss, 0, std::max(epochs, 1) * sizeof(float), n->stream));
  std::vector<int> perm(S);
  std::vector<int> n_batches(std::max(epochs, 1), 0);
  for (int ep = 0; ep < epochs; ++ep) {
    for (long i = 0; i < S; ++i) perm[i] = (int)i;
    std::mt19937_64 rng(seed * 0x9E3779B97F4A7C15ULL + (uint64_t)ep);
    for (long i = S - 1; i > 0; --i) {  // Fisher-Yates with an explicit draw
      const long j = (long)(rng() % (uint64_t)(i + 1));
      std::swap(perm[i], perm[j]);
    }
    THIP(hipStreamSynchronize(n->stream));  // perm is reused across epochs
    THIP(hipMemcpyAsync(dperm, perm.data(), S * sizeof(int), hipMemcpyHostToDevice, n->stream));
    for (long off = 0; off < S; off += B) {
      const int b = (int)std::min<long>(B, S - off);
      THIP(nn_gather(dA, dJ, T, n->sh.W, dperm + off, b, n->X, n->target, n->stream));
      THIP(nn_forward(n->sh, n->theta, n->X, b, n->wk, n->stream));
      THIP(nn_backward(n->sh, n->theta, n->X, n->target, b, n->wk, n->grad, n->stream));
      THIP(nn_accumulate(n->wk.loss, dloss + ep, n->stream));
      if (flags & TDDFT_NN_FREEZE_LINEAR)  // b3 and ws are the last W + 1 parameters
        THIP(nn_zero(n->grad + n->np - (n->sh.W + 1), n->sh.W + 1, n->stream));
      const float lr = (flags & TDDFT_NN_COSINE_LR)
                           ? (float)(0.5 * n->cfg.lr * (1.0 + std::cos(M_PI * (double)ep / (double)epochs)))
                           : n->cfg.lr;
      st = nn_adam_now(n, lr);
      if (st != TDDFT_OK) return cleanup(st);
      ++n_batches[ep];
    }
  }
  std::vector<float> el(std::max(epochs, 1));
  THIP(hipMemcpyAsync(el.data(), dloss, el.size() * sizeof(float), hipMemcpyDeviceToHost, n->stream));
  THIP(hipStreamSynchronize(n->stream));
#undef THIP
  if (loss_per_epoch)
    for (int ep = 0; ep < epochs; ++ep) loss_per_epoch[ep] = el[ep] / (float)std::max(n_batches[ep], 1);
  n->has_grad = true;
  return cleanup(TDDFT_OK);
}

const char* tddft_nn_last_error(const tddft_nn* n) { return n ? n->err.c_str() : "null network"; }

void tddft_nn_free(tddft_nn* n) {
  if (!n) return;
  if (n->stream) (void)hipStreamSynchronize(n->stream);
  nn_release_work(n);
  for (float* p : {n->theta, n->m, n->v, n->grad})
    if (p) (void)hipFree(p);
  if (n->stream) (void)hipStreamDestroy(n->stream);
  delete n;
}

}  // extern "C"

// ===========================================================================
// multiscale

struct tddft_ms {
  tddft_ms_config cfg{};
  tddft_config cell{};
  std::vector<double> kpt, kw, psi0, vloc;
  struct AtomCopy {
    std::vector<int32_t> idx;
    std::vector<double> x, beta, e_kb;
    int32_t npts = 0, n_proj = 0;
  };
  std::vector<AtomCopy> atoms;
  tddft_batch* full = nullptr;  // every medium point
  tddft_batch* sent = nullptr;  // sentinel points (surrogate mode)
  hipStream_t stream = nullptr;
  double *A[3] = {nullptr, nullptr, nullptr};  // prev, now, new (rotating)
  double* I = nullptr;                          // [n_x]
  double* Iold = nullptr;                       // [n_x] the current of the previous step
  double* energy = nullptr;                     // [2]: work on the medium, field energy (per area)
  int steps = 0;
  int mode = 0;  // 0 cells, 1 network
  int fallbacks = 0;
  double last_check = 0.0;
  std::vector<double> hist;  // cells mode: medium A at t_0 .. t_steps, [steps + 1][n_mat]
  // surrogate mode
  tddft_nn* nn = nullptr;
  double a_max = 0, tol = 0;
  std::vector<int> sentinels;
  int check_every = 0, checked_to = 0;
  float *ring = nullptr, *Xw = nullptr;
  NNWork wk{};
  int* flag = nullptr;
  double *dhist = nullptr, *dIhist = nullptr;  // [cap][n_mat] medium A and I per step
  int hist_cap = 0;
  // the A and I rows of one tddft_ms_step call, staged on the device and
  // copied to the caller once at its end ([out_cap][n_x] each)
  double *dAout = nullptr, *dIout = nullptr;
  int out_cap = 0;
  std::string err;
};

namespace {

tddft_status ms_fail(tddft_ms* ms, tddft_status st, const std::string& msg) {
  if (ms) ms->err = msg;
  return st;
}

#define MHIP(expr)                                                                        \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return ms_fail(ms, TDDFT_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

std::vector<tddft_atom> ms_atoms(const tddft_ms* ms) {
  std::vector<tddft_atom> out(ms->atoms.size());
  for (size_t a = 0; a < ms->atoms.size(); ++a) {
    const auto& c = ms->atoms[a];
    out[a].npts = c.npts;
    out[a].n_proj = c.n_proj;
    out[a].idx = c.idx.data();
    out[a].x = c.x.data();
    out[a].beta = c.beta.data();
    out[a].e_kb = c.e_kb.data();
  }
  return out;
}

tddft_status ms_make_batch(tddft_ms* ms, int n_cells, tddft_batch** out) {
  std::vector<tddft_config> cfgs(n_cells, ms->cell);
  std::vector<const double*> ps(n_cells, ms->psi0.data());
  tddft_status st = tddft_batch_create(n_cells, cfgs.data(), ps.data(), out);
  if (st != TDDFT_OK) return ms_fail(ms, st, "cell batch: creation failed");
  std::vector<tddft_atom> at = ms_atoms(ms);
  for (int c = 0; c < n_cells; ++c) {
    st = tddft_batch_set_potential(*out, c, ms->vloc.data(), (int32_t)at.size(), at.data());
    if (st != TDDFT_OK) return ms_fail(ms, st, std::string("cell batch: ") + tddft_batch_last_error(*out));
  }
  return TDDFT_OK;
}

// propagate `b` (cells for the medium indices `which`) through macroscopic
// steps s0 .. s1 - 1 of the medium history `h` ([.][n_mat], row s = t_s);
// returns the cell currents along the axis at t_{s0+1} .. t_{s1}: [s1 - s0][which]
tddft_status ms_run_cells(tddft_ms* ms, tddft_batch* b, const std::vector<int>& which, const std::vector<double>& h,
                          int s0, int s1, std::vector<double>& I_out) {
  const int nm = ms->cfg.n_mat, ns = ms->cfg.n_sub, ax = ms->cfg.axis;
  const int nsteps = (s1 - s0) * ns;
  const int nc = (int)which.size();
  std::vector<std::vector<double>> tab(nc, std::vector<double>((size_t)(nsteps + 1) * 3, 0.0));
  std::vector<std::vector<double>> J(nc, std::vector<double>((size_t)nsteps * 3, 0.0));
  for (int c = 0; c < nc; ++c) {
    const int m = which[c];
    for (int s = s0; s < s1; ++s) {
      const double a0 = h[(size_t)s * nm + m], a1 = h[(size_t)(s + 1) * nm + m];
      for (int u = 0; u <= ns; ++u) {
        if (u == ns && s + 1 < s1) continue;  // the next step writes its start
        tab[c][((size_t)(s - s0) * ns + u) * 3 + ax] = a0 + ((double)u / ns) * (a1 - a0);
      }
    }
  }
  std::vector<const double*> tp(nc);
  std::vector<double*> jp(nc);
  for (int c = 0; c < nc; ++c) {
    tp[c] = tab[c].data();
    jp[c] = J[c].data();
  }
  tddft_status st = tddft_batch_propagate(b, nsteps, tp.data(), jp.data());
  if (st != TDDFT_OK) return ms_fail(ms, st, std::string("cells: ") + tddft_batch_last_error(b));
  I_out.assign((size_t)(s1 - s0) * nc, 0.0);
  for (int c = 0; c < nc; ++c)
    for (int s = s0; s < s1; ++s) I_out[(size_t)(s - s0) * nc + c] = J[c][((size_t)(s - s0 + 1) * ns - 1) * 3 + ax];
  return TDDFT_OK;
}

tddft_status ms_reserve_hist(tddft_ms* ms, int need) {
  if (need <= ms->hist_cap) return TDDFT_OK;
  const int cap = std::max(need, 2 * ms->hist_cap + 64);
  const size_t nm = ms->cfg.n_mat;
  double *h = nullptr, *hi = nullptr;
  if (nalloc(&h, (size_t)cap * nm) || nalloc(&hi, (size_t)cap * nm)) {
    if (h) (void)hipFree(h);
    return ms_fail(ms, TDDFT_ENOMEM, "device allocation failed (history)");
  }
  MHIP(hipMemsetAsync(h, 0, (size_t)cap * nm * sizeof(double), ms->stream));
  MHIP(hipMemsetAsync(hi, 0, (size_t)cap * nm * sizeof(double), ms->stream));
  if (ms->dhist) {
    MHIP(hipMemcpyAsync(h, ms->dhist, (size_t)ms->hist_cap * nm * sizeof(double), hipMemcpyDeviceToDevice,
                        ms->stream));
    MHIP(hipMemcpyAsync(hi, ms->dIhist, (size_t)ms->hist_cap * nm * sizeof(double), hipMemcpyDeviceToDevice,
                        ms->stream));
    MHIP(hipStreamSynchronize(ms->stream));
    (void)hipFree(ms->dhist);
    (void)hipFree(ms->dIhist);
  }
  ms->dhist = h;
  ms->dIhist = hi;
  ms->hist_cap = cap;
  return TDDFT_OK;
}

// switch every medium point to its cell: replay the A history from t = 0
tddft_status ms_fallback(tddft_ms* ms) {
  const int nm = ms->cfg.n_mat;
  std::vector<double> h((size_t)(ms->steps + 1) * nm);
  MHIP(hipMemcpyAsync(h.data(), ms->dhist, h.size() * sizeof(double), hipMemcpyDeviceToHost, ms->stream));
  MHIP(hipStreamSynchronize(ms->stream));
  tddft_status st;
  if (!ms->full && (st = ms_make_batch(ms, nm, &ms->full)) != TDDFT_OK) return st;
  std::vector<int> all(nm);
  for (int m = 0; m < nm; ++m) all[m] = m;
  std::vector<double> Ic;
  if (ms->steps > 0) {
    st = ms_run_cells(ms, ms->full, all, h, 0, ms->steps, Ic);
    if (st != TDDFT_OK) return st;
  } else {
    Ic.assign(nm, 0.0);
  }
  std::vector<double> I(ms->cfg.n_x, 0.0);
  const size_t last = ms->steps > 0 ? (size_t)(ms->steps - 1) * nm : 0;
  for (int m = 0; m < nm; ++m) I[ms->cfg.x0 + m] = ms->steps > 0 ? Ic[last + m] : 0.0;
  MHIP(hipMemcpyAsync(ms->I, I.data(), I.size() * sizeof(double), hipMemcpyHostToDevice, ms->stream));
  // the work on the medium, again from the cells' currents (I = 0 at t_0)
  if (ms->steps > 0) {
    std::vector<double> Ih((size_t)(ms->steps + 1) * nm, 0.0);
    std::copy(Ic.begin(), Ic.end(), Ih.begin() + nm);
    double *dA = nullptr, *dI = nullptr;
    if (nalloc(&dA, h.size()) || nalloc(&dI, Ih.size())) {
      if (dA) (void)hipFree(dA);
      return ms_fail(ms, TDDFT_ENOMEM, "device allocation failed (work history)");
    }
    hipError_t e = hipMemcpyAsync(dA, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, ms->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(dI, Ih.data(), Ih.size() * sizeof(double), hipMemcpyHostToDevice, ms->stream);
    if (e == hipSuccess)
      e = launch_ms_work_history(dA, dI, ms->steps, nm, ms->cfg.dx, ms->cfg.dt, ms->energy, ms->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ms->stream);
    (void)hipFree(dA);
    (void)hipFree(dI);
    if (e != hipSuccess) return ms_fail(ms, TDDFT_EDEVICE, std::string("work history: ") + hipGetErrorString(e));
  }
  MHIP(hipStreamSynchronize(ms->stream));
  ms->hist = h;
  ms->mode = 0;
  ms->fallbacks += 1;
  return TDDFT_OK;
}

// compare the sentinel cells with the network over steps checked_to .. steps
tddft_status ms_check(tddft_ms* ms, bool* trip) {
  *trip = false;
  int flag = 0;
  MHIP(hipMemcpyAsync(&flag, ms->flag, sizeof(int), hipMemcpyDeviceToHost, ms->stream));
  MHIP(hipStreamSynchronize(ms->stream));
  if (flag) {
    ms->last_check = INFINITY;
    *trip = true;
    return TDDFT_OK;
  }
  if (ms->sentinels.empty() || ms->steps <= ms->checked_to) return TDDFT_OK;
  const int nm = ms->cfg.n_mat;
  const int s0 = ms->checked_to, s1 = ms->steps;
  std::vector<double> h((size_t)(s1 + 1) * nm), In((size_t)(s1 + 1) * nm);
  MHIP(hipMemcpyAsync(h.data(), ms->dhist, h.size() * sizeof(double), hipMemcpyDeviceToHost, ms->stream));
  MHIP(hipMemcpyAsync(In.data(), ms->dIhist, In.size() * sizeof(double), hipMemcpyDeviceToHost, ms->stream));
  MHIP(hipStreamSynchronize(ms->stream));
  std::vector<double> Ic;
  tddft_status st = ms_run_cells(ms, ms->sent, ms->sentinels, h, s0, s1, Ic);
  if (st != TDDFT_OK) return st;
  const int nc = (int)ms->sentinels.size();
  double err = 0.0;
  for (int s = s0; s < s1; ++s)
    for (int c = 0; c < nc; ++c) {
      const double ic = Ic[(size_t)(s - s0) * nc + c];
      err = std::max(err, std::fabs(In[(size_t)(s + 1) * nm + ms->sentinels[c]] - ic));
    }
  // relative to the network's output scale: early in a run the cells' current
  // is near zero and a ratio to it would flag rounding-size differences
  ms->last_check = err / std::fabs(ms->nn->cfg.j_scale);
  ms->checked_to = s1;
  if (!(ms->last_check <= ms->tol)) *trip = true;
  return TDDFT_OK;
}

}  // namespace

extern "C" {

tddft_status tddft_ms_create(const tddft_ms_config* cfg, const tddft_config* cell, const double* psi0,
                             const double* v_loc, int32_t n_atoms, const tddft_atom* atoms, tddft_ms** out) {
  if (!out) return TDDFT_EINVAL;
  *out = nullptr;
  if (!cfg || !cell || !psi0 || !v_loc || n_atoms < 0 || (n_atoms > 0 && !atoms)) return TDDFT_EINVAL;
  if (cfg->n_x < 4 || cfg->n_mat < 1 || cfg->x0 < 1 || cfg->x0 + cfg->n_mat > cfg->n_x - 1) return TDDFT_EINVAL;
  if (!(cfg->dx > 0.0) || !(cfg->dt > 0.0) || cfg->n_sub < 1 || cfg->axis < 0 || cfg->axis > 2) return TDDFT_EINVAL;
  if (kC * cfg->dt / cfg->dx > 1.0 + 1e-12) return TDDFT_EINVAL;  // Courant condition of the leapfrog
  if (std::fabs(cell->dt - cfg->dt / cfg->n_sub) > 1e-12 * std::fabs(cfg->dt)) return TDDFT_EINVAL;
  if (cell->n_k < 1 || cell->n_orb < 1 || !cell->kpt || !cell->kw) return TDDFT_EINVAL;
  tddft_ms* ms = new tddft_ms();
  ms->cfg = *cfg;
  ms->cell = *cell;
  ms->kpt.assign(cell->kpt, cell->kpt + 3 * cell->n_k);
  ms->kw.assign(cell->kw, cell->kw + cell->n_k);
  ms->cell.kpt = ms->kpt.data();
  ms->cell.kw = ms->kw.data();
  ms->cell.stream = nullptr;
  const size_t N = (size_t)cell->n[0] * cell->n[1] * cell->n[2];
  ms->psi0.assign(psi0, psi0 + 2 * N * cell->n_orb * cell->n_k);
  ms->vloc.assign(v_loc, v_loc + N);
  ms->atoms.resize(n_atoms);
  for (int a = 0; a < n_atoms; ++a) {
    auto& c = ms->atoms[a];
    const tddft_atom& s = atoms[a];
    if (s.npts < 1 || s.n_proj < 1 || s.n_proj > kMaxProj || !s.idx || !s.x || !s.beta || !s.e_kb) {
      delete ms;
      return TDDFT_EINVAL;
    }
    c.npts = s.npts;
    c.n_proj = s.n_proj;
    c.idx.assign(s.idx, s.idx + s.npts);
    c.x.assign(s.x, s.x + 3 * (size_t)s.npts);
    c.beta.assign(s.beta, s.beta + (size_t)s.n_proj * s.npts);
    c.e_kb.assign(s.e_kb, s.e_kb + s.n_proj);
  }
  auto bad = [&](tddft_status st) {
    tddft_ms_free(ms);
    return st;
  };
  if (hipStreamCreate(&ms->stream) != hipSuccess) return bad(TDDFT_EDEVICE);
  const size_t nx = cfg->n_x;
  if (nalloc(&ms->A[0], nx) || nalloc(&ms->A[1], nx) || nalloc(&ms->A[2], nx) || nalloc(&ms->I, nx) ||
      nalloc(&ms->Iold, nx) || nalloc(&ms->energy, 2) || nalloc(&ms->flag, 1))
    return bad(TDDFT_ENOMEM);
  for (double* p : {ms->A[0], ms->A[1], ms->A[2], ms->I, ms->Iold})
    if (hipMemsetAsync(p, 0, nx * sizeof(double), ms->stream) != hipSuccess) return bad(TDDFT_EDEVICE);
  if (hipMemsetAsync(ms->energy, 0, 2 * sizeof(double), ms->stream) != hipSuccess) return bad(TDDFT_EDEVICE);
  if (hipMemsetAsync(ms->flag, 0, sizeof(int), ms->stream) != hipSuccess ||
      hipStreamSynchronize(ms->stream) != hipSuccess)
    return bad(TDDFT_EDEVICE);
  ms->hist.assign((size_t)cfg->n_mat, 0.0);  // A = 0 at t_0
  *out = ms;
  return TDDFT_OK;
}

tddft_status tddft_ms_attach_surrogate(tddft_ms* ms, tddft_nn* nn, double a_max, int32_t n_sentinel,
                                       const int32_t* sentinels, int32_t check_every, double tol) {
  if (!ms) return TDDFT_EINVAL;
  if (ms->steps > 0 || ms->full || ms->nn) return ms_fail(ms, TDDFT_ESTATE, "attach_surrogate after the first step");
  if (!nn || !(a_max > 0.0) || n_sentinel < 0 || (n_sentinel > 0 && !sentinels) || check_every < 1 || !(tol > 0.0))
    return ms_fail(ms, TDDFT_EINVAL, "bad surrogate arguments");
  for (int i = 0; i < n_sentinel; ++i)
    if (sentinels[i] < 0 || sentinels[i] >= ms->cfg.n_mat) return ms_fail(ms, TDDFT_EINVAL, "sentinel out of range");
  ms->nn = nn;
  ms->a_max = a_max;
  ms->tol = tol;
  ms->check_every = check_every;
  ms->sentinels.assign(sentinels, sentinels + n_sentinel);
  const size_t nm = ms->cfg.n_mat, W = nn->sh.W, H = nn->sh.H;
  if (nalloc(&ms->ring, nm * W) || nalloc(&ms->Xw, nm * W) || nalloc(&ms->wk.h1, nm * H) ||
      nalloc(&ms->wk.h2, nm * H) || nalloc(&ms->wk.y, nm))
    return ms_fail(ms, TDDFT_ENOMEM, "device allocation failed (surrogate)");
  MHIP(hipMemsetAsync(ms->ring, 0, nm * W * sizeof(float), ms->stream));
  tddft_status st = ms_reserve_hist(ms, 256);
  if (st != TDDFT_OK) return st;
  if (n_sentinel > 0 && (st = ms_make_batch(ms, n_sentinel, &ms->sent)) != TDDFT_OK) return st;
  MHIP(hipStreamSynchronize(ms->stream));
  ms->mode = 1;
  return TDDFT_OK;
}

tddft_status tddft_ms_step(tddft_ms* ms, int32_t n_macro, const double* inc, double* A_out, double* I_out) {
  if (!ms) return TDDFT_EINVAL;
  if (n_macro < 0) return ms_fail(ms, TDDFT_EINVAL, "negative step count");
  const auto& g = ms->cfg;
  const int nx = g.n_x, nm = g.n_mat;
  const double S = kC * g.dt / g.dx;
  const double S2 = S * S, src = 4.0 * M_PI * kC * g.dt * g.dt, q = (S - 1.0) / (S + 1.0);
  tddft_status st;
  if (ms->mode == 0 && !ms->full && (st = ms_make_batch(ms, nm, &ms->full)) != TDDFT_OK) return st;
  if ((A_out || I_out) && n_macro > ms->out_cap) {
    MHIP(hipStreamSynchronize(ms->stream));
    if (ms->dAout) (void)hipFree(ms->dAout);
    if (ms->dIout) (void)hipFree(ms->dIout);
    ms->dAout = ms->dIout = nullptr;
    ms->out_cap = 0;
    if (nalloc(&ms->dAout, (size_t)n_macro * nx) || nalloc(&ms->dIout, (size_t)n_macro * nx))
      return ms_fail(ms, TDDFT_ENOMEM, "device allocation failed (output rows)");
    ms->out_cap = n_macro;
  }
  std::vector<double> Anew(nx), Inew(nx);
  const std::vector<int> all = [&] {
    std::vector<int> v(nm);
    for (int m = 0; m < nm; ++m) v[m] = m;
    return v;
  }();
  for (int n = 0; n < n_macro; ++n) {
    const double iv[4] = {inc ? inc[2 * n] : 0.0, inc ? inc[2 * n + 1] : 0.0, inc ? inc[2 * n + 2] : 0.0,
                          inc ? inc[2 * n + 3] : 0.0};
    MHIP(launch_fdtd_step(ms->A[1], ms->A[0], ms->I, ms->A[2], nx, S2, src, q, iv, ms->stream));
    MHIP(hipMemcpyAsync(ms->Iold, ms->I, nx * sizeof(double), hipMemcpyDeviceToDevice, ms->stream));
    if (ms->mode == 0) {
      MHIP(hipMemcpyAsync(Anew.data(), ms->A[2], nx * sizeof(double), hipMemcpyDeviceToHost, ms->stream));
      MHIP(hipStreamSynchronize(ms->stream));
      const size_t row = ms->hist.size();
      ms->hist.resize(row + nm);
      for (int m = 0; m < nm; ++m) ms->hist[row + m] = Anew[g.x0 + m];
      std::vector<double> Ic;
      st = ms_run_cells(ms, ms->full, all, ms->hist, ms->steps, ms->steps + 1, Ic);
      if (st != TDDFT_OK) return st;
      std::fill(Inew.begin(), Inew.end(), 0.0);
      for (int m = 0; m < nm; ++m) Inew[g.x0 + m] = Ic[m];
      MHIP(hipMemcpyAsync(ms->I, Inew.data(), nx * sizeof(double), hipMemcpyHostToDevice, ms->stream));
    } else {
      const int slot = (ms->steps + 1) % ms->nn->sh.W;
      if ((st = ms_reserve_hist(ms, ms->steps + 2)) != TDDFT_OK) return st;
      MHIP(launch_ms_gate(ms->A[2], g.x0, nm, ms->a_max, ms->flag, ms->stream));
      MHIP(hipMemcpyAsync(ms->dhist + (size_t)(ms->steps + 1) * nm, ms->A[2] + g.x0, nm * sizeof(double),
                          hipMemcpyDeviceToDevice, ms->stream));
      MHIP(launch_ring_push(ms->A[2], g.x0, nm, ms->ring, ms->nn->sh.W, slot, 1.0 / ms->nn->cfg.a_scale, ms->stream));
      MHIP(launch_ring_windows(ms->ring, nm, ms->nn->sh.W, slot, ms->Xw, ms->stream));
      MHIP(nn_forward(ms->nn->sh, ms->nn->theta, ms->Xw, nm, ms->wk, ms->stream));
      MHIP(launch_scatter_current(ms->wk.y, g.x0, nm, nx, ms->nn->cfg.j_scale, ms->I, ms->stream));
      MHIP(hipMemcpyAsync(ms->dIhist + (size_t)(ms->steps + 1) * nm, ms->I + g.x0, nm * sizeof(double),
                          hipMemcpyDeviceToDevice, ms->stream));
    }
    MHIP(launch_ms_work_step(ms->A[2], ms->A[1], ms->Iold, ms->I, g.x0, nm, g.dx, g.dt, ms->energy, ms->stream));
    if (A_out)
      MHIP(hipMemcpyAsync(ms->dAout + (size_t)n * nx, ms->A[2], nx * sizeof(double), hipMemcpyDeviceToDevice,
                          ms->stream));
    if (I_out)
      MHIP(hipMemcpyAsync(ms->dIout + (size_t)n * nx, ms->I, nx * sizeof(double), hipMemcpyDeviceToDevice,
                          ms->stream));
    double* t = ms->A[0];
    ms->A[0] = ms->A[1];
    ms->A[1] = ms->A[2];
    ms->A[2] = t;
    ms->steps += 1;
    if (ms->mode == 1 && (ms->steps % ms->check_every == 0 || n == n_macro - 1)) {
      bool trip = false;
      if ((st = ms_check(ms, &trip)) != TDDFT_OK) return st;
      if (trip) {
        if ((st = ms_fallback(ms)) != TDDFT_OK) return st;
        if (I_out)  // the current of this step now comes from the cells
          MHIP(hipMemcpyAsync(ms->dIout + (size_t)n * nx, ms->I, nx * sizeof(double), hipMemcpyDeviceToDevice,
                              ms->stream));
      }
    }
  }
  if (A_out && n_macro > 0)
    MHIP(hipMemcpyAsync(A_out, ms->dAout, (size_t)n_macro * nx * sizeof(double), hipMemcpyDeviceToHost, ms->stream));
  if (I_out && n_macro > 0)
    MHIP(hipMemcpyAsync(I_out, ms->dIout, (size_t)n_macro * nx * sizeof(double), hipMemcpyDeviceToHost, ms->stream));
  MHIP(hipStreamSynchronize(ms->stream));
  return TDDFT_OK;
}

tddft_status tddft_ms_status(tddft_ms* ms, int32_t* mode, int32_t* fallbacks, double* last_check,
                             int32_t* steps_done) {
  if (!ms) return TDDFT_EINVAL;
  if (mode) *mode = ms->mode;
  if (fallbacks) *fallbacks = ms->fallbacks;
  if (last_check) *last_check = ms->last_check;
  if (steps_done) *steps_done = ms->steps;
  return TDDFT_OK;
}

tddft_status tddft_ms_energy(tddft_ms* ms, double* em, double* work) {
  if (!ms) return TDDFT_EINVAL;
  MHIP(launch_em_energy(ms->A[1], ms->A[0], ms->cfg.n_x, ms->cfg.dx, ms->cfg.dt, ms->energy + 1, ms->stream));
  double v[2];
  MHIP(hipMemcpyAsync(v, ms->energy, sizeof(v), hipMemcpyDeviceToHost, ms->stream));
  MHIP(hipStreamSynchronize(ms->stream));
  if (work) *work = v[0];
  if (em) *em = v[1];
  return TDDFT_OK;
}

const char* tddft_ms_last_error(const tddft_ms* ms) { return ms ? ms->err.c_str() : "null multiscale run"; }

void tddft_ms_free(tddft_ms* ms) {
  if (!ms) return;
  if (ms->stream) (void)hipStreamSynchronize(ms->stream);
  if (ms->full) tddft_batch_free(ms->full);
  if (ms->sent) tddft_batch_free(ms->sent);
  for (double* p : {ms->A[0], ms->A[1], ms->A[2], ms->I, ms->Iold, ms->energy, ms->dhist, ms->dIhist, ms->dAout,
                    ms->dIout})
    if (p) (void)hipFree(p);
  for (float* p : {ms->ring, ms->Xw, ms->wk.h1, ms->wk.h2, ms->wk.y})
    if (p) (void)hipFree(p);
  if (ms->flag) (void)hipFree(ms->flag);
  if (ms->stream) (void)hipStreamDestroy(ms->stream);
  delete ms;
}

}  // extern "C"
