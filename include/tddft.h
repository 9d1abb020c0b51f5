/*
 * tddft.h - C ABI of the real-time, real-space TDKS time step on one MI355X.
 *
 * The library evolves Kohn-Sham Bloch orbitals w_nk on a uniform grid over a
 * cuboid cell with the fourth-order truncated Taylor expansion of
 * exp(-i dt h) (Program Summary of the paper), where
 *
 *   h w = 1/2 (-i grad + k + A/c)^2 w + (V_loc + V_H + V_xc) w + V_NL w
 *
 * (Sec. 4.1, Eq. TDKS_solid; Sec. 3.1, Eq. TDKS with V_ext = E.r in the
 * isolated length gauge). The Laplacian and gradient are 9-point-per-axis
 * central differences; V_NL is the separable Kleinman-Bylander form with the
 * phase exp(-i (k + A/c).x) that keeps the nonlocal term gauge invariant
 * (Sec. 4.1). After every step the library forms the density (Eq. rho), the
 * macroscopic current (Eq. macro_current, nonlocal part included) and updates
 * the Hartree and adiabatic LDA (Perdew-Zunger) potentials (Sec. 3.1).
 *
 * Units: atomic (Hartree, bohr, hbar = m = e = 1), c = 137.035999084.
 *
 * Conventions shared by every entry point:
 *  - Grid arrays are [n3][n2][n1] with x fastest; the flat index of point
 *    (i1, i2, i3) is (i3 * n2 + i2) * n1 + i1. Periodic grids sit at r = j h,
 *    isolated grids at r = (j - (N - 1) / 2) h with w = 0 outside the box.
 *  - Orbitals are [n_k][n_orb][n3][n2][n1] complex128, interleaved (re, im)
 *    doubles, normalised to one with the weight h1 h2 h3.
 *  - Every pointer argument is a HOST pointer, borrowed for the duration of
 *    the call only; the library copies what it needs. Output buffers are
 *    owned by the caller.
 *  - Every call returns a status; none aborts or exits. tddft_last_error()
 *    gives the message of the last failure on a context. After
 *    TDDFT_EDEVICE or TDDFT_ENUMERIC the context is poisoned: only
 *    tddft_last_error and tddft_free remain valid on it.
 *  - One context per thread; separate contexts are independent.
 */
#ifndef TDDFT_H
#define TDDFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TDDFT_ABI_VERSION 1u

typedef struct tddft_ctx tddft_ctx;

typedef enum {
  TDDFT_OK = 0,
  TDDFT_EINVAL = 1,    /* bad argument or configuration                       */
  TDDFT_ENOMEM = 2,    /* device allocation failed                            */
  TDDFT_EDEVICE = 3,   /* a HIP call failed (context poisoned)                */
  TDDFT_EUNSTABLE = 4, /* dt * |lambda|max(h) > 2 sqrt 2: the Taylor step grows */
  TDDFT_ESTATE = 5,    /* call out of order (e.g. propagate before set_potential) */
  TDDFT_ENUMERIC = 6   /* NaN or Inf in the orbitals (context poisoned)       */
} tddft_status;

enum { TDDFT_PERIODIC = 0, TDDFT_ISOLATED = 1 };
enum { TDDFT_C128 = 0, TDDFT_MIXED = 1 };        /* precision of the orbital stream */
enum { TDDFT_VELOCITY = 0, TDDFT_LENGTH = 1 };   /* gauge of the applied field     */
/* Exchange-correlation potential (Sec. 3.1: adiabatic LDA; Sec. 4.1: the
 * Becke-Johnson potential and the Tran-Blaha variant as alternatives).
 * TDDFT_XC_TB09 and TDDFT_XC_BJ use the exchange potential
 *   v_x = c v_BR + (3c - 2)(1/pi) sqrt(5/12) sqrt(2 t_s / rho_s)
 * with the Becke-Roussel hole potential v_BR (gamma = 1), rho_s = rho/2 and
 * t_s = tau/2, tau = sum_k w_k sum_n |(grad_h + i kappa_k) w_nk|^2 from the
 * orbitals (kappa_k = k + A/c at the orbitals' time; k in the length gauge),
 * grad rho and lap rho by the same 9-point differences, v_x = 0 where
 * rho < 1e-30; plus PZ81 correlation. TB09: c = -0.012 + 1.023 sqrt(g),
 * g = (1/Omega) int |grad rho| / rho, re-evaluated with every potential
 * update; BJ: c = 1. These potentials have no energy functional: the energy
 * reports the LDA exchange-correlation energy of the density. */
enum { TDDFT_XC_NONE = 0, TDDFT_XC_PZ81 = 1, TDDFT_XC_TB09 = 2, TDDFT_XC_BJ = 3 };

#define TDDFT_FLAG_ALLOW_UNSTABLE 0x1u /* skip the Taylor stability refusal      */
#define TDDFT_FLAG_DEBUG_SYNC 0x2u     /* synchronise and check after each kernel */
#define TDDFT_FLAG_NO_GRAPH 0x4u       /* launch kernels directly, no hipGraph    */
#define TDDFT_FLAG_STREAMING 0x8u      /* one kernel per Horner stage even when the
                                          orbital fits in LDS (the fused step) */
#define TDDFT_FLAG_PREDICTOR_CORRECTOR 0x20u /* Program Summary ("a predictor-corrector
                                          step when necessary"): each step is first
                                          predicted under V(t_n); the density of the
                                          prediction gives V(t_{n+1}), and the step is
                                          redone from t_n under (V(t_n) + V(t_{n+1})) / 2.
                                          Twice the work per step; one more copy of
                                          the orbitals in device memory */
#define TDDFT_FLAG_NORM_WATCHDOG 0x40u /* failure detection: propagate returns
                                          ENUMERIC (and poisons the context) once an
                                          orbital norm is further than 1e-3 from 1.
                                          The fourth-order step conserves norms to
                                          about 1e-6 per 1000 steps within its
                                          stability bound, so a trip means growth
                                          (ALLOW_UNSTABLE) or corrupted state */

typedef struct {
  uint32_t abi_version;   /* TDDFT_ABI_VERSION                                  */
  uint32_t struct_size;   /* sizeof(tddft_config)                                */
  int32_t n[3];           /* grid points along x, y, z; each >= 8                */
  double cell[3];         /* box lengths (bohr); h = cell / n                    */
  int32_t boundary;       /* TDDFT_PERIODIC or TDDFT_ISOLATED                     */
  int32_t n_orb;          /* doubly occupied orbitals per k-point (>= 1)         */
  int32_t n_k;            /* k-points (>= 1; isolated: 1)                        */
  const double *kpt;      /* [n_k][3] bohr^-1 (host, borrowed)                   */
  const double *kw;       /* [n_k] weights summing to 1 (host, borrowed)         */
  double dt;              /* time step (a.u.), nonzero; negative runs backwards  */
  int32_t precision;      /* TDDFT_C128, or TDDFT_MIXED: complex FP32 orbitals,
                             stencil and Taylor terms; FP64 density, current,
                             Poisson solve, norms and projector inner products */
  int32_t hartree;        /* 0 off, 1 on                                          */
  int32_t xc;             /* TDDFT_XC_NONE, _PZ81, _TB09 or _BJ                   */
  int32_t gauge;          /* TDDFT_VELOCITY, or TDDFT_LENGTH (isolated only)      */
  uint32_t flags;         /* TDDFT_FLAG_*                                         */
  void *stream;           /* hipStream_t for all work, or NULL (default stream)   */
  /* optional device allocator; both NULL -> hipMalloc / hipFree */
  void *(*dev_alloc)(size_t bytes, void *user);
  void (*dev_free)(void *ptr, void *user);
  void *alloc_user;
} tddft_config;

/* One atom's separable projectors, restricted to its sphere |x| < r_c.
 * x is the minimum-image offset r - R_a of each sphere point. */
typedef struct {
  int32_t npts;           /* sphere points (>= 1)                                 */
  int32_t n_proj;         /* projectors on this atom, 1..4                        */
  const int32_t *idx;     /* [npts] flat grid index, distinct                      */
  const double *x;        /* [npts][3] offsets (bohr)                              */
  const double *beta;     /* [n_proj][npts] real projector values                  */
  const double *e_kb;     /* [n_proj] KB energies (Ha)                             */
} tddft_atom;

/* Version of the ABI this library implements. */
uint32_t tddft_abi_version(void);

/* Create a context: validate cfg, allocate device state, upload psi0
 * ([n_k][n_orb][n3][n2][n1] complex128), form rho(0) by Eq. rho (Sec. 3.1:
 * rho = sum_k w_k sum_n 2 |w_nk|^2). The grid and boundary follow Sec. 2.1
 * (uniform Cartesian grid; periodic cell or isolated box with vacuum beyond
 * the faces), the k-points Sec. 4.1. Errors: EINVAL (bad cfg, NULL psi0/out),
 * ENOMEM (an allocation, including one by dev_alloc, returned NULL),
 * EDEVICE. On failure *out is NULL and nothing stays allocated. */
tddft_status tddft_init(const tddft_config *cfg, const double *psi0, tddft_ctx **out);

/* Install the ionic potential (Sec. 3.1: local part plus the separable
 * Kleinman-Bylander nonlocal part; Sec. 4.1 for its phase exp(-i kappa.x)):
 * v_loc [n3][n2][n1] (Ha) and n_atoms atom projector tables (n_atoms may be
 * 0, atoms then NULL; the tables are copied). Recomputes the Hartree
 * potential (Poisson equation of Sec. 3.1, by FFT: 4 pi / G^2 for periodic
 * cells, the free-space kernel on a doubled box for isolated ones) and the
 * xc potential from the current density, and checks the Taylor stability
 * bound |lambda| dt <= 2 sqrt 2 (EUNSTABLE unless TDDFT_FLAG_ALLOW_UNSTABLE).
 * Errors: EINVAL (NULL v_loc, non-finite values, an index out of the grid
 * or repeated within an atom), ENOMEM, EDEVICE, EUNSTABLE. May be called
 * again to replace the tables. */
tddft_status tddft_set_potential(tddft_ctx *ctx, const double *v_loc, int32_t n_atoms,
                                 const tddft_atom *atoms);

/* Advance nsteps steps of dt (Program Summary: the fourth-order truncated
 * Taylor expansion of exp(-i dt h); Sec. 4.1, Eq. TDKS_solid for h with the
 * vector potential, Eq. TDKS for the isolated form). A is the host table
 * [nsteps + 1][3] of the vector potential at t_n = n dt (velocity gauge:
 * kappa = k + A/c at the step midpoint; length gauge: E_n = -(A_{n+1} - A_n)
 * / (c dt) enters as E.r). The potential is frozen at rho(t_n) during a step;
 * after it the density (Eq. rho), Hartree and xc potentials are rebuilt. If
 * J_out is not NULL it receives [nsteps][3]: the current I(t_{n+1}) of
 * Eq. macro_current (nonlocal part included) after each step. Errors:
 * ESTATE (no set_potential yet, or a poisoned context), EINVAL (bad
 * arguments, non-finite A), EUNSTABLE (|A| makes the step unstable),
 * EDEVICE, ENUMERIC (NaN or Inf in the norms or the current: poisoned). */
tddft_status tddft_propagate(tddft_ctx *ctx, int32_t nsteps, const double *A, double *J_out);

/* Density [n3][n2][n1] (Eq. rho; may be NULL) and macroscopic current [3]
 * (Eq. macro_current, nonlocal part included; may be NULL) at the current
 * time; the current uses the last A seen (0 before any propagate). Errors:
 * EINVAL, ESTATE (poisoned), EDEVICE. */
tddft_status tddft_density_current(tddft_ctx *ctx, double *rho, double *J);

/* Copy the orbitals back as complex128 [n_k][n_orb][n3][n2][n1]. */
tddft_status tddft_get_orbitals(tddft_ctx *ctx, double *psi);

/* Replace the orbitals (same layout as psi0) and re-form rho and the
 * potential; the device state then equals a fresh init from psi (resume). */
tddft_status tddft_set_orbitals(tddft_ctx *ctx, const double *psi);

/* Total energy (Sec. 4.1: the electronic energy whose change is the
 * excitation energy): sum_k w_k sum_n 2 <w|h_kin + V_loc + V_NL|w>
 * + 1/2 int rho V_H + int rho eps_xc (ion-ion constant omitted), at the last
 * A seen. Errors: EINVAL, ESTATE (no set_potential, or poisoned), EDEVICE. */
tddft_status tddft_energy(tddft_ctx *ctx, double *E);

/* The mixing parameter c of the BJ / TB09 exchange at the last potential
 * update (1 for BJ). ESTATE for the other xc choices. */
tddft_status tddft_xc_parameter(tddft_ctx *ctx, double *c);

/* Orbital norms <w|w>, [n_k][n_orb]. */
tddft_status tddft_norms(tddft_ctx *ctx, double *norms);

/* Induced dipole d = -int r (rho - rho_0) dr, r from the box centre (Sec. 3.1). */
tddft_status tddft_dipole(tddft_ctx *ctx, double d[3]);

/* Impulsive kick of an isolated system: w <- exp(-i F0 r_axis) w (Sec. 3.1),
 * axis 0..2; re-forms rho and the potential. EINVAL for periodic cells. */
tddft_status tddft_kick(tddft_ctx *ctx, double F0, int32_t axis);

/* Ground-state preparation (Sec. 2.1: the real-time run starts from the
 * static Kohn-Sham solution), at A = 0. Each of n_iter iterations applies the
 * imaginary-time Taylor step w <- sum_{m=0..4} (-tau h)^m / m! w with the
 * potential frozen at the current density, orthonormalises the orbitals of
 * every k-point (Gram-Schmidt in orbital order, as Cholesky-QR applied twice)
 * and rebuilds the density and the Hartree + xc potential. tau > 0 with
 * tau * lambda_max(h) <= 1.59, else EUNSTABLE (the damping polynomial
 * P4(-x) must decrease over the whole spectrum, so that every mode is damped
 * more than every lower one). energies (may be NULL) receives the total
 * energy after each iteration. The final density becomes rho_0 of the
 * dipole. */
tddft_status tddft_ground_state(tddft_ctx *ctx, int32_t n_iter, double tau, double *energies);

/* Keep a copy of the current orbitals (normally the ground state, before any
 * field) as the reference for tddft_excited_electrons. At most 64 orbitals
 * per k-point (EINVAL otherwise). */
tddft_status tddft_set_reference(tddft_ctx *ctx);

/* Number density of excited electron-hole pairs (Sec. 4.2, Fig. Si_pulse):
 * the occupied weight that has left the span of the reference orbitals of the
 * same k-point, n_ex = (1/Omega) sum_k w_k 2 [n_orb - sum_{m,n}
 * |<ref_mk|w_nk>|^2] (bohr^-3). The paper names the quantity without a
 * formula; this projection is exact once the field has returned to its
 * starting value. ESTATE before tddft_set_reference. */
tddft_status tddft_excited_electrons(tddft_ctx *ctx, double *n_ex);

/* Electronic excitation energy (Sec. 4.1: the energy at time t minus that of
 * the ground state), E_ex = E(t) - E(ref) in Ha per cell, with E(ref) the
 * energy when tddft_set_reference was called (divide by the cell volume for
 * the energy per unit volume). ESTATE before set_reference, and for the BJ /
 * TB09 potentials, which have no energy functional: Sec. 4.1 takes the work
 * of the field there (tddft_work). */
tddft_status tddft_excitation_energy(tddft_ctx *ctx, double *E_ex);

/* JSON text (NUL-terminated in buf) of how the context runs its step:
 * {"path": "fused"} for the LDS-resident step, else the per-stage
 * kernel's decomposition chosen by the tuner at set_potential: "key" (device,
 * grid, boundary, orbital count, precision), "source" ("tuned", "cache" or
 * "default" under TDDFT_FLAG_NO_TUNE), "stage" (bc: 0 whole periodic plane,
 * 1 periodic tiles, 2 isolated tiles; TX x TY tile, zs z slabs, xmap XCD
 * renumbering, ms per middle stage) and the timed "candidates". The tuner
 * times every decomposition that fits the grid (all compute identical bits;
 * the observe pass keeps its own, so the current is unaffected) and keeps the
 * fastest per key for the process, and in the JSON file named by the
 * environment variable TDDFT_TUNE_CACHE when set. EINVAL if len is too small. */
tddft_status tddft_report(tddft_ctx *ctx, char *buf, size_t len);

/* Mean device time per step of the last propagate, from HIP events (ms). */
tddft_status tddft_last_timing(tddft_ctx *ctx, double *ms_per_step);

/* Kernels of one step that tddft_time_kernel can time in isolation. */
enum { TDDFT_KERNEL_STAGE = 0, TDDFT_KERNEL_PROJECT = 1, TDDFT_KERNEL_OBSERVE = 2,
       TDDFT_KERNEL_DENSITY = 3, TDDFT_KERNEL_FUSED = 4 };

/* Launch one kernel of the step `reps` times back to back on the context's
 * stream and return the mean duration per launch from HIP events around the
 * launches (ms). TDDFT_KERNEL_STAGE is a middle Horner stage (reads u_s and w,
 * writes u_{s-1}); it and the projection use the two stage buffers, whose
 * contents are scratch between steps, so the state is unchanged.
 * TDDFT_KERNEL_FUSED is the whole four-stage update of a context that takes the
 * LDS-resident step (EINVAL otherwise); the orbitals are saved to the stage
 * buffers before and restored after, so the state is unchanged too.
 * TDDFT_KERNEL_DENSITY is the pass that sums the density over the orbitals
 * (with the kinetic energy density under BJ / TB09) into its partial sums,
 * which are scratch between steps. Requires
 * set_potential; EINVAL for an unknown kernel or reps < 1. */
tddft_status tddft_time_kernel(tddft_ctx *ctx, int32_t which, int32_t reps, double *ms_per_launch);

/* Message of the last failure on ctx; with ctx NULL, of the last failed call
 * on this thread that takes no context (the spectra and work entry points). */
const char *tddft_last_error(const tddft_ctx *ctx);
void tddft_free(tddft_ctx *ctx);

/* ---- Spectra and work from time series --------------------------------
 * Post-processing of one run's recorded series on the device. Host arrays in
 * and out, as everywhere; each call allocates its device buffers, computes,
 * copies back and frees before returning. Time integrals use the trapezoid
 * rule on t_n = n dt, n = 0 .. n_t - 1, with T = (n_t - 1) dt. The mask is
 * f(u) = 1 - 3u^2 + 2u^3 (Sec. 3.1). Every sum runs in a fixed order (same
 * bits on every call). Errors: EINVAL (n_t < 2, n < 1, NULL pointer, dt or
 * the kick zero or not finite, non-finite input, unknown flag), ENOMEM,
 * EDEVICE; the message is tddft_last_error(NULL). */
#define TDDFT_SPECTRUM_NO_MASK 0x1u        /* f = 1 instead of the cubic mask          */
#define TDDFT_SPECTRUM_SUBTRACT_MEAN 0x2u  /* I -> I - mean(I) first (Sec. 4.2: removes a
                                              small constant current so that sigma(0) = 0) */

/* Conductivity of a periodic system after a kick A(t) = A0 theta(t)
 * (Sec. 4.1, Eq. sigma_ft): sigma(w) = -(c / A0) int_0^T dt e^{i w t}
 * f(t / T) I(t), one component. I [n_t]: the current at t_n (I[0] just after
 * the kick); omega [n_w] (Ha); sigma [n_w][2] receives (re, im); eps
 * ([n_w][2], may be NULL) the dielectric function eps = 1 + 4 pi i sigma / w
 * (Sec. 4.1; not finite at w = 0). */
tddft_status tddft_conductivity(int32_t n_t, const double *I, double dt, double A0, int32_t n_w,
                                const double *omega, uint32_t flags, double *sigma, double *eps);

/* Oscillator-strength distribution of an isolated system after an impulsive
 * kick F0 (Sec. 3.1, Eq. distribution, in atomic units and per unit kick):
 * df/dE = (2 E / pi) Im int_0^T f(t / T) d(t) e^{i E t} dt / F0, with the
 * mask always applied. d [n_t]: one dipole component at t_n (d[0] = 0 at the
 * kick); E [n_E] (Ha); dfdE [n_E]. */
tddft_status tddft_oscillator_strength(int32_t n_t, const double *d, double dt, double F0, int32_t n_E,
                                       const double *E, double *dfdE);

/* Work of the field on the electrons of one cell (Sec. 4.1, W(t), the
 * excitation energy for xc potentials without an energy functional):
 * W_n = volume sum_{m<n} dt (I_m + I_{m+1}) / 2 . E_m with
 * E_m = -(A_{m+1} - A_m) / (c dt), so that dE/dt = +volume I . E (the sign
 * with I as in Eq. macro_current and E = -(1/c) dA/dt). I, A [n_t][3]: the
 * current and the vector potential at t_n (A is the propagate table, I[0]
 * the current before the first step); W [n_t] (Ha per cell). */
tddft_status tddft_work(int32_t n_t, const double *I, const double *A, double dt, double volume, double *W);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as tddft_conductivity, same bits, with DEVICE arrays I [n_t],
 * omega [n_w], sigma [n_w][2] and eps ([n_w][2] or NULL) owned by the caller,
 * enqueued on `stream` (a hipStream_t, NULL for the default stream) without
 * waiting for it. Allocates nothing: the chunk partials and the mean live in
 * a fixed 8 MiB device array per GPU, held until the process ends, which
 * every call on that GPU shares; calls that overlap on one GPU (other
 * streams, other threads) race on it and must be serialised by the caller.
 * Every slot is written before it is read, so no clearing is needed. Limit:
 * 1 + min(64, ceil(n_t / 256)) * n_w <= 524288 (n_w <= 8191 for series of
 * 16384 samples or more), else EINVAL. The device inputs are not checked for
 * finiteness. Errors: EINVAL, EDEVICE; message in tddft_last_error(NULL). */
tddft_status tddft_conductivity_noalloc(int32_t n_t, const double *I, double dt, double A0, int32_t n_w,
                                        const double *omega, uint32_t flags, double *sigma, double *eps,
                                        void *stream);

/* ---- Batches of independent cells -------------------------------------
 * Many cells with their own grid, orbital and k-point counts, atoms and
 * field tables advance together: one hipGraph-captured batch step holds, per
 * group of cells with the same cubic grid (12, 16 or 20 points per axis, or
 * 24 for complex FP32 orbitals: the orbital must fit in LDS), one
 * persistent launch of the fused step whose workgroups pull (cell, orbital)
 * items from a device queue, largest cells first; other cells run the
 * per-stage kernels on forked streams inside the same graph. The persistent
 * grid of every group is chosen by timing candidates on the first steps
 * (every candidate computes identical bits), and every per-stage cell's
 * decomposition by the tuner of tddft_report, unless
 * TDDFT_FLAG_NO_TUNE is set in cfgs[0].flags. When the cells of a group
 * share their Hartree and xc switches (LDA or none), the start and the end of
 * their step (field, phases, current, density, Poisson, potential) run as one
 * launch per kernel for the group. Every cell behaves as its own context
 * would alone, bit for bit; the current of a cell is its own. */
#define TDDFT_FLAG_NO_TUNE 0x10u

typedef struct tddft_batch tddft_batch;

/* n_cells configurations and initial orbitals (layout as in tddft_init).
 * All cells use cfgs[0].precision, cfgs[0].stream (NULL: a stream owned by
 * the batch) and cfgs[0].flags (TDDFT_FLAG_PREDICTOR_CORRECTOR: EINVAL, single
 * contexts only). Errors as tddft_init; on failure *out = NULL. */
tddft_status tddft_batch_create(int32_t n_cells, const tddft_config *cfgs, const double *const *psi0,
                                tddft_batch **out);
/* As tddft_set_potential for one cell (0 <= cell < n_cells). */
tddft_status tddft_batch_set_potential(tddft_batch *b, int32_t cell, const double *v_loc, int32_t n_atoms,
                                       const tddft_atom *atoms);
/* Advance every cell nsteps steps; A[c] is cell c's table [nsteps + 1][3],
 * J_out (may be NULL, or hold NULL entries) receives [nsteps][3] per cell. */
tddft_status tddft_batch_propagate(tddft_batch *b, int32_t nsteps, const double *const *A, double *const *J_out);
/* The context of one cell, for tddft_get_orbitals, tddft_density_current,
 * tddft_energy, tddft_norms; owned by the batch (do not free). NULL if out of range. */
tddft_ctx *tddft_batch_cell(tddft_batch *b, int32_t cell);
/* Mean device time per batch step of the last propagate (ms). */
tddft_status tddft_batch_last_timing(tddft_batch *b, double *ms_per_step);
/* JSON text of the plan (per group: grid, cells, items, column split,
 * persistent workgroups, whether the step's ends run per group) and the
 * tuner's measurements, NUL-terminated in buf. */
tddft_status tddft_batch_report(tddft_batch *b, char *buf, size_t len);
const char *tddft_batch_last_error(const tddft_batch *b);
void tddft_batch_free(tddft_batch *b);

/* ---- Learned current surrogate -----------------------------------------
 * A network that stands in for the microscopic cell of the multiscale
 * coupling (Sec. 5, Eqs. Maxwell_ms and TDKS_ms): it maps the causal window
 * of the last `window` macroscopic samples of the vector potential at one
 * point to the current there. Form (the paper has none): x = A / a_scale;
 * h1 = tanh(W1 x + b1) (window -> hidden); h2 = tanh(W2 h1 + b2);
 * y = w3 . h2 + b3 + ws . x; I = j_scale y. Loss: mean of (y - target)^2.
 * Training: Adam (Kingma and Ba 2015, Algorithm 1) on the device. FP32.
 * Parameters, flat, host order: W1 [hidden][window], b1 [hidden],
 * W2 [hidden][hidden], b2 [hidden], w3 [hidden], b3 [1], ws [window]. */
typedef struct tddft_nn tddft_nn;

typedef struct {
  int32_t window;         /* input samples W, 1..4096                            */
  int32_t hidden;         /* hidden width H, 1..1024                             */
  double a_scale;         /* input scale: x = A / a_scale (nonzero)              */
  double j_scale;         /* output scale: I = j_scale y (nonzero)               */
  float lr, beta1, beta2, eps;  /* Adam hyper-parameters                        */
} tddft_nn_config;

/* Number of parameters for a window and hidden width. */
int64_t tddft_nn_num_params(int32_t window, int32_t hidden);
/* Create with initial parameters (host, n_params floats, copied). Adam's
 * moments start at zero. EINVAL on bad sizes; ENOMEM/EDEVICE on HIP failure. */
tddft_status tddft_nn_create(const tddft_nn_config *cfg, const float *params, tddft_nn **out);
tddft_status tddft_nn_get_params(tddft_nn *nn, float *params);
/* Replace the parameters and reset Adam's moments and step count. */
tddft_status tddft_nn_set_params(tddft_nn *nn, const float *params);
/* y [batch] = network(x [batch][window]) for already scaled inputs. */
tddft_status tddft_nn_forward(tddft_nn *nn, int32_t batch, const float *x, float *y);
/* Loss and its gradient (grad may be NULL) for a batch with scaled targets;
 * the gradient is kept on the device for tddft_nn_adam_step. */
tddft_status tddft_nn_loss_grad(tddft_nn *nn, int32_t batch, const float *x, const float *target, float *loss,
                                float *grad);
/* One Adam step with the gradient of the last tddft_nn_loss_grad. ESTATE if
 * there is none. */
tddft_status tddft_nn_adam_step(tddft_nn *nn);
/* Train on trajectories: A and J are [n_traj][T] raw (unscaled) samples at
 * the macroscopic times; every (trajectory, t) is one sample whose input is
 * the window of A ending at t (zeros before the start) and whose target is
 * J(t). Each epoch visits the samples in an order drawn from `seed` and the
 * epoch number, in batches of `batch` (the last one may be smaller); one Adam
 * step per batch. loss_per_epoch (may be NULL) gets each epoch's mean batch
 * loss. */
tddft_status tddft_nn_train(tddft_nn *nn, int32_t n_traj, int32_t T, const double *A, const double *J,
                            int32_t epochs, int32_t batch, uint64_t seed, float *loss_per_epoch);
/* Training options of tddft_nn_train_ex. */
#define TDDFT_NN_COSINE_LR 0x1u      /* lr of epoch e: lr (1 + cos(pi e / epochs)) / 2 */
#define TDDFT_NN_FREEZE_LINEAR 0x2u  /* keep b3 and ws fixed (their gradient is zeroed) */
/* tddft_nn_train with options (flags 0 is tddft_nn_train). */
tddft_status tddft_nn_train_ex(tddft_nn *nn, int32_t n_traj, int32_t T, const double *A, const double *J,
                               int32_t epochs, int32_t batch, uint64_t seed, uint32_t flags,
                               float *loss_per_epoch);
/* Set the linear part of the network to the least-squares linear response:
 * ws and b3 minimise sum (ws . x + b3 - y)^2 + lambda |(ws, b3)|^2 over every
 * (trajectory, t) sample of the trajectories (A, J as in tddft_nn_train)
 * whose largest |A| is within a_fit, with lambda = lambda_rel times the mean
 * diagonal of the normal matrix; the normal equations are formed and solved
 * (Cholesky) in FP64 on the device. w3 is set to 0, so the network equals the
 * fit until trained further (the weak-field response is then carried by the
 * skip and the hidden layers learn what is left); Adam's state is reset.
 * Within a window the linear response of the cells to A is exact in the
 * weak-field limit (Sec. 5 couples the cells through A alone). Errors:
 * EINVAL (fewer than W + 1 samples within a_fit, bad arguments), ENUMERIC
 * (normal matrix not positive definite), ENOMEM, EDEVICE. */
tddft_status tddft_nn_fit_linear(tddft_nn *nn, int32_t n_traj, int32_t T, const double *A, const double *J,
                                 double a_fit, double lambda_rel);
const char *tddft_nn_last_error(const tddft_nn *nn);
void tddft_nn_free(tddft_nn *nn);

/* ---- Multiscale light propagation (Sec. 5) --------------------------------
 * A(X, t) along one polarisation axis on a 1-D grid X_j = j dx obeys
 * (1/c^2) d^2A/dt^2 - d^2A/dX^2 = (4 pi / c) I (Eq. Maxwell_ms), leapfrog in
 * X and t with first-order Mur absorbing ends; an incident wave enters at the
 * left end (the Mur condition acts on A - A_inc there). The points x0 ..
 * x0 + n_mat - 1 hold the medium: each is a cell (Eq. TDKS_ms) advanced n_sub
 * steps of dt / n_sub per macroscopic step, with A interpolated linearly; its
 * current after the last of them is I there. The medium starts at rest
 * (I = 0 at t = 0) and the field starts at zero. */
typedef struct tddft_ms tddft_ms;

typedef struct {
  int32_t n_x;            /* macroscopic points, >= 4                            */
  int32_t x0, n_mat;      /* medium: points x0 .. x0 + n_mat - 1, 1 <= x0,
                             x0 + n_mat <= n_x - 1, n_mat >= 1                   */
  double dx;              /* grid spacing (bohr)                                 */
  double dt;              /* macroscopic time step; c dt / dx <= 1               */
  int32_t n_sub;          /* cell steps per macroscopic step (>= 1); the cell
                             configuration's dt must equal dt / n_sub           */
  int32_t axis;           /* polarisation axis in the cell frame: 0, 1 or 2      */
} tddft_ms_config;

/* Every medium point starts from the same cell: configuration, orbitals
 * (layout as tddft_init; normally the ground state), local potential and
 * atoms as for tddft_set_potential. The cells are created when first needed
 * (at once without a surrogate). */
tddft_status tddft_ms_create(const tddft_ms_config *cfg, const tddft_config *cell, const double *psi0,
                             const double *v_loc, int32_t n_atoms, const tddft_atom *atoms, tddft_ms **out);
/* Couple through a trained network (borrowed; must outlive the run) instead
 * of the cells. The cells remain the fallback: if |A| at a medium point
 * exceeds a_max (the trained range), or if every `check_every` steps the
 * sentinel points, which run full cells alongside, disagree with the network
 * by more than tol (max |I_net - I_cell| over the interval, relative to the
 * network's output scale |j_scale|), every medium point switches to its cell, which
 * first replays its A history from t = 0, and the run continues with cells.
 * sentinels are medium indices (0 .. n_mat - 1). Must precede the first step. */
tddft_status tddft_ms_attach_surrogate(tddft_ms *ms, tddft_nn *nn, double a_max, int32_t n_sentinel,
                                       const int32_t *sentinels, int32_t check_every, double tol);
/* Advance n_macro steps. inc [n_macro + 1][2]: incident A at X_0 and X_1 at
 * t_n .. t_{n + n_macro} (NULL: none). A_out and I_out (may be NULL):
 * [n_macro][n_x] after each step. */
tddft_status tddft_ms_step(tddft_ms *ms, int32_t n_macro, const double *inc, double *A_out, double *I_out);
/* mode: 0 cells, 1 network; fallbacks taken; the last sentinel error; steps done. */
tddft_status tddft_ms_status(tddft_ms *ms, int32_t *mode, int32_t *fallbacks, double *last_check,
                             int32_t *steps_done);
/* Energy monitor (Sec. 5: the total energy is that of the electromagnetic
 * field and of the electronic excitations; its conservation checks the run),
 * per unit area of the slab (Ha / bohr^2), at the current step:
 * em = (1/8 pi) [sum_j E_j^2 + sum_j B_{j+1/2}^2] dX with E = -(A^n - A^{n-1})/(c dt)
 * and B = (A_{j+1} - A_j)/dX; work = the energy the field has given the medium
 * since t = 0, W = sum_steps dt dX sum_medium (I^n + I^{n+1})/2 E^{n+1/2} (the
 * work route to the excitation energy of Sec. 4.1; dE/dt = +I . E per volume).
 * em + work changes only by the flux through the ends of the grid. Either
 * pointer may be NULL. After a fallback the work is recomputed from the cells'
 * currents. */
tddft_status tddft_ms_energy(tddft_ms *ms, double *em, double *work);
const char *tddft_ms_last_error(const tddft_ms *ms);
void tddft_ms_free(tddft_ms *ms);

#ifdef __cplusplus
}
#endif
#endif /* TDDFT_H */
