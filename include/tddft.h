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
enum { TDDFT_XC_NONE = 0, TDDFT_XC_PZ81 = 1 };

#define TDDFT_FLAG_ALLOW_UNSTABLE 0x1u /* skip the Taylor stability refusal      */
#define TDDFT_FLAG_DEBUG_SYNC 0x2u     /* synchronise and check after each kernel */
#define TDDFT_FLAG_NO_GRAPH 0x4u       /* launch kernels directly, no hipGraph    */
#define TDDFT_FLAG_STREAMING 0x8u      /* one kernel per Horner stage even when the
                                          orbital fits in LDS (the fused step) */

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
  int32_t xc;             /* TDDFT_XC_NONE or TDDFT_XC_PZ81                       */
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
 * ([n_k][n_orb][n3][n2][n1] complex128), form rho(0). Errors: EINVAL
 * (bad cfg, NULL psi0/out), ENOMEM, EDEVICE. On failure *out is NULL. */
tddft_status tddft_init(const tddft_config *cfg, const double *psi0, tddft_ctx **out);

/* Install the ionic potential: v_loc [n3][n2][n1] (Ha) and n_atoms atom
 * projector tables (n_atoms may be 0, atoms then NULL). Recomputes the
 * Hartree and xc potentials from the current density and checks the
 * Taylor stability bound |lambda| dt <= 2 sqrt 2 (EUNSTABLE unless
 * TDDFT_FLAG_ALLOW_UNSTABLE). May be called again to replace the tables. */
tddft_status tddft_set_potential(tddft_ctx *ctx, const double *v_loc, int32_t n_atoms,
                                 const tddft_atom *atoms);

/* Advance nsteps steps of dt. A is the host table [nsteps + 1][3] of the
 * vector potential at t_n = n dt (velocity gauge: kappa = k + A/c at the step
 * midpoint; length gauge: E_n = -(A_{n+1} - A_n) / (c dt) enters as E.r).
 * The potential is frozen at rho(t_n) during a step. If J_out is not NULL it
 * receives [nsteps][3]: the current I(t_{n+1}) after each step. Errors:
 * ESTATE (no set_potential yet), EINVAL, EDEVICE, ENUMERIC. */
tddft_status tddft_propagate(tddft_ctx *ctx, int32_t nsteps, const double *A, double *J_out);

/* Density [n3][n2][n1] (may be NULL) and current [3] (may be NULL) at the
 * current time; the current uses the last A seen (0 before any propagate). */
tddft_status tddft_density_current(tddft_ctx *ctx, double *rho, double *J);

/* Copy the orbitals back as complex128 [n_k][n_orb][n3][n2][n1]. */
tddft_status tddft_get_orbitals(tddft_ctx *ctx, double *psi);

/* Replace the orbitals (same layout as psi0) and re-form rho and the
 * potential; the device state then equals a fresh init from psi (resume). */
tddft_status tddft_set_orbitals(tddft_ctx *ctx, const double *psi);

/* Total energy: sum_k w_k sum_n 2 <w|h_kin + V_loc + V_NL|w> + 1/2 int rho V_H
 * + int rho eps_xc (ion-ion constant omitted), at the last A seen. */
tddft_status tddft_energy(tddft_ctx *ctx, double *E);

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
 * tau * lambda_max(h) <= 2.7, else EUNSTABLE (the damping polynomial must
 * stay below one). energies (may be NULL) receives the total energy after
 * each iteration. The final density becomes rho_0 of the dipole. */
tddft_status tddft_ground_state(tddft_ctx *ctx, int32_t n_iter, double tau, double *energies);

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
 * buffers before and restored after, so the state is unchanged too. Requires
 * set_potential; EINVAL for an unknown kernel or reps < 1. */
tddft_status tddft_time_kernel(tddft_ctx *ctx, int32_t which, int32_t reps, double *ms_per_launch);

const char *tddft_last_error(const tddft_ctx *ctx);
void tddft_free(tddft_ctx *ctx);

/* ---- Batches of independent cells -------------------------------------
 * Many cells with their own grid, orbital and k-point counts, atoms and
 * field tables advance together: one hipGraph-captured batch step holds, per
 * group of cells with the same cubic grid (12, 16 or 20 points per axis), one
 * persistent launch of the fused step whose workgroups pull (cell, orbital)
 * items from a device queue, largest cells first; other cells run the
 * per-stage kernels on forked streams inside the same graph. The persistent
 * grid of every group is chosen by timing candidates on the first steps
 * (every candidate computes identical bits), unless
 * TDDFT_FLAG_NO_TUNE is set in cfgs[0].flags. Every cell behaves as its own
 * context would alone; the current of a cell is its own. */
#define TDDFT_FLAG_NO_TUNE 0x10u

typedef struct tddft_batch tddft_batch;

/* n_cells configurations and initial orbitals (layout as in tddft_init).
 * All cells use cfgs[0].precision, cfgs[0].stream (NULL: a stream owned by
 * the batch) and cfgs[0].flags. Errors as tddft_init; on failure *out = NULL. */
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
/* JSON text of the plan and the tuner's measurements, NUL-terminated in buf. */
tddft_status tddft_batch_report(tddft_batch *b, char *buf, size_t len);
const char *tddft_batch_last_error(const tddft_batch *b);
void tddft_batch_free(tddft_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* TDDFT_H */
