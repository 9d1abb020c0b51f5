"""Plain FP64 CPU oracle of the real-time TDKS time step (test infrastructure).

THIS MODULE IS TEST INFRASTRUCTURE. Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it. It shares no code with the HIP
library: it is written from the paper's equations, in NumPy, without
blocking, fusion or reordering, so that each function can be read against
the passage it follows.

What it computes (atomic units, hbar = m = e = 1):

* Bloch orbitals w_nk on a uniform grid over a cuboid, periodic or with
  vacuum (zero) outside the box (Sec. 2.1).
* h w = 1/2 (-i grad + k + A/c)^2 w + V w + V_NL^kappa w (Sec. 4.1,
  Eq. TDKS_solid), with the square expanded on the grid as
  -1/2 Lap_h w - i kappa . grad_h w + 1/2 |kappa|^2 w, kappa = k + A/c, and
  Lap_h, grad_h the 9-point-per-axis central differences; in the isolated
  length gauge kappa = k and V gains E(t) . r (Sec. 3.1).
* V_NL: separable Kleinman-Bylander projectors (Sec. 3.1) carrying the phase
  exp(-i kappa . x) so that the nonlocal term depends on A (Sec. 4.1).
* The time step: the Taylor expansion of exp(-i dt h) truncated after the
  fourth power (Program Summary), with V fixed at rho(t_n) and kappa taken
  at the step-midpoint vector potential.
* rho = 2 sum |psi|^2 (Eq. rho) weighted over k-points; the macroscopic
  current I(t) of Eq. macro_current including the nonlocal part.
* Hartree potential (Eq. TDKS): periodic 4 pi rho(G) / G^2; isolated by
  free-space convolution on a doubled box. Adiabatic LDA of Perdew and
  Zunger (Sec. 3.1).
* Energy, induced dipole (Sec. 3.1) and excitation energy by work (Sec. 4.1).

Readings where the paper is silent are recorded in the design notes and in
the docstrings below (finite-difference order, Taylor order, sampling of A,
occupations, the nonlocal current, projector and potential shapes).

Parity pins: every function here is pinned by a test in tests/test_oracle_*.py
against a closed form, a brute-force construction or an invariant.
"""
from __future__ import annotations

from fractions import Fraction
from typing import Optional, Sequence

import numpy as np

C_LIGHT = 137.035999084   # 1/alpha, CODATA 2018
FD_HALF_WIDTH = 4          # neighbours per side and axis (9 points per axis)


# --------------------------------------------------------------------------
# finite-difference weights (uniform Cartesian grid, Sec. 2.1)


def _solve_exact(A, b):
    """Gaussian elimination over the rationals."""
    n = len(b)
    M = [list(map(Fraction, row)) + [Fraction(v)] for row, v in zip(A, b)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [M[i][n] / M[i][i] for i in range(n)]


def fd_weights(M: int = FD_HALF_WIDTH):
    """Central weights on 2M+1 points by Taylor matching.

    Second derivative: h^2 f'' ~ c_0 f_0 + sum_{m=1..M} c_m (f_m + f_-m), exact
    for polynomials of degree <= 2M+1. First derivative: h f' ~ sum d_m
    (f_m - f_-m), exact to the same degree. Returned as Fractions
    (c_0..c_M), (d_1..d_M)."""
    # even moments p = 2, 4, ..., 2M: sum_m c_m m^p = [p == 2]
    A = [[m ** p for m in range(1, M + 1)] for p in range(2, 2 * M + 1, 2)]
    b = [1 if p == 2 else 0 for p in range(2, 2 * M + 1, 2)]
    c = _solve_exact(A, b)
    c0 = -2 * sum(c)
    # odd moments p = 1, 3, ..., 2M-1: 2 sum_m d_m m^p = [p == 1]
    A = [[2 * m ** p for m in range(1, M + 1)] for p in range(1, 2 * M, 2)]
    b = [1 if p == 1 else 0 for p in range(1, 2 * M, 2)]
    d = _solve_exact(A, b)
    return [c0] + c, d


_C2, _D1 = fd_weights()
C2 = np.array([float(x) for x in _C2])
D1 = np.array([float(x) for x in _D1])


# --------------------------------------------------------------------------
# grid


class Grid:
    """Uniform grid over a cuboid (Sec. 2.1). ``periodic`` or vacuum."""

    def __init__(self, n: Sequence[int], cell: Sequence[float], boundary: str):
        self.n = tuple(int(v) for v in n)          # (n1, n2, n3)
        self.cell = tuple(float(v) for v in cell)
        self.periodic = boundary == "periodic"
        self.h = tuple(self.cell[i] / self.n[i] for i in range(3))
        self.dV = self.h[0] * self.h[1] * self.h[2]
        self.volume = self.cell[0] * self.cell[1] * self.cell[2]
        self.shape = (self.n[2], self.n[1], self.n[0])

    def coords(self):
        """x, y, z coordinate arrays: j h (periodic) or (j - (N-1)/2) h."""
        out = []
        for N, h in zip(self.n, self.h):
            j = np.arange(N, dtype=np.float64)
            out.append(j * h if self.periodic else (j - (N - 1) / 2.0) * h)
        return out

    def r_fields(self):
        """Position vector components on the grid, each of shape ``shape``."""
        x, y, z = self.coords()
        return (np.broadcast_to(x[None, None, :], self.shape),
                np.broadcast_to(y[None, :, None], self.shape),
                np.broadcast_to(z[:, None, None], self.shape))

    def inner(self, a, b):
        """<a|b> = h1 h2 h3 sum conj(a) b over the last three axes."""
        return self.dV * np.sum(np.conj(a) * b, axis=(-3, -2, -1))


def _axis(mu: int) -> int:
    return -1 - mu          # x -> last axis, y -> -2, z -> -3


def shifted(f, m: int, mu: int, grid: Grid):
    """g[j] = f[j + m] along axis mu; periodic wrap or zero outside the box."""
    ax = _axis(mu)
    if grid.periodic:
        return np.roll(f, -m, axis=ax)
    g = np.zeros_like(f)
    N = f.shape[ax]
    src = [slice(None)] * f.ndim
    dst = [slice(None)] * f.ndim
    if m >= 0:
        src[ax] = slice(m, N)
        dst[ax] = slice(0, N - m)
    else:
        src[ax] = slice(0, N + m)
        dst[ax] = slice(-m, N)
    if N - abs(m) > 0:
        g[tuple(dst)] = f[tuple(src)]
    return g


def second_derivative(f, mu: int, grid: Grid):
    h = grid.h[mu]
    out = C2[0] * f
    for m in range(1, FD_HALF_WIDTH + 1):
        out = out + C2[m] * (shifted(f, m, mu, grid) + shifted(f, -m, mu, grid))
    return out / (h * h)


def first_derivative(f, mu: int, grid: Grid):
    h = grid.h[mu]
    out = np.zeros_like(f)
    for m in range(1, FD_HALF_WIDTH + 1):
        out = out + D1[m - 1] * (shifted(f, m, mu, grid) - shifted(f, -m, mu, grid))
    return out / h


def laplacian(f, grid: Grid):
    return sum(second_derivative(f, mu, grid) for mu in range(3))


def gradient(f, grid: Grid):
    return [first_derivative(f, mu, grid) for mu in range(3)]


# --------------------------------------------------------------------------
# pseudopotential tables, re-derived from the atom parameters


def local_potential(grid: Grid, atoms, depth, width, cut: float = 10.0):
    """Sum over atoms and periodic images of -U exp(-|x|^2 / 2 w^2), |x| <= cut w."""
    x, y, z = grid.coords()
    V = np.zeros(grid.shape)
    for R, U, w in zip(atoms, depth, width):
        rc = cut * w
        if grid.periodic:
            reach = [int(np.ceil(rc / L)) + 1 for L in grid.cell]
            imgs = [(a, b, c) for a in range(-reach[0], reach[0] + 1)
                    for b in range(-reach[1], reach[1] + 1)
                    for c in range(-reach[2], reach[2] + 1)]
        else:
            imgs = [(0, 0, 0)]
        for (a, b, c) in imgs:
            dx = x - R[0] - a * grid.cell[0]
            dy = y - R[1] - b * grid.cell[1]
            dz = z - R[2] - c * grid.cell[2]
            r2 = dx[None, None, :] ** 2 + dy[None, :, None] ** 2 + dz[:, None, None] ** 2
            V += np.where(r2 <= rc * rc, -U * np.exp(-r2 / (2 * w * w)), 0.0)
    return V


def projector_table(grid: Grid, R, n_proj: int, r_c: float = 2.0, sigma: float = 1.0):
    """Grid points with |x| < r_c around R (minimum image) and the normalised
    s (and p_x, p_y, p_z) projector values on them.

    Returns (flat index ascending, offsets [npts,3], beta [n_proj, npts])."""
    rx, ry, rz = grid.r_fields()
    d = [rx - R[0], ry - R[1], rz - R[2]]
    if grid.periodic:
        d = [d[i] - grid.cell[i] * np.round(d[i] / grid.cell[i]) for i in range(3)]
    inside = (d[0] ** 2 + d[1] ** 2 + d[2] ** 2 < r_c * r_c).ravel()
    pts = np.nonzero(inside)[0]                  # C order = flat index, ascending
    offs = np.stack([d[0].ravel()[pts], d[1].ravel()[pts], d[2].ravel()[pts]], axis=1)
    r2 = (offs ** 2).sum(axis=1)
    g = np.exp(-r2 / (2 * sigma ** 2)) * (1.0 - r2 / r_c ** 2) ** 2
    rows = [g] + ([offs[:, 0] / r_c * g, offs[:, 1] / r_c * g, offs[:, 2] / r_c * g] if n_proj == 4 else [])
    beta = np.array(rows)
    for p in range(beta.shape[0]):
        beta[p] /= np.sqrt(grid.dV * np.sum(beta[p] ** 2))
    return np.array(pts, dtype=np.int64), offs, beta


# --------------------------------------------------------------------------
# Hamiltonian (Eq. TDKS_solid; Eq. TDKS for the isolated length gauge)


class Projector:
    """One atom's KB projectors: idx [npts], x [npts,3], beta [P,npts], e_kb [P]."""

    def __init__(self, idx, x, beta, e_kb):
        self.idx = np.asarray(idx, dtype=np.int64)
        self.x = np.asarray(x, dtype=np.float64)
        self.beta = np.asarray(beta, dtype=np.float64)
        self.e_kb = np.asarray(e_kb, dtype=np.float64)


def nl_projections(W, projs, kappa, grid: Grid):
    """u_p = <beta_p^kappa | w> = h^3 sum_x beta_p(x) exp(+i kappa.x) w(r) and
    the first moments v_p = <x beta_p^kappa | w> (vector), for every orbital.

    W: [n_orb, n3, n2, n1]. Returns lists over atoms of u [n_orb, P] and
    v [n_orb, P, 3]."""
    Wf = W.reshape(W.shape[0], -1)
    us, vs = [], []
    for pr in projs:
        phase = np.exp(1j * (pr.x @ kappa))
        g = Wf[:, pr.idx] * phase[None, :]
        us.append(grid.dV * g @ pr.beta.T)
        vs.append(grid.dV * np.einsum("ni,pi,ic->npc", g, pr.beta, pr.x))
    return us, vs


def apply_nonlocal(W, projs, kappa, grid: Grid):
    """sum_p |beta_p^kappa> E_p <beta_p^kappa|w>, beta^kappa = beta(x) exp(-i kappa.x)."""
    out = np.zeros_like(W)
    Of = out.reshape(W.shape[0], -1)
    us, _ = nl_projections(W, projs, kappa, grid)
    for pr, u in zip(projs, us):
        phase = np.exp(1j * (pr.x @ kappa))
        Of[:, pr.idx] += ((u * pr.e_kb[None, :]) @ pr.beta) * np.conj(phase)[None, :]
    return out


def apply_h(W, kappa, V, projs, grid: Grid):
    """h w for a block of orbitals sharing one kappa.

    h = -1/2 Lap_h - i kappa.grad_h + 1/2 |kappa|^2 + V + V_NL^kappa."""
    kappa = np.asarray(kappa, dtype=np.float64)
    out = -0.5 * laplacian(W, grid)
    grads = gradient(W, grid)
    for mu in range(3):
        out = out - 1j * kappa[mu] * grads[mu]
    out = out + (0.5 * float(kappa @ kappa) + V) * W
    if projs:
        out = out + apply_nonlocal(W, projs, kappa, grid)
    return out


def taylor_step(W, dt, hop, order: int = 4):
    """sum_{m=0..order} (-i dt h)^m / m! w (Program Summary: truncated Taylor)."""
    term = W
    out = W.copy()
    for m in range(1, order + 1):
        term = (-1j * dt / m) * hop(term)
        out = out + term
    return out


def imaginary_time_step(W, tau, hop, order: int = 4):
    """sum_{m=0..order} (-tau h)^m / m! w: the truncated Taylor expansion of
    exp(-tau h), which shrinks the high eigencomponents relative to the low
    ones while tau * lambda_max stays inside the polynomial's decreasing range
    (preparation of the initial state, Sec. 2.1)."""
    term = W
    out = W.copy()
    for m in range(1, order + 1):
        term = (-tau / m) * hop(term)
        out = out + term
    return out


def gram_schmidt(W, grid: Grid):
    """Orthonormalise the orbitals of one k-point in their index order (the
    Gram-Schmidt step that is sequential over orbitals, Sec. 3.2), with
    <a|b> = h^3 sum conj(a) b. W: [n_orb, n3, n2, n1]."""
    Q = np.array(W, dtype=np.complex128, copy=True)
    for i in range(Q.shape[0]):
        v = Q[i]
        for j in range(i):
            v = v - grid.inner(Q[j], v) * Q[j]
        Q[i] = v / np.sqrt(np.real(grid.inner(v, v)))
    return Q


# --------------------------------------------------------------------------
# density, current, dipole (Eq. rho, Eq. macro_current, Sec. 3.1)


def density(psi, kw, grid: Grid):
    """rho(r) = sum_k w_k sum_n 2 |w_nk(r)|^2 (spin-saturated, Eq. rho)."""
    return 2.0 * np.einsum("k,knzyx->zyx", np.asarray(kw), np.abs(psi) ** 2)


def current(psi, kpts, kw, A, projs, grid: Grid, gauge: str = "velocity"):
    """Macroscopic current density I (Eq. macro_current), occupations 2 w_k.

    I = -(1/Omega) sum_k w_k sum_n 2 [<w|-i grad_h|w> + kappa <w|w>
         + sum_p 2 E_p Im(conj(v_p) u_p)],
    the last term being <w| -i [x, V_NL^kappa] |w> (the nonlocal current)."""
    total = np.zeros(3)
    for ik, k in enumerate(kpts):
        kappa = np.asarray(k, dtype=np.float64) + (np.asarray(A) / C_LIGHT if gauge == "velocity" else 0.0)
        W = psi[ik]
        grads = gradient(W, grid)
        acc = np.zeros(3)
        norms = np.real(grid.inner(W, W))
        for mu in range(3):
            acc[mu] += np.sum(np.real(grid.inner(W, -1j * grads[mu])))
        acc += kappa * np.sum(norms)
        if projs:
            us, vs = nl_projections(W, projs, kappa, grid)
            for pr, u, v in zip(projs, us, vs):
                acc += np.sum(2.0 * pr.e_kb[None, :, None] * np.imag(np.conj(v) * u[:, :, None]), axis=(0, 1))
        total += kw[ik] * 2.0 * acc
    return -total / grid.volume


def excited_electrons(psi_ref, psi, kw, grid: Grid):
    """Number density of excited electron-hole pairs (Sec. 4.2, Fig. Si_pulse):
    the occupied weight that has left the space of the reference (ground-state)
    orbitals of the same k-point,
        n_ex = (1/Omega) sum_k w_k 2 [n_orb - sum_{m,n} |<ref_mk|psi_nk>|^2].
    The paper names the quantity without a formula; this projection reading
    is exact once the applied field has returned to its starting value."""
    n_orb = psi.shape[1]
    total = 0.0
    for ik in range(psi.shape[0]):
        O = np.array([[grid.inner(psi_ref[ik, m], psi[ik, n]) for n in range(n_orb)] for m in range(n_orb)])
        total += kw[ik] * 2.0 * (n_orb - float(np.sum(np.abs(O) ** 2)))
    return total / grid.volume


def dipole(rho, rho0, grid: Grid):
    """d_mu = -int r_mu (rho - rho_0) dr, r from the box centre (Sec. 3.1)."""
    x, y, z = grid.coords()
    c = [np.mean(x), np.mean(y), np.mean(z)]
    rx, ry, rz = grid.r_fields()
    dr = rho - rho0
    return -grid.dV * np.array([np.sum((rx - c[0]) * dr), np.sum((ry - c[1]) * dr),
                                np.sum((rz - c[2]) * dr)])


# --------------------------------------------------------------------------
# Hartree (Eq. TDKS) and LDA (Sec. 3.1)


def hartree_periodic(rho, grid: Grid):
    """V_H(G) = 4 pi rho(G) / |G|^2, G = 2 pi m / L, with the G = 0 term dropped."""
    g = [2 * np.pi * np.fft.fftfreq(grid.n[i], d=1.0 / grid.n[i]) / grid.cell[i] for i in range(3)]
    G2 = g[2][:, None, None] ** 2 + g[1][None, :, None] ** 2 + g[0][None, None, :] ** 2
    K = np.zeros_like(G2)
    K[G2 > 0] = 4 * np.pi / G2[G2 > 0]
    return np.real(np.fft.ifftn(np.fft.fftn(rho) * K))


def box_integral_inv_r(a, b, c):
    """int_0^a int_0^b int_0^c dx dy dz / |r| in closed form."""
    d = np.sqrt(a * a + b * b + c * c)
    return (a * b * np.arcsinh(c / np.hypot(a, b)) + b * c * np.arcsinh(a / np.hypot(b, c))
            + c * a * np.arcsinh(b / np.hypot(c, a))
            - a * a / 2 * np.arctan(b * c / (a * d)) - b * b / 2 * np.arctan(c * a / (b * d))
            - c * c / 2 * np.arctan(a * b / (c * d)))


def coulomb_self_cell(h):
    """Average of 1/|r| over one grid cell centred on the origin."""
    return 8.0 * box_integral_inv_r(h[0] / 2, h[1] / 2, h[2] / 2) / (h[0] * h[1] * h[2])


def coulomb_kernel_isolated(grid: Grid):
    """g(r - r') on the doubled box: 1/|d| at offsets d != 0, the cell average at 0."""
    ds = []
    for N, h in zip(grid.n, grid.h):
        i = np.arange(2 * N)
        ds.append(np.where(i < N, i, i - 2 * N) * h)
    r = np.sqrt(ds[2][:, None, None] ** 2 + ds[1][None, :, None] ** 2 + ds[0][None, None, :] ** 2)
    g = np.zeros_like(r)
    g[r > 0] = 1.0 / r[r > 0]
    g[0, 0, 0] = coulomb_self_cell(grid.h)
    return g


def hartree_isolated(rho, grid: Grid, kernel=None):
    """V_H(r) = h^3 sum_r' rho(r') g(r - r'), by zero-padded FFT convolution
    on a box twice as long in each direction (Hockney-Eastwood)."""
    g = coulomb_kernel_isolated(grid) if kernel is None else kernel
    pad = np.zeros(g.shape)
    pad[:grid.n[2], :grid.n[1], :grid.n[0]] = rho
    conv = np.real(np.fft.ifftn(np.fft.fftn(pad) * np.fft.fftn(g)))
    return grid.dV * conv[:grid.n[2], :grid.n[1], :grid.n[0]]


def hartree_isolated_direct(rho, grid: Grid):
    """The same sum evaluated pair by pair (brute force, small grids only)."""
    rx, ry, rz = [f.ravel() for f in grid.r_fields()]
    q = rho.ravel()
    g0 = coulomb_self_cell(grid.h)
    V = np.empty_like(q)
    for i in range(q.size):
        d = np.sqrt((rx - rx[i]) ** 2 + (ry - ry[i]) ** 2 + (rz - rz[i]) ** 2)
        inv = np.where(d > 0, 1.0 / np.where(d > 0, d, 1.0), g0)
        V[i] = grid.dV * np.dot(inv, q)
    return V.reshape(rho.shape)


PZ_GAMMA, PZ_BETA1, PZ_BETA2 = -0.1423, 1.0529, 0.3334
PZ_A, PZ_B, PZ_C, PZ_D = 0.0311, -0.048, 0.0020, -0.0116


def pz81_correlation(rho):
    """Perdew-Zunger 1981 correlation, spin-unpolarised: returns (v_c, eps_c).

    r_s >= 1: Pade form in sqrt(r_s); r_s < 1: high-density logarithmic form;
    v_c = eps_c - (r_s/3) d eps_c/d r_s. Densities below 1e-30 give zero."""
    rho = np.asarray(rho, dtype=np.float64)
    v = np.zeros_like(rho)
    e = np.zeros_like(rho)
    m = rho >= 1e-30
    rs = (3.0 / (4.0 * np.pi * rho[m])) ** (1.0 / 3.0)
    ec = np.empty_like(rs)
    vc = np.empty_like(rs)
    hi = rs >= 1.0
    s = np.sqrt(rs[hi])
    den = 1.0 + PZ_BETA1 * s + PZ_BETA2 * rs[hi]
    ec[hi] = PZ_GAMMA / den
    vc[hi] = ec[hi] * (1.0 + 7.0 / 6.0 * PZ_BETA1 * s + 4.0 / 3.0 * PZ_BETA2 * rs[hi]) / den
    lo = ~hi
    l = np.log(rs[lo])
    ec[lo] = PZ_A * l + PZ_B + PZ_C * rs[lo] * l + PZ_D * rs[lo]
    vc[lo] = PZ_A * l + (PZ_B - PZ_A / 3.0) + 2.0 / 3.0 * PZ_C * rs[lo] * l + (2.0 * PZ_D - PZ_C) / 3.0 * rs[lo]
    v[m] = vc
    e[m] = ec
    return v, e


def lda_pz81(rho):
    """Perdew-Zunger 1981 LDA, spin-unpolarised: returns (v_xc, eps_xc).

    Exchange eps_x = -(3/4)(3 rho/pi)^(1/3), v_x = (4/3) eps_x, plus the
    correlation above. Densities below 1e-30 give zero."""
    rho = np.asarray(rho, dtype=np.float64)
    v, e = pz81_correlation(rho)
    m = rho >= 1e-30
    vx = -(3.0 * rho[m] / np.pi) ** (1.0 / 3.0)
    v[m] = vx + v[m]
    e[m] = 0.75 * vx + e[m]
    return v, e


# --------------------------------------------------------------------------
# the time-dependent system


class TDKS:
    """Self-consistent real-time propagation of one cell (the whole method).

    Mirrors the library's calls: construct with the inputs and the initial
    orbitals, ``propagate(A)`` over a vector-potential table A[n] = A(t_n),
    then read ``rho``, ``current()``, ``energy()``, ``psi``."""

    def __init__(self, n, cell, boundary, kpts, kw, psi0, dt, v_loc, projectors,
                 hartree=True, xc=True, gauge="velocity", predictor_corrector=False):
        self.grid = Grid(n, cell, boundary)
        self.kpts = np.asarray(kpts, dtype=np.float64)
        self.kw = np.asarray(kw, dtype=np.float64)
        self.psi = np.array(psi0, dtype=np.complex128, copy=True)
        self.dt = float(dt)
        self.v_loc = np.asarray(v_loc, dtype=np.float64)
        self.projs = [Projector(p.idx, p.x, p.beta, p.e_kb) for p in projectors]
        self.use_hartree = bool(hartree)
        # xc: False / None (none), True or "lda" (PZ81), "tb09" or "bj" (Sec. 4.1)
        self.xc_kind = ("lda" if xc is True else xc) if xc else None
        if self.xc_kind not in (None, "lda", "tb09", "bj"):
            raise ValueError(f"unknown xc {xc!r}")
        self.use_xc = self.xc_kind is not None
        self.mgga_c = None
        self.gauge = gauge
        self.predictor_corrector = bool(predictor_corrector)
        self._hker = coulomb_kernel_isolated(self.grid) if (hartree and not self.grid.periodic) else None
        self.A_now = np.zeros(3)            # A at the current time (for the current)
        self.rho = density(self.psi, self.kw, self.grid)
        self.rho0 = self.rho.copy()
        self._update_potential(self.psi, self.A_now)

    @classmethod
    def from_system(cls, s, psi0=None, predictor_corrector=False):
        return cls(s.n, s.cell, s.boundary, s.kpts, s.kw, s.psi0 if psi0 is None else psi0, s.dt,
                   s.v_loc, s.projectors, hartree=s.hartree, xc=s.xc, gauge=s.gauge,
                   predictor_corrector=predictor_corrector)

    # potentials ----------------------------------------------------------
    def _update_potential(self, psi, A):
        """V_KS from self.rho; the BJ / TB09 exchange also needs the orbitals
        psi (their kinetic energy density) and the vector potential A at
        their time."""
        g = self.grid
        self.v_h = np.zeros(g.shape)
        self.v_xc = np.zeros(g.shape)
        self.e_xc = np.zeros(g.shape)
        if self.use_hartree:
            self.v_h = hartree_periodic(self.rho, g) if g.periodic else hartree_isolated(self.rho, g, self._hker)
        if self.xc_kind == "lda":
            self.v_xc, self.e_xc = lda_pz81(self.rho)
        elif self.xc_kind is not None:
            from . import mgga
            self.v_xc, self.e_xc, self.mgga_c = mgga.mgga_potential(psi, self.kpts, self.kw, A, self.rho, g,
                                                                   self.xc_kind, self.gauge)
        self.v_ks = self.v_loc + self.v_h + self.v_xc

    def _external(self, E):
        rx, ry, rz = self.grid.r_fields()
        return E[0] * rx + E[1] * ry + E[2] * rz

    # one step (Program Summary: truncated Taylor; V frozen over the step) --
    def _taylor_all(self, psi, V, A0, A1):
        """The Taylor step of every k-point from psi under the potential V."""
        if self.gauge == "length":
            E = -(A1 - A0) / (C_LIGHT * self.dt)
            V = V + self._external(E)
            shift = np.zeros(3)
        else:
            shift = 0.5 * (A0 + A1) / C_LIGHT
        out = np.empty_like(psi)
        for ik, k in enumerate(self.kpts):
            kappa = k + shift
            hop = lambda X, kappa=kappa: apply_h(X, kappa, V, self.projs, self.grid)
            out[ik] = taylor_step(psi[ik], self.dt, hop)
        return out

    def step(self, A0, A1):
        """One step. Plain: the potential is frozen at rho(t_n). With the
        predictor-corrector (Program Summary: "when necessary"), a predicted
        step gives rho and V at t_{n+1}, and the step is redone from t_n under
        the mean of V(t_n) and the predicted V(t_{n+1})."""
        A0 = np.asarray(A0, dtype=np.float64)
        A1 = np.asarray(A1, dtype=np.float64)
        V = self.v_ks
        if self.predictor_corrector:
            pred = self._taylor_all(self.psi, V, A0, A1)
            V_n = V
            self.rho = density(pred, self.kw, self.grid)
            self._update_potential(pred, A1)
            V = 0.5 * (V_n + self.v_ks)
        self.psi = self._taylor_all(self.psi, V, A0, A1)
        self.A_now = A1
        self.rho = density(self.psi, self.kw, self.grid)
        self._update_potential(self.psi, self.A_now)

    def ground_state(self, n_iter, tau):
        """Prepare the initial state (Sec. 2.1) at A = 0: each iteration damps
        every k-point's orbitals with the imaginary-time Taylor polynomial under
        the potential of the current density, orthonormalises them by
        Gram-Schmidt, and rebuilds the density and potential. Returns the energy
        after each iteration; the final density becomes rho_0."""
        energies = np.empty(n_iter)
        zero = np.zeros(3)
        for it in range(n_iter):
            V = self.v_ks
            for ik, k in enumerate(self.kpts):
                hop = lambda X, k=k: apply_h(X, k, V, self.projs, self.grid)
                W = imaginary_time_step(self.psi[ik], tau, hop)
                self.psi[ik] = gram_schmidt(W, self.grid)
            self.rho = density(self.psi, self.kw, self.grid)
            self._update_potential(self.psi, zero)
            energies[it] = self.energy(zero)
        self.A_now = zero
        self.rho0 = self.rho.copy()
        return energies

    def propagate(self, A):
        """Step through the table A[0..nsteps]; returns I(t_{n+1}) per step."""
        A = np.asarray(A, dtype=np.float64)
        J = np.empty((A.shape[0] - 1, 3))
        for n in range(A.shape[0] - 1):
            self.step(A[n], A[n + 1])
            J[n] = self.current()
        return J

    # observables ----------------------------------------------------------
    def current(self, A=None):
        A = self.A_now if A is None else A
        return current(self.psi, self.kpts, self.kw, A, self.projs, self.grid, self.gauge)

    def dipole(self):
        return dipole(self.rho, self.rho0, self.grid)

    def norms(self):
        return np.real(self.grid.inner(self.psi, self.psi))

    def energy(self, A=None):
        """E = sum_k w_k sum_n 2 <w| h_kin(kappa) + V_loc + V_NL^kappa |w>
        + 1/2 int rho V_H + int rho eps_xc (ion-ion constant omitted)."""
        A = self.A_now if A is None else np.asarray(A, dtype=np.float64)
        g = self.grid
        e = 0.0
        for ik, k in enumerate(self.kpts):
            kappa = k + (A / C_LIGHT if self.gauge == "velocity" else 0.0)
            W = self.psi[ik]
            hW = apply_h(W, kappa, self.v_loc, self.projs, g)
            e += self.kw[ik] * 2.0 * float(np.sum(np.real(g.inner(W, hW))))
        e += 0.5 * g.dV * float(np.sum(self.rho * self.v_h))
        e += g.dV * float(np.sum(self.rho * self.e_xc))
        return e
