"""Plain FP64 CPU oracle of the Becke-Johnson and Tran-Blaha exchange
potentials (test infrastructure).

THIS MODULE IS TEST INFRASTRUCTURE. Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it. It shares no code with the HIP
library.

Sec. 4.1 names the Becke-Johnson (BJ) potential and the Tran-Blaha variant
(TB09) as alternatives to the adiabatic LDA for solids, without formulas; the
formulas below are the published ones (Becke and Johnson, J. Chem. Phys. 124,
221101 (2006); Tran and Blaha, Phys. Rev. Lett. 102, 226401 (2009); the
Becke-Roussel exchange-hole potential, Phys. Rev. A 39, 3761 (1989)). For the
spin-saturated systems here every spin quantity is half the total:
rho_s = rho/2, t_s = tau/2.

* v_x = c v_BR + (3c - 2) (1/pi) sqrt(5/12) sqrt(2 t_s / rho_s)
  (c = 1 is BJ; TB09 takes c = alpha + beta sqrt(g) with
  g = (1/Omega) int |grad rho| / rho over the cell, alpha = -0.012,
  beta = 1.023 bohr^(1/2)).
* v_BR = -(1/b)(1 - e^-x - x e^-x / 2), b^3 = x^3 e^-x / (8 pi rho_s), where
  x solves x e^(-2x/3) / (x - 2) = (2/3) pi^(2/3) rho_s^(5/3) / Q_s,
  Q_s = (1/6)(lap rho_s - 2 gamma D_s), D_s = T_s - |grad rho_s|^2 / (4 rho_s),
  T_s = sum_i |grad psi_i,s|^2 = 2 t_s, gamma = 1 (the curvature of the
  exact exchange hole).
* The correlation part is the PZ81 LDA correlation.

Readings where the paper is silent (all recorded in the design notes):
tau is taken from the orbitals with the same 9-point first derivative as the
Hamiltonian and the gauge-invariant form |(grad_h + i kappa) w|^2, with
kappa = k + A/c for the A at the orbitals' time (k in the length gauge);
grad rho and lap rho use the same finite differences on the density; densities
below 1e-30 give v_x = 0; the energy of these potential-only models is
reported with the LDA exchange-correlation energy density.

Pins (tests/test_oracle_mgga.py): the Becke-Roussel potential of the hydrogen
1s density equals the exact exchange (= minus Hartree) potential; Q equals the
curvature of the exact spherically averaged exchange hole of a set of
orbitals; exchange scaling v[rho_l](r) = l v[rho](l r); tau of plane waves in
closed form; g of a cosine-modulated density in closed form.
"""
from __future__ import annotations

import numpy as np

from .tdks import C_LIGHT, Grid, first_derivative, gradient, laplacian, lda_pz81, pz81_correlation

BR_GAMMA = 1.0
TB09_ALPHA = -0.012
TB09_BETA = 1.023          # bohr^(1/2)
RHO_MIN = 1e-30


def kinetic_energy_density(psi, kpts, kw, A, grid: Grid, gauge: str = "velocity"):
    """tau(r) = sum_k w_k sum_n 2 * 1/2 |(grad_h + i kappa) w_nk(r)|^2, the
    spin-saturated kinetic energy density of the Bloch orbitals (reading:
    gauge-invariant form, kappa = k + A/c, k alone in the length gauge)."""
    tau = np.zeros(grid.shape)
    for ik, k in enumerate(kpts):
        kappa = np.asarray(k, dtype=np.float64) + (np.asarray(A) / C_LIGHT if gauge == "velocity" else 0.0)
        W = psi[ik]
        acc = np.zeros(grid.shape)
        for mu in range(3):
            d = first_derivative(W, mu, grid) + 1j * kappa[mu] * W
            acc += np.sum(np.abs(d) ** 2, axis=0)
        tau += kw[ik] * acc          # 2 (spin) x 1/2
    return tau


def br89_q(rho_s, grad_sq_s, lap_s, T_s, gamma: float = BR_GAMMA):
    """Q_s = (1/6)(lap rho_s - 2 gamma D_s), D_s = T_s - |grad rho_s|^2 / (4 rho_s)."""
    D = T_s - 0.25 * grad_sq_s / rho_s
    return (lap_s - 2.0 * gamma * D) / 6.0


def _br_f(x):
    return x * np.exp(-2.0 * x / 3.0) / (x - 2.0)


def br89_x(y):
    """The root x of x e^(-2x/3) / (x - 2) = y for every y (array): the left
    side falls from 0 to -inf on (0, 2) and from +inf to 0 on (2, inf), so
    y < 0 has its root in (0, 2) and y > 0 in (2, inf); y = +-inf gives 2.
    Plain bisection, halving until the midpoint equals an end."""
    y = np.asarray(y, dtype=np.float64)
    lo = np.where(y < 0, 0.0, 2.0)
    hi = np.where(y < 0, 2.0, 4.0)
    grow = (y > 0) & np.isfinite(y)
    for _ in range(64):                       # bracket of the y > 0 branch
        with np.errstate(divide="ignore", invalid="ignore"):
            g = grow & (_br_f(hi) > y)
        if not g.any():
            break
        lo = np.where(g, hi, lo)
        hi = np.where(g, 2.0 * hi, hi)
    inf = ~np.isfinite(y)
    active = ~inf
    for _ in range(2200):
        mid = 0.5 * (lo + hi)
        active &= (mid > lo) & (mid < hi)
        if not active.any():
            break
        with np.errstate(divide="ignore", invalid="ignore"):
            right = _br_f(mid) > y
        lo = np.where(active & right, mid, lo)
        hi = np.where(active & ~right, mid, hi)
    x = 0.5 * (lo + hi)
    return np.where(inf, 2.0, x)


def br89_potential(rho_s, grad_sq_s, lap_s, T_s, gamma: float = BR_GAMMA):
    """Becke-Roussel exchange-hole potential of one spin channel (pointwise
    arrays: rho_s, |grad rho_s|^2, lap rho_s, T_s = sum |grad psi|^2)."""
    rho_s = np.asarray(rho_s, dtype=np.float64)
    Q = br89_q(rho_s, grad_sq_s, lap_s, T_s, gamma)
    with np.errstate(divide="ignore"):
        y = np.where(Q == 0.0, np.inf, (2.0 / 3.0) * np.pi ** (2.0 / 3.0) * rho_s ** (5.0 / 3.0) / Q)
    x = br89_x(y)
    ex = np.exp(-x)
    b = np.cbrt(x ** 3 * ex / (8.0 * np.pi * rho_s))
    return -(1.0 - ex - 0.5 * x * ex) / b


def tb09_g(rho, grid: Grid):
    """g = (1/Omega) h^3 sum |grad_h rho| / rho over points with rho >= 1e-30."""
    gx, gy, gz = gradient(rho, grid)
    m = rho >= RHO_MIN
    r = np.where(m, rho, 1.0)
    ratio = np.where(m, np.sqrt(gx * gx + gy * gy + gz * gz) / r, 0.0)
    return grid.dV * float(np.sum(ratio)) / grid.volume


def tb09_c(rho, grid: Grid):
    """c = alpha + beta sqrt(g)."""
    return TB09_ALPHA + TB09_BETA * np.sqrt(tb09_g(rho, grid))


def mbj_pointwise(rho, grad_sq, lap, tau, c):
    """v_x = c v_BR + (3c - 2)(1/pi) sqrt(5/12) sqrt(2 t_s / rho_s) from the
    total (spin-saturated) rho, |grad rho|^2, lap rho and tau, split into one
    spin channel: rho_s = rho/2, |grad rho_s|^2 = |grad rho|^2 / 4,
    lap rho_s = lap rho / 2, t_s = tau/2, T_s = 2 t_s. Arrays with rho >= 1e-30."""
    rho_s = 0.5 * np.asarray(rho, dtype=np.float64)
    t_s = 0.5 * np.asarray(tau, dtype=np.float64)
    vbr = br89_potential(rho_s, 0.25 * np.asarray(grad_sq), 0.5 * np.asarray(lap), 2.0 * t_s)
    kin = np.sqrt(5.0 / 12.0) / np.pi * np.sqrt(2.0 * t_s / rho_s)
    return c * vbr + (3.0 * c - 2.0) * kin


def mbj_exchange(rho, tau, grid: Grid, c: float):
    """The exchange potential on the grid: grad rho and lap rho by the 9-point
    differences, zero where rho < 1e-30."""
    rho = np.asarray(rho, dtype=np.float64)
    gx, gy, gz = gradient(rho, grid)
    lap = laplacian(rho, grid)
    m = rho >= RHO_MIN
    v = np.zeros_like(rho)
    v[m] = mbj_pointwise(rho[m], (gx * gx + gy * gy + gz * gz)[m], lap[m], np.asarray(tau)[m], c)
    return v


def mgga_potential(psi, kpts, kw, A, rho, grid: Grid, kind: str, gauge: str = "velocity"):
    """(v_xc, eps_xc, c) for kind "tb09" (c from the density) or "bj" (c = 1):
    v_xc = v_x + PZ81 correlation; eps_xc is the LDA energy density (the
    potential has no energy functional of its own)."""
    tau = kinetic_energy_density(psi, kpts, kw, A, grid, gauge)
    c = tb09_c(rho, grid) if kind == "tb09" else 1.0
    vx = mbj_exchange(rho, tau, grid, c)
    vc, _ = pz81_correlation(rho)
    _, e = lda_pz81(rho)
    return vx + vc, e, c
