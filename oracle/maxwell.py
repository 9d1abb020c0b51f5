"""Plain FP64 oracle of the multiscale light-propagation step (test infrastructure).

THIS MODULE IS TEST INFRASTRUCTURE: only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it. It shares no code with the HIP
library.

Sec. 5: a linearly polarised pulse at normal incidence on a slab. The vector
potential A(X, t) along the polarisation axis obeys the 1-D wave equation with
the macroscopic current as source (Eq. Maxwell_ms),

    (1/c^2) d^2A/dt^2 - d^2A/dX^2 = (4 pi / c) I(X, t),

and every macroscopic point X inside the medium holds its own microscopic cell
whose Bloch orbitals evolve under the uniform A(X, t) (Eq. TDKS_ms); its
current I(X, t) (Eq. macro_current) feeds back into the wave equation.

Discretisation (readings, the paper gives none):
* central differences in X and t (leapfrog):
  A^{n+1}_j = 2 A^n_j - A^{n-1}_j + S^2 (A^n_{j+1} - 2 A^n_j + A^n_{j-1})
              + 4 pi c dt^2 I^n_j,          S = c dt / dX;
* first-order Mur absorbing ends (Mur 1981):
  A^{n+1}_0 = A^n_1 + q (A^{n+1}_1 - A^n_0), q = (S - 1) / (S + 1), and the
  mirror image at the far end;
* each macroscopic step of dt is n_sub microscopic TDKS steps of dt / n_sub,
  with A interpolated linearly between A^n_j and A^{n+1}_j; the current of a
  cell after its last microscopic step is I^{n+1}_j;
* the medium starts at rest: I^0 = 0 (the pulse starts in the vacuum in front
  of the surface and the cells hold the ground state, Sec. 5).
"""
from __future__ import annotations

import math

import numpy as np

C_LIGHT = 137.035999084


def leapfrog(A_now, A_prev, I, dx, dt):
    """Interior update of the wave equation (Eq. Maxwell_ms); end points are
    returned unchanged and set by ``mur_ends``."""
    A_now = np.asarray(A_now, dtype=np.float64)
    S2 = (C_LIGHT * dt / dx) ** 2
    A_new = A_now.copy()
    n = A_now.shape[0]
    for j in range(1, n - 1):
        A_new[j] = (2.0 * A_now[j] - A_prev[j] + S2 * (A_now[j + 1] - 2.0 * A_now[j] + A_now[j - 1])
                    + 4.0 * math.pi * C_LIGHT * dt * dt * I[j])
    return A_new


def mur_ends(A_new, A_now, dx, dt, inc_now=(0.0, 0.0), inc_new=(0.0, 0.0)):
    """First-order Mur absorbing boundary at both ends (in place). At the
    left end the condition acts on the scattered field A - A_inc, so that an
    incident wave given at X_0 and X_1 (inc_now at t_n, inc_new at t_{n+1})
    enters the grid while reflected waves leave it."""
    S = C_LIGHT * dt / dx
    q = (S - 1.0) / (S + 1.0)
    n = A_new.shape[0]
    A_new[0] = inc_new[0] + (A_now[1] - inc_now[1]) + q * ((A_new[1] - inc_new[1]) - (A_now[0] - inc_now[0]))
    A_new[n - 1] = A_now[n - 2] + q * (A_new[n - 2] - A_now[n - 1])
    return A_new


def em_energy(A_now, A_prev, dx, dt):
    """Field energy per unit area, (1/8 pi) sum (E^2 + B^2) dX with
    E = -(1/c) dA/dt (backward difference) and B = dA/dX (forward
    difference, summed over the links)."""
    E = -(A_now - A_prev) / (C_LIGHT * dt)
    B = np.diff(A_now) / dx
    return (np.sum(E * E) + np.sum(B * B)) * dx / (8.0 * math.pi)


def medium_work(A_hist, I_hist, dx, dt):
    """Work of the field on the medium per unit area after each step:
    W_n = sum_{s<n} dt dX sum_m (I_m^s + I_m^{s+1})/2 E_m^{s+1/2}, with
    E^{s+1/2} = -(A^{s+1} - A^s)/(c dt); A_hist, I_hist [(n + 1)][n_mat] at
    the medium points from t_0 (I^0 = 0). Returns W [n + 1] (W_0 = 0)."""
    A = np.asarray(A_hist, dtype=np.float64)
    I = np.asarray(I_hist, dtype=np.float64)
    E = -(A[1:] - A[:-1]) / (C_LIGHT * dt)
    inc = dt * dx * np.sum(0.5 * (I[:-1] + I[1:]) * E, axis=1)
    return np.concatenate([[0.0], np.cumsum(inc)])


class Multiscale:
    """Coupled Maxwell + microscopic cells (Sec. 5). ``cells`` are objects with
    ``propagate(A_table) -> J`` (the oracle's TDKS); the material occupies the
    grid points x0 .. x0 + n_mat - 1."""

    def __init__(self, n_x, x0, n_mat, dx, dt, n_sub, axis, cells):
        assert 1 <= x0 and x0 + n_mat <= n_x - 1 and len(cells) == n_mat
        self.n_x, self.x0, self.n_mat = n_x, x0, n_mat
        self.dx, self.dt, self.n_sub, self.axis = dx, dt, n_sub, axis
        self.cells = cells
        self.A_now = np.zeros(n_x)
        self.A_prev = np.zeros(n_x)
        self.I = np.zeros(n_x)

    def step(self, n_macro, inc=None):
        """Advance n_macro macroscopic steps. ``inc`` [n_macro + 1][2] is the
        incident A at X_0 and X_1 for t_n .. t_{n + n_macro} (or None: no
        incident wave). Returns (A, I) after each step, both [n_macro][n_x]."""
        As = np.empty((n_macro, self.n_x))
        Is = np.empty((n_macro, self.n_x))
        for n in range(n_macro):
            A_new = leapfrog(self.A_now, self.A_prev, self.I, self.dx, self.dt)
            if inc is None:
                mur_ends(A_new, self.A_now, self.dx, self.dt)
            else:
                mur_ends(A_new, self.A_now, self.dx, self.dt, inc[n], inc[n + 1])
            I_new = np.zeros(self.n_x)
            for m, cell in enumerate(self.cells):
                j = self.x0 + m
                tab = np.zeros((self.n_sub + 1, 3))
                for s in range(self.n_sub + 1):
                    tab[s, self.axis] = self.A_now[j] + (s / self.n_sub) * (A_new[j] - self.A_now[j])
                J = cell.propagate(tab)
                I_new[j] = J[-1, self.axis]
            self.A_prev, self.A_now, self.I = self.A_now, A_new, I_new
            As[n] = A_new
            Is[n] = I_new
        return As, Is
