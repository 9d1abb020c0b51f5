"""Workflow of the learned multiscale coupling (Sec. 5), built from the
library's entry points: prepare a cell's ground state, drive copies of it with
field histories on the batch path to make training trajectories, train the
current surrogate with the library's kernels, and run the coupled slab with
or without it. Only orchestration and field tables live here; every step of
the method runs in libtddft.so."""
from __future__ import annotations

import time

import numpy as np

from .binding import Multiscale, Surrogate, TDDFT, TDDFTBatch


def ground_state(system, *, n_iter=300, tau=0.02, precision="c128", imag_time=None):
    """Orbitals and the energies of the last two of n_iter imaginary-time
    iterations of step tau. With imag_time, tau is the largest of 0.06, 0.05, 0.04, ... that the
    library accepts for this cell (tau lambda_max <= 1.59) and n_iter covers
    that much imaginary time."""
    from .binding import EUNSTABLE, TDDFTError
    def run(t, n, tau):
        # energies of the last two iterations only (one host round trip each)
        if n > 2:
            t.ground_state(n - 2, tau, energies=False)
        return t.ground_state(min(n, 2), tau)
    with TDDFT(system, precision=precision) as t:
        t.set_potential()
        if imag_time is None:
            E = run(t, n_iter, tau)
        else:
            for tau in (0.06, 0.05, 0.04, 0.033, 0.028, 0.024, 0.02, 0.016, 0.012, 0.008):
                try:
                    E = run(t, int(round(imag_time / tau)), tau)
                    break
                except TDDFTError as e:
                    if e.status != EUNSTABLE:
                        raise
            else:
                raise RuntimeError("no stable imaginary-time step")
        psi = t.orbitals()
    return psi, E


def micro_table(a_macro, n_sub, axis):
    """Cell field table [(T - 1) n_sub + 1][3] from macroscopic samples: A
    along `axis`, linear between consecutive samples, as the coupled run
    feeds its cells."""
    a = np.asarray(a_macro, dtype=np.float64)
    T = a.shape[0]
    tab = np.zeros(((T - 1) * n_sub + 1, 3))
    for s in range(T - 1):
        for u in range(n_sub):
            tab[s * n_sub + u, axis] = a[s] + (u / n_sub) * (a[s + 1] - a[s])
    tab[-1, axis] = a[-1]
    return tab


def trajectories(system, psi0, A_macro, *, n_sub, axis=0, precision="mixed"):
    """Drive one copy of the cell per row of A_macro [n_traj][T] on the batch
    path; returns the current at the macroscopic times, J [n_traj][T]
    (J[:, 0] = 0: the cell starts at rest), and the device time (s)."""
    A_macro = np.asarray(A_macro, dtype=np.float64)
    n_traj, T = A_macro.shape
    cells = []
    for _ in range(n_traj):
        c = _copy_with_orbitals(system, psi0)
        cells.append(c)
    tabs = [micro_table(A_macro[i], n_sub, axis) for i in range(n_traj)]
    t0 = time.perf_counter()
    with TDDFTBatch(cells, precision=precision) as b:
        Js = b.propagate(tabs)
    el = time.perf_counter() - t0
    J = np.zeros((n_traj, T))
    for i in range(n_traj):
        J[i, 1:] = Js[i][n_sub - 1::n_sub, axis]
    return J, el


def _copy_with_orbitals(system, psi0):
    import copy
    c = copy.copy(system)
    c.psi0 = psi0
    return c


def train(A_macro, J_macro, params, *, window, hidden, a_scale, j_scale, epochs, batch, seed=0, lr=1e-3,
          a_fit=None, cosine=False):
    """A Surrogate trained on the trajectories; returns it and the losses.

    With a_fit, the skip weights and output bias are first set to the
    least-squares linear response of the trajectories whose largest |A| is
    within a_fit and kept fixed; Adam then trains the hidden layers on what
    the linear response leaves (the nonlinear part)."""
    nn = Surrogate(window, hidden, params, a_scale=a_scale, j_scale=j_scale, lr=lr)
    if a_fit is not None:
        nn.fit_linear(A_macro, J_macro, a_fit=a_fit)
    losses = nn.train(A_macro, J_macro, epochs=epochs, batch=batch, seed=seed, cosine=cosine,
                      freeze_linear=a_fit is not None)
    return nn, losses


def run_slab(system, psi0, inc, *, n_x, x0, n_mat, dx, dt, n_sub, axis=0, precision="mixed", nn=None,
             a_max=None, sentinels=(), check_every=50, tol=1e-3):
    """One coupled run; returns A, I [n_macro][n_x], the wall time (s) and the
    run's status."""
    import torch
    n_macro = np.asarray(inc).shape[0] - 1
    with Multiscale(system, psi0, n_x=n_x, x0=x0, n_mat=n_mat, dx=dx, dt=dt, n_sub=n_sub, axis=axis,
                    precision=precision) as ms:
        if nn is not None:
            ms.attach_surrogate(nn, a_max=a_max, sentinels=sentinels, check_every=check_every, tol=tol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        A, I = ms.step(n_macro, inc)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st = ms.status()
    return A, I, el, st
