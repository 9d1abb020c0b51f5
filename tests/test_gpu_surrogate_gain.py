"""What the trained surrogate gains over the cells it replaces (Sec. 5).

The cell of every macroscopic point (12^3 diamond-like cell, 8 orbitals,
2^3 k-points) is first relaxed to its ground state; copies of it driven by
seeded, varied fields on the batch path give the training trajectories; the
network is trained by the library's own kernels; then the same slab and
incident pulse run once with a cell at every point and once through the
network with two sentinel cells. The test states the gain: the coupled run
is several times faster, the sentinels never trip, and the transmitted and
reflected field stays within the stated error of the cells-only run.
"""
import numpy as np
import pytest

import synth
from oracle import maxwell
from gpu_helpers import announce

pytestmark = pytest.mark.gpu
C = maxwell.C_LIGHT


def test_surrogate_coupled_slab_gain():
    from paper_1804_01404_amd import pipeline
    n_sub, dt = 4, 0.32
    cell = synth.multiscale_cell(nk=2, n=12, n_orb=8, dt=dt / n_sub)
    announce("surrogate gain: ground state")
    psi, E = pipeline.ground_state(cell, n_iter=3000, tau=0.06)
    assert abs(E[-1] - E[-2]) < 1e-6 * abs(E[-1])
    T = 300
    A_tr = synth.random_field_tables(48, T, dt, 1, a_max=12.0)
    announce("surrogate gain: training trajectories")
    J_tr, t_gen = pipeline.trajectories(cell, psi, A_tr, n_sub=n_sub, axis=0)
    a_scale, j_scale = float(np.abs(A_tr).max()), float(np.abs(J_tr).max())
    W, H = T, 16
    announce("surrogate gain: training")
    nn, losses = pipeline.train(A_tr, J_tr, synth.surrogate_init(W, H, 1), window=W, hidden=H,
                                a_scale=a_scale, j_scale=j_scale, epochs=150, batch=256, seed=1, lr=2e-3)
    assert losses[-1] < 0.1 * losses[0]
    dx, n_mat, n_vac = 147.6, 16, 12
    n_x = n_mat + 2 * n_vac
    inc = synth.incident_table(T, dt, dx, delay=0.0, E0=3e-3, omega=1.55 / 27.211386245988, T=100.0)
    announce("surrogate gain: slab with cells")
    A_c, I_c, t_cells, st_c = pipeline.run_slab(cell, psi, inc, n_x=n_x, x0=n_vac, n_mat=n_mat, dx=dx, dt=dt,
                                                n_sub=n_sub, axis=0)
    announce("surrogate gain: slab with the network")
    with nn:
        A_s, I_s, t_net, st_s = pipeline.run_slab(cell, psi, inc, n_x=n_x, x0=n_vac, n_mat=n_mat, dx=dx,
                                                  dt=dt, n_sub=n_sub, axis=0, nn=nn, a_max=a_scale,
                                                  sentinels=[0, n_mat // 2], check_every=50, tol=0.1)
    field_err = float(np.max(np.abs(A_s - A_c)) / np.max(np.abs(A_c)))
    speedup = t_cells / t_net
    announce(f"surrogate gain: speedup {speedup:.1f}x, field error {field_err:.3g}, "
             f"sentinel error {st_s['last_check']:.3g}, cells {t_cells:.2f} s, network {t_net:.2f} s")
    assert st_c["mode"] == "cells"
    assert st_s["mode"] == "network" and st_s["fallbacks"] == 0
    assert speedup > 3.0
    assert field_err < 0.2
