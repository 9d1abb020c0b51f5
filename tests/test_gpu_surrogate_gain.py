"""What the trained surrogate gains over the cells it replaces (Sec. 5).

The cell of every macroscopic point (12^3 diamond-like cell, 8 orbitals,
2^3 k-points) is first relaxed to its ground state (converged until its
current in zero field is below 1e-6 of the training currents: a state that
still carries a drifting current cannot be mapped from A alone); copies of
it driven by seeded, varied fields and random cos^2 pulses on the batch path
give the training trajectories; the library sets the network's linear part to the
least-squares linear response of the weak-field trajectories and trains the
hidden layers (Adam, cosine schedule) on the rest; then the same slab and
incident pulse run once with a cell at every point and once through the
network with two sentinel cells checked every 50 steps at the stated
spot-check error of 1e-3. The test states the gain: the coupled run is
faster than the cells-only run (by 1.2x at least: of the 16 points two stay
cells as sentinels, and each macroscopic step adds its own launches and a
host wait, while the cells-only run steps all 16 cells in one batched graph;
the 256-point slab of the benchmark shows the gain at scale), the sentinels
never trip (no fallback), and the transmitted and reflected field stays
within 2e-3 of the cells-only run.
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
    psi, E = pipeline.ground_state(cell, n_iter=12000, tau=0.06)
    assert abs(E[-1] - E[-2]) < 1e-12 * abs(E[-1])
    T = 300
    # varied fields and random cos^2 pulses (peak field 1e-4 .. 1e-2 a.u., 0.5 .. 3 eV)
    P, _ = synth.random_pulse_tables(64, T, dt, 3, e0_range=(1e-4, 1e-2), ev_range=(0.5, 3.0),
                                     t_range=(40.0, 200.0))
    A_tr = np.vstack([synth.random_field_tables(192, T, dt, 1, a_max=12.0), P])
    announce("surrogate gain: training trajectories")
    J_tr, t_gen = pipeline.trajectories(cell, psi, A_tr, n_sub=n_sub, axis=0)
    a_scale, j_scale = float(np.abs(A_tr).max()), float(np.abs(J_tr).max())
    zero = np.zeros((1, T))
    J0, _ = pipeline.trajectories(cell, psi, zero, n_sub=n_sub, axis=0)
    assert np.max(np.abs(J0)) < 1e-6 * j_scale     # the ground state carries no current
    W, H = T, 16
    announce("surrogate gain: training")
    nn, losses = pipeline.train(A_tr, J_tr, synth.surrogate_init(W, H, 1), window=W, hidden=H,
                                a_scale=a_scale, j_scale=j_scale, epochs=60, batch=256, seed=1, lr=2e-3,
                                a_fit=a_scale / 8, cosine=True)
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
                                                  sentinels=[0, n_mat // 2], check_every=50, tol=1e-3)
    field_err = float(np.max(np.abs(A_s - A_c)) / np.max(np.abs(A_c)))
    speedup = t_cells / t_net
    announce(f"surrogate gain: speedup {speedup:.1f}x, field error {field_err:.3g}, "
             f"sentinel error {st_s['last_check']:.3g}, cells {t_cells:.2f} s, network {t_net:.2f} s")
    assert st_c["mode"] == "cells"
    assert st_s["mode"] == "network" and st_s["fallbacks"] == 0 and st_s["last_check"] < 1e-3
    assert speedup > 1.2
    assert field_err < 2e-3
