"""Pins of the oracle's multiscale step (Sec. 5) and of the surrogate network.

Maxwell (Eq. Maxwell_ms, leapfrog + Mur):
* at Courant number 1 the leapfrog update is exact for any right- or
  left-moving profile, the Mur ends absorb exactly and the left end injects an
  incident wave exactly;
* at Courant number < 1 a discrete plane wave with the leapfrog dispersion
  relation sin(w dt/2) = S sin(k dX/2) is advanced exactly;
* with a plasma source I = -(n_e/c) A the discrete dispersion becomes
  4 sin^2(w dt/2) = 4 S^2 sin^2(k dX/2) + w_p^2 dt^2, w_p^2 = 4 pi n_e;
* the coupled driver with real TDKS cells holding a constant orbital (a
  free-electron medium: each cell returns -(n_e/c) A) equals the scalar plasma
  model step by step.

Surrogate:
* the backward pass equals central finite differences of the loss (FP64);
* with zero hidden weights the forward pass is the closed form
  w3 . tanh(b2) + b3 + ws . x;
* the first Adam step moves every parameter by lr g / (|g| + eps);
* causal windows of a short hand-made trajectory.
"""
import math

import numpy as np
import pytest

import synth

from oracle import maxwell, surrogate, tdks
from synth.systems import rng_for

C = maxwell.C_LIGHT


def _profile(u):
    """A compactly supported bump (zero outside 20 < u < 40)."""
    v = np.where((u > 20.0) & (u < 40.0), np.sin(math.pi * (u - 20.0) / 20.0) ** 2, 0.0)
    return v * np.cos(0.4 * u)


def test_leapfrog_exact_at_courant_one():
    n, dx = 200, 2.0
    dt = dx / C
    X = np.arange(n) * dx

    def exact(t):
        # a right-moving bump and a left-moving one starting near the far end
        return _profile((X - C * t) / dx) + 0.5 * _profile(((n - 1) * dx - X - C * t) / dx)
    A_prev, A_now = exact(-dt), exact(0.0)
    I = np.zeros(n)
    for s in range(1, 260):
        A_new = maxwell.leapfrog(A_now, A_prev, I, dx, dt)
        maxwell.mur_ends(A_new, A_now, dx, dt)
        ref = exact(s * dt)
        assert np.max(np.abs(A_new - ref)) < 1e-13
        A_prev, A_now = A_now, A_new
    # both bumps have left through the absorbing ends
    assert np.max(np.abs(A_now)) < 1e-13


def test_mur_absorbs_and_injects_exactly_at_courant_one():
    n, dx = 120, 3.0
    dt = dx / C
    steps = 600
    inc = synth.incident_table(steps, dt, dx, delay=5.0, E0=2e-3, omega=6.0, T=2.0)
    A_prev = np.zeros(n)
    A_now = np.zeros(n)
    I = np.zeros(n)
    X = np.arange(n) * dx
    for s in range(steps):
        A_new = maxwell.leapfrog(A_now, A_prev, I, dx, dt)
        maxwell.mur_ends(A_new, A_now, dx, dt, inc[s], inc[s + 1])
        t = (s + 1) * dt
        ref = synth.cos2_pulse_potential(t - 5.0 - X / C, 2e-3, 6.0, 2.0)
        assert np.max(np.abs(A_new - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))
        A_prev, A_now = A_now, A_new
    # after the pulse has crossed, the field is the constant tail of the
    # incident potential; E = 0 everywhere
    assert np.max(np.abs(A_now - A_prev)) < 1e-12


def test_discrete_plane_wave_dispersion():
    n, dx = 64, 1.7
    S = 0.6
    dt = S * dx / C
    k = 2 * math.pi * 5 / (n * dx)
    w = 2.0 / dt * math.asin(S * math.sin(k * dx / 2))
    X = np.arange(n) * dx
    wave = lambda t: np.cos(k * X - w * t)
    A_new = maxwell.leapfrog(wave(0.0), wave(-dt), np.zeros(n), dx, dt)
    assert np.max(np.abs(A_new[1:-1] - wave(dt)[1:-1])) < 1e-12


def test_plasma_dispersion():
    n, dx = 64, 1.7
    S = 0.5
    dt = S * dx / C
    n_e = 0.03
    k = 2 * math.pi * 3 / (n * dx)
    wp2 = 4 * math.pi * n_e
    w = 2.0 / dt * math.asin(math.sqrt(S * S * math.sin(k * dx / 2) ** 2 + wp2 * dt * dt / 4))
    X = np.arange(n) * dx
    wave = lambda t: np.cos(k * X - w * t)
    A0 = wave(0.0)
    A_new = maxwell.leapfrog(A0, wave(-dt), -(n_e / C) * A0, dx, dt)
    assert np.max(np.abs(A_new[1:-1] - wave(dt)[1:-1])) < 1e-12


def _plane_wave_cell(dt_micro):
    """A free-electron cell: one constant orbital (G = 0) at k = 0, V = 0, no
    projectors, no Hartree or xc. Its current is -(2/Omega)(A/c) |w|^2 and the
    Taylor step keeps |w|^2 to O((|A/c|^2 dt/2)^6)."""
    n, L = (8, 8, 8), (5.0, 5.0, 5.0)
    grid = tdks.Grid(n, L, "periodic")
    psi = np.full((1, 1) + grid.shape, 1.0 / math.sqrt(grid.volume), dtype=np.complex128)
    cell = tdks.TDKS(n, L, "periodic", np.zeros((1, 3)), [1.0], psi, dt_micro, np.zeros(grid.shape), [],
                     hartree=False, xc=False)
    n_e = 2.0 / grid.volume
    return cell, n_e


def test_driver_with_plane_wave_cells_is_the_plasma_model():
    n_x, x0, n_mat = 24, 6, 10
    dx, n_sub = 40.0, 3
    dt = 0.6 * dx / C
    cells = []
    for _ in range(n_mat):
        cell, n_e = _plane_wave_cell(dt / n_sub)
        cells.append(cell)
    ms = maxwell.Multiscale(n_x, x0, n_mat, dx, dt, n_sub, 2, cells)
    steps = 30
    inc = synth.incident_table(steps, dt, dx, delay=0.0, E0=5e-3, omega=0.2, T=12.0)
    As, Is = ms.step(steps, inc)
    # scalar model: the same leapfrog with I = -(n_e/c) A inside the medium
    A_prev, A_now, I = np.zeros(n_x), np.zeros(n_x), np.zeros(n_x)
    mat = slice(x0, x0 + n_mat)
    Amax, Imax = np.max(np.abs(As)), np.max(np.abs(Is))
    for s in range(steps):
        A_new = maxwell.leapfrog(A_now, A_prev, I, dx, dt)
        maxwell.mur_ends(A_new, A_now, dx, dt, inc[s], inc[s + 1])
        I = np.zeros(n_x)
        I[mat] = -(n_e / C) * A_new[mat]
        assert np.max(np.abs(As[s] - A_new)) < 1e-12 * Amax
        assert np.max(np.abs(Is[s] - I)) < 1e-12 * Imax
        A_prev, A_now = A_now, A_new
    assert np.max(np.abs(As[-1][mat])) > 1e-3   # the pulse reached the medium


# ------------------------------------------------------------------ surrogate
W_, H_ = 7, 5


def _theta(seed):
    rng = rng_for(seed)
    return rng.normal(scale=0.5, size=surrogate.n_params(W_, H_))


def test_backward_equals_finite_differences():
    th = _theta(9901)
    rng = rng_for(9902)
    x = rng.normal(size=(11, W_))
    t = rng.normal(size=11)
    loss, g = surrogate.loss_and_grad(th, x, t, W_, H_)
    h = 1e-6
    fd = np.empty_like(th)
    for i in range(th.shape[0]):
        e = np.zeros_like(th)
        e[i] = h
        lp, _ = surrogate.loss_and_grad(th + e, x, t, W_, H_)
        lm, _ = surrogate.loss_and_grad(th - e, x, t, W_, H_)
        fd[i] = (lp - lm) / (2 * h)
    assert np.max(np.abs(g - fd)) < 1e-8 * max(1.0, np.max(np.abs(g)))


def test_forward_closed_form_without_hidden_weights():
    th = _theta(9903)
    W1, b1, W2, b2, w3, b3, ws = surrogate.unpack(th, W_, H_)
    W1 = np.zeros_like(W1)
    W2 = np.zeros_like(W2)
    th0 = surrogate.pack(W1, b1, W2, b2, w3, b3, ws)
    x = rng_for(9904).normal(size=(4, W_))
    y, _, _ = surrogate.forward(th0, x, W_, H_)
    ref = np.array([np.dot(w3, np.tanh(b2)) + b3[0] + np.dot(ws, xi) for xi in x])
    assert np.max(np.abs(y - ref)) < 1e-14


def test_first_adam_step_closed_form():
    th = _theta(9905)
    g = rng_for(9906).normal(size=th.shape)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    lr, eps = 3e-3, 1e-8
    th1, m1, v1 = surrogate.adam_step(th, g, m, v, 1, lr=lr, eps=eps)
    assert np.max(np.abs(th1 - (th - lr * g / (np.abs(g) + eps)))) < 1e-15
    assert np.max(np.abs(m1 - 0.1 * g)) < 1e-16
    assert np.max(np.abs(v1 - 0.001 * g * g)) < 1e-16


def test_windows_by_hand():
    A = np.array([[1.0, 2.0, 3.0, 4.0]])
    J = np.array([[10.0, 20.0, 30.0, 40.0]])
    X, Y = surrogate.windows(A, J, 3, a_scale=2.0, j_scale=10.0)
    assert np.array_equal(X, np.array([[0, 0, 0.5], [0, 0.5, 1.0], [0.5, 1.0, 1.5], [1.0, 1.5, 2.0]]))
    assert np.array_equal(Y, np.array([1.0, 2.0, 3.0, 4.0]))


def test_field_energy_plus_medium_work_is_conserved():
    """A pulse crossing a plasma slab (I = -(n_e/c) A in the medium, the
    free-electron response): the field energy plus the work done on the
    medium stays at the initial field energy while the pulse is inside the
    grid (to the O(dt^2) of the two energy differences), the medium gives its
    energy back after the pulse has passed (a reactive medium), and the
    energy leaves through the Mur ends."""
    n, dx, S, n_e = 400, 20.0, 0.5, 0.03
    dt = S * dx / C
    x0, n_mat = 250, 60
    X = np.arange(n) * dx

    def prof(u):
        return 1e-2 * np.where((u > 20) & (u < 60), np.sin(math.pi * (u - 20) / 40) ** 2, 0.0) * np.cos(0.35 * u)
    A_prev, A_now = prof((X + C * dt) / dx - 60), prof(X / dx - 60)
    I = np.zeros(n)
    A_hist, I_hist = [A_now[x0:x0 + n_mat].copy()], [I[x0:x0 + n_mat].copy()]
    em0 = maxwell.em_energy(A_now, A_prev, dx, dt)
    dev, wmax = [], 0.0
    for s in range(700):
        A_new = maxwell.leapfrog(A_now, A_prev, I, dx, dt)
        maxwell.mur_ends(A_new, A_now, dx, dt)
        I_new = np.zeros(n)
        I_new[x0:x0 + n_mat] = -(n_e / C) * A_new[x0:x0 + n_mat]
        A_prev, A_now, I = A_now, A_new, I_new
        A_hist.append(A_now[x0:x0 + n_mat].copy())
        I_hist.append(I[x0:x0 + n_mat].copy())
        if s < 500:
            W = maxwell.medium_work(np.array(A_hist), np.array(I_hist), dx, dt)[-1]
            wmax = max(wmax, abs(W))
            dev.append(abs(maxwell.em_energy(A_now, A_prev, dx, dt) + W - em0) / em0)
    assert wmax > 1e-2 * em0                   # the medium takes a visible share
    # the two energy differences are offset by half a step: O(dt^2), ~1e-3 here;
    # a wrong sign, factor or missing dX in the work moves the sum by >= 3e-2
    assert max(dev) < 3e-3
    assert abs(W) < 1e-3 * wmax                # given back after the pulse
    assert maxwell.em_energy(A_now, A_prev, dx, dt) < 1e-2 * em0


def test_medium_work_closed_form():
    """Constant field and current: W_n = n dt dX n_mat I E."""
    dx, dt, n_mat, steps = 5.0, 0.1, 7, 9
    E0, I0 = 2e-3, -3e-4
    A = np.array([-C * E0 * dt * s * np.ones(n_mat) for s in range(steps + 1)])
    Ih = np.full((steps + 1, n_mat), I0)
    W = maxwell.medium_work(A, Ih, dx, dt)
    ref = np.arange(steps + 1) * dt * dx * n_mat * I0 * E0
    assert np.max(np.abs(W - ref)) < 1e-15 * abs(ref[-1])


def test_linear_fit_recovers_an_exact_linear_response():
    """Currents made by a known causal filter plus a constant (and, for
    strong trajectories beyond a_fit, a cubic term): the least-squares fit
    over the weak trajectories returns the filter and the constant."""
    rng = rng_for(31)
    W, T, n = 24, 60, 20
    A = np.cumsum(rng.normal(size=(n, T)), axis=1) * 0.05
    A[:, 0] = 0.0
    A[n // 2:] *= 40.0                          # strong trajectories
    k = rng.normal(size=W)
    J = np.zeros_like(A)
    for i in range(n):
        for t in range(T):
            win = np.zeros(W)
            seg = A[i, max(0, t - W + 1):t + 1]
            win[W - seg.shape[0]:] = seg
            J[i, t] = win @ k + 0.3
    J[n // 2:] += 0.01 * A[n // 2:] ** 3
    a_scale, j_scale = 2.0, 5.0
    a_fit = np.max(np.abs(A[: n // 2]))
    ws, b3 = surrogate.fit_linear(A, J, W, a_scale, j_scale, a_fit, lambda_rel=0.0)
    assert np.max(np.abs(ws - k * a_scale / j_scale)) < 1e-9 * np.max(np.abs(k))
    assert abs(b3 - 0.3 / j_scale) < 1e-10
