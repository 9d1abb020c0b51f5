"""Pins of the oracle's operators against closed forms and brute force.

* finite-difference weights: textbook rationals and Taylor moments;
* plane waves are exact eigenvectors of the discrete h with the known
  finite-difference symbol, and the whole self-consistent step reduces to a
  scalar recursion for them;
* the dense 8^3 Hamiltonian built column by column equals an independent
  Kronecker-sum construction; the propagator equals the eigen-decomposition
  form P4(-i eps dt)^n exactly; norm and energy follow the closed forms;
* Hermiticity of h and projector normalisation.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import tdks
from synth.systems import build_system, rng_for
from oracle_helpers import tiny_periodic

C = 137.035999084


def _p4(z):
    return 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24


# ---------------------------------------------------------------- FD weights
def test_fd_weights_textbook_values():
    c, d = tdks.fd_weights(4)
    # Fornberg (1988), Math. Comp. 51, 699, Table 1: 8th-order central weights
    golden = {}
    with open(__file__.replace("test_oracle_operators.py", "golden/fd_weights_8th_order.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                key, *vals = line.split()
                golden[key] = [Fraction(v) for v in vals]
    assert c == golden["second"]
    assert d == golden["first"]


@pytest.mark.parametrize("M", [1, 2, 3, 4])
def test_fd_moments(M):
    c, d = tdks.fd_weights(M)
    assert c[0] + 2 * sum(c[1:]) == 0
    assert sum(cm * m * m for m, cm in enumerate(c) if m) == 1
    for p in range(4, 2 * M + 1, 2):
        assert sum(cm * m ** p for m, cm in enumerate(c) if m) == 0
    assert 2 * sum(dm * (m + 1) for m, dm in enumerate(d)) == 1
    for p in range(3, 2 * M, 2):
        assert sum(dm * (m + 1) ** p for m, dm in enumerate(d)) == 0


def test_fd_symbol_limits():
    c, d = tdks.C2, tdks.D1
    K2 = lambda th: -c[0] - 2 * sum(c[m] * np.cos(m * th) for m in range(1, 5))
    K1 = lambda th: 2 * sum(d[m - 1] * np.sin(m * th) for m in range(1, 5))
    # the largest eigenvalue of -d^2 (times h^2) sits at theta = pi
    assert abs(K2(np.pi) - 6.501587301587302) < 1e-12
    th = np.linspace(0, np.pi, 1001)
    assert np.all(K2(th) <= K2(np.pi) + 1e-12)
    # 8th-order accuracy: K2 - th^2 ~ a th^10 and K1 - th ~ b th^9 as th -> 0
    r2 = [(K2(t) - t * t) / t ** 10 for t in (0.2, 0.3)]
    r1 = [(K1(t) - t) / t ** 9 for t in (0.2, 0.3)]
    assert abs(r2[0] / r2[1] - 1) < 0.05 and abs(r1[0] / r1[1] - 1) < 0.05


# ---------------------------------------------------------------- plane waves
def _plane_wave_setup(n=(12, 10, 8), cell=(7.2, 6.0, 5.6)):
    grid = tdks.Grid(n, cell, "periodic")
    x, y, z = grid.r_fields()
    return grid, (x, y, z)


def _symbols(G, h):
    c, d = tdks.C2, tdks.D1
    th = np.asarray(G) * np.asarray(h)
    K2 = -c[0] - 2 * sum(c[m] * np.cos(m * th) for m in range(1, 5))
    K1 = 2 * sum(d[m - 1] * np.sin(m * th) for m in range(1, 5))
    return K2, K1


def test_plane_wave_eigenvalue():
    grid, (x, y, z) = _plane_wave_setup()
    kappa = np.array([0.13, -0.07, 0.21])
    V0 = -0.37
    for m in [(0, 0, 0), (1, 0, 0), (2, -1, 3), (-5, 4, -3), (6, 5, 4)]:
        G = np.array([2 * np.pi * m[i] / grid.cell[i] for i in range(3)])
        w = np.exp(1j * (G[0] * x + G[1] * y + G[2] * z))[None] / np.sqrt(grid.volume)
        hw = tdks.apply_h(w, kappa, V0 * np.ones(grid.shape), [], grid)
        K2, K1 = _symbols(G, grid.h)
        eps = 0.5 * np.sum(K2 / np.array(grid.h) ** 2) + np.sum(kappa * K1 / np.array(grid.h)) \
            + 0.5 * kappa @ kappa + V0
        assert np.max(np.abs(hw - eps * w)) < 1e-12 * max(1.0, abs(eps)) * np.max(np.abs(w))


def test_plane_wave_selfconsistent_recursion():
    """Hartree + LDA on: a set of plane waves keeps rho uniform, so V_H = 0,
    V_xc is uniform and each orbital only picks up the scalar factor
    P4(-i eps_j(n) dt) each step; the current is the closed-form sum."""
    n, cell = (10, 10, 10), (6.0, 6.0, 6.0)
    grid = tdks.Grid(n, cell, "periodic")
    x, y, z = grid.r_fields()
    ms = [(0, 0, 0), (1, 0, 0), (0, -1, 0), (1, 1, 2)]
    kpt = np.array([[0.11, -0.04, 0.07]])
    dt, nsteps = 0.05, 6
    A0 = np.array([0.9, -0.4, 0.3])
    A = np.tile(A0, (nsteps + 1, 1))
    A[3:] *= 1.5   # change the field mid-run
    V0 = -0.21
    psi = np.empty((1, len(ms)) + grid.shape, dtype=np.complex128)
    Gs = []
    for j, m in enumerate(ms):
        G = np.array([2 * np.pi * m[i] / cell[i] for i in range(3)])
        Gs.append(G)
        psi[0, j] = np.exp(1j * (G[0] * x + G[1] * y + G[2] * z)) / np.sqrt(grid.volume)
    sysm = tdks.TDKS(n, cell, "periodic", kpt, [1.0], psi, dt, V0 * np.ones(grid.shape), [],
                     hartree=True, xc=True)
    J = sysm.propagate(A)
    # scalar recursion
    a = np.ones(len(ms), dtype=np.complex128)
    hv = np.array(grid.h)
    for step in range(nsteps):
        rho = 2 * np.sum(np.abs(a) ** 2) / grid.volume
        vxc = tdks.lda_pz81(np.array([rho]))[0][0]
        kap = kpt[0] + 0.5 * (A[step] + A[step + 1]) / C
        for j, G in enumerate(Gs):
            K2, K1 = _symbols(G, hv)
            eps = 0.5 * np.sum(K2 / hv ** 2) + np.sum(kap * K1 / hv) + 0.5 * kap @ kap + V0 + vxc
            a[j] *= _p4(-1j * eps * dt)
        kap1 = kpt[0] + A[step + 1] / C
        Jref = np.zeros(3)
        for j, G in enumerate(Gs):
            K2, K1 = _symbols(G, hv)
            Jref += 2 * np.abs(a[j]) ** 2 * (K1 / hv + kap1)
        Jref *= -1.0 / grid.volume
        assert np.allclose(J[step], Jref, rtol=1e-12, atol=1e-15)
    for j in range(len(ms)):
        assert np.max(np.abs(sysm.psi[0, j] - a[j] * psi[0, j])) < 1e-13 * np.max(np.abs(psi[0, j]))
    assert np.max(np.abs(sysm.v_h)) < 1e-12


# ---------------------------------------------------------------- dense 8^3
def _dense_system():
    rng = rng_for(808)
    n, L = 8, 5.2
    atoms = rng.uniform(0, L, size=(2, 3))
    s = build_system(name="dense8", n=(n, n, n), cell=(L, L, L), boundary="periodic", n_orb=2,
                     kpts=np.array([[0.17, -0.23, 0.05]]), kw=np.ones(1), atoms=atoms, rng=rng,
                     n_proj=4, dt=0.03, nsteps=0, A=np.zeros((1, 3)), hartree=False, xc=False,
                     r_c=1.6)
    return s


def _kron_hamiltonian(grid, kappa, V, projs):
    """Independent construction: Kronecker sums of 1-D circulants + diagonal +
    dense separable nonlocal matrix."""
    c, d = tdks.C2, tdks.D1
    mats2, mats1 = [], []
    for mu in range(3):
        N, h = grid.n[mu], grid.h[mu]
        D2 = np.zeros((N, N))
        D1 = np.zeros((N, N))
        for j in range(N):
            D2[j, j] += c[0] / h ** 2
            for m in range(1, 5):
                D2[j, (j + m) % N] += c[m] / h ** 2
                D2[j, (j - m) % N] += c[m] / h ** 2
                D1[j, (j + m) % N] += d[m - 1] / h
                D1[j, (j - m) % N] -= d[m - 1] / h
        mats2.append(D2)
        mats1.append(D1)
    I = [np.eye(grid.n[mu]) for mu in range(3)]

    def lift(Mx, My, Mz):
        return np.kron(Mz, np.kron(My, Mx))
    lap = lift(mats2[0], I[1], I[2]) + lift(I[0], mats2[1], I[2]) + lift(I[0], I[1], mats2[2])
    grads = [lift(mats1[0], I[1], I[2]), lift(I[0], mats1[1], I[2]), lift(I[0], I[1], mats1[2])]
    H = -0.5 * lap.astype(np.complex128)
    for mu in range(3):
        H += -1j * kappa[mu] * grads[mu]
    H += np.diag(0.5 * kappa @ kappa + V.ravel())
    npt = grid.shape[0] * grid.shape[1] * grid.shape[2]
    for pr in projs:
        B = np.zeros((npt, pr.beta.shape[0]), dtype=np.complex128)
        ph = np.exp(-1j * pr.x @ kappa)
        for p in range(pr.beta.shape[0]):
            B[pr.idx, p] = pr.beta[p] * ph
        H += grid.dV * B @ np.diag(pr.e_kb) @ B.conj().T
    return H


def test_dense_hamiltonian_two_constructions():
    s = _dense_system()
    grid = tdks.Grid(s.n, s.cell, s.boundary)
    kappa = s.kpts[0] + np.array([0.3, 0.1, -0.2]) / C
    projs = [tdks.Projector(p.idx, p.x, p.beta, p.e_kb) for p in s.projectors]
    npt = 512
    E = np.eye(npt, dtype=np.complex128).reshape((npt,) + grid.shape)
    Hcols = tdks.apply_h(E, kappa, s.v_loc, projs, grid).reshape(npt, npt).T
    Hk = _kron_hamiltonian(grid, kappa, s.v_loc, projs)
    assert np.max(np.abs(Hcols - Hk)) < 1e-12 * np.max(np.abs(Hk))
    assert np.max(np.abs(Hk - Hk.conj().T)) < 1e-12 * np.max(np.abs(Hk))


def test_dense_propagator_eigen_form():
    s = _dense_system()
    grid = tdks.Grid(s.n, s.cell, s.boundary)
    A0 = np.array([0.3, 0.1, -0.2])
    kappa = s.kpts[0] + A0 / C
    projs = [tdks.Projector(p.idx, p.x, p.beta, p.e_kb) for p in s.projectors]
    H = _kron_hamiltonian(grid, kappa, s.v_loc, projs)
    eps, U = np.linalg.eigh(H)
    nsteps = 25
    for dt in (s.dt, -s.dt, 0.11):
        osys = tdks.TDKS(s.n, s.cell, s.boundary, s.kpts, s.kw, s.psi0, dt, s.v_loc, s.projectors,
                         hartree=False, xc=False)
        osys.propagate(np.tile(A0, (nsteps + 1, 1)))
        for j in range(2):
            c0 = U.conj().T @ s.psi0[0, j].ravel()
            g = _p4(-1j * eps * dt) ** nsteps
            ref = (U @ (g * c0)).reshape(grid.shape)
            got = osys.psi[0, j]
            assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))
            # norm and energy closed forms
            norm = grid.dV * np.sum(np.abs(c0) ** 2 * np.abs(g) ** 2)
            assert abs(norm - np.real(grid.inner(got, got))) < 1e-12
            en = grid.dV * np.sum(np.abs(c0) ** 2 * eps * np.abs(g) ** 2)
            hg = (H @ got.ravel())
            assert abs(en - grid.dV * np.real(np.vdot(got.ravel(), hg))) < 1e-11 * max(1, abs(en))
    # truncation error of T4 against exp(-i H n dt), reported for the record
    dt = s.dt
    ex = sla.expm(-1j * H * nsteps * dt) @ s.psi0[0, 0].ravel()
    t4 = U @ (_p4(-1j * eps * dt) ** nsteps * (U.conj().T @ s.psi0[0, 0].ravel()))
    rel = np.linalg.norm(ex - t4) / np.linalg.norm(ex)
    xmax = np.max(np.abs(eps)) * dt
    assert rel < 25 * xmax ** 5 / 120 + 1e-12


def test_stability_bound_closed_form():
    """|P4(-ix)|^2 = 1 - x^6/72 + x^8/576: stable iff |x| <= 2 sqrt 2."""
    x = np.linspace(0, 3.2, 321)
    lhs = np.abs(_p4(-1j * x)) ** 2
    assert np.allclose(lhs, 1 - x ** 6 / 72 + x ** 8 / 576, rtol=0, atol=1e-12)
    assert np.all(lhs[x <= 2 * np.sqrt(2)] <= 1 + 1e-12)
    assert np.all(lhs[x > 2 * np.sqrt(2) + 1e-9] > 1)


# ---------------------------------------------------------------- Hermiticity
@pytest.mark.parametrize("boundary", ["periodic", "isolated"])
def test_hamiltonian_hermitian(boundary):
    rng = rng_for(909)
    if boundary == "periodic":
        s = tiny_periodic(kpts=[[0.2, -0.1, 0.3]], n_orb=2)
        kappa = s.kpts[0] + np.array([0.5, 0.0, -0.3]) / C
    else:
        from oracle_helpers import tiny_isolated
        s = tiny_isolated(n_orb=2)
        kappa = np.array([0.1, 0.2, -0.1])
    grid = tdks.Grid(s.n, s.cell, s.boundary)
    projs = [tdks.Projector(p.idx, p.x, p.beta, p.e_kb) for p in s.projectors]
    a = rng.normal(size=grid.shape) + 1j * rng.normal(size=grid.shape)
    b = rng.normal(size=grid.shape) + 1j * rng.normal(size=grid.shape)
    ha = tdks.apply_h(a[None], kappa, s.v_loc, projs, grid)[0]
    hb = tdks.apply_h(b[None], kappa, s.v_loc, projs, grid)[0]
    lhs = grid.inner(a, hb)
    rhs = np.conj(grid.inner(b, ha))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    for pr in projs:
        assert np.allclose(grid.dV * np.sum(pr.beta ** 2, axis=1), 1.0, atol=1e-13)
