"""Pins of the oracle's ground-state preparation (initial state, Sec. 2.1).

* Gram-Schmidt in orbital order equals the Q factor of a library QR whose R
  has a positive diagonal;
* the imaginary-time Taylor polynomial multiplies a plane wave by the closed
  form P4(-tau eps) with the finite-difference eigenvalue eps;
* one iteration equals the brute-force dense construction P4(-tau H) W
  followed by QR, with H built by Kronecker sums;
* without Hartree and xc the iteration converges to the lowest eigenvector of
  the dense H, with the energy 2 eps_0;
* with Hartree and LDA it converges to a self-consistent solution: the final
  orbital is an eigenvector of h[rho] built from its own density, and the
  energy settles from above.
"""
import numpy as np

from oracle import tdks
from oracle_helpers import tiny_periodic
from synth.systems import rng_for
from test_oracle_operators import _kron_hamiltonian, _symbols


def _p4(z):
    return 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24


def _qr_reference(W, grid):
    """Q of the library QR of the columns sqrt(h^3) w_j, phases fixed so that
    diag(R) > 0, mapped back to orbitals."""
    n = W.shape[0]
    M = np.sqrt(grid.dV) * W.reshape(n, -1).T
    Q, R = np.linalg.qr(M)
    ph = np.diag(R) / np.abs(np.diag(R))
    Q = Q * ph[None, :]
    return (Q.T / np.sqrt(grid.dV)).reshape(W.shape)


def test_gram_schmidt_equals_qr():
    grid = tdks.Grid((6, 5, 7), (4.0, 3.5, 5.0), "periodic")
    rng = rng_for(4401)
    W = rng.standard_normal((5,) + grid.shape) + 1j * rng.standard_normal((5,) + grid.shape)
    Q = tdks.gram_schmidt(W, grid)
    ref = _qr_reference(W, grid)
    assert np.max(np.abs(Q - ref)) < 1e-12 * np.max(np.abs(ref))
    S = np.array([[grid.inner(a, b) for b in Q] for a in Q])
    assert np.max(np.abs(S - np.eye(5))) < 1e-13
    # the first orbital is only normalised
    assert np.max(np.abs(Q[0] - W[0] / np.sqrt(np.real(grid.inner(W[0], W[0]))))) < 1e-14


def test_imaginary_time_polynomial_on_plane_waves():
    grid = tdks.Grid((8, 8, 8), (5.0, 5.0, 5.0), "periodic")
    x, y, z = grid.r_fields()
    kappa = np.array([0.2, -0.1, 0.05])
    V0 = 0.3
    hv = np.array(grid.h)
    for m in [(0, 0, 0), (1, 0, 0), (2, -3, 1), (4, 4, 4)]:
        G = np.array([2 * np.pi * m[i] / grid.cell[i] for i in range(3)])
        w = np.exp(1j * (G[0] * x + G[1] * y + G[2] * z))[None]
        K2, K1 = _symbols(G, hv)
        eps = 0.5 * np.sum(K2 / hv ** 2) + np.sum(kappa * K1 / hv) + 0.5 * kappa @ kappa + V0
        for tau in (0.01, 0.07):
            hop = lambda X: tdks.apply_h(X, kappa, V0 * np.ones(grid.shape), [], grid)
            out = tdks.imaginary_time_step(w, tau, hop)
            assert np.max(np.abs(out - _p4(-tau * eps) * w)) < 1e-12 * max(1.0, abs(_p4(-tau * eps)))


def test_one_iteration_brute_force():
    s = tiny_periodic(n=6, L=4.2, n_orb=3, kpts=np.array([[0.21, -0.13, 0.4]]), n_atoms=2,
                      hartree=True, xc=True, seed=4402, real=False)
    o = tdks.TDKS.from_system(s)
    grid = o.grid
    H = _kron_hamiltonian(grid, s.kpts[0], o.v_ks, o.projs)
    tau = 1.5 / np.max(np.abs(np.linalg.eigvalsh(H)))
    npt = H.shape[0]
    P = np.eye(npt, dtype=np.complex128)
    term = np.eye(npt, dtype=np.complex128)
    for m in range(1, 5):
        term = term @ (-tau * H) / m
        P = P + term
    W0 = s.psi0[0]
    W1 = (P @ W0.reshape(3, -1).T).T.reshape(W0.shape)
    ref = _qr_reference(W1, grid)
    E = o.ground_state(1, tau)
    assert np.max(np.abs(o.psi[0] - ref)) < 1e-11 * np.max(np.abs(ref))
    rho = 2.0 * np.sum(np.abs(ref) ** 2, axis=0)
    assert np.max(np.abs(o.rho0 - rho)) < 1e-11 * np.max(rho)
    assert np.isfinite(E[0])


def test_converges_to_lowest_eigenvector():
    s = tiny_periodic(n=8, L=4.0, n_orb=1, hartree=False, xc=False, seed=101)
    o = tdks.TDKS.from_system(s)
    H = _kron_hamiltonian(o.grid, s.kpts[0], o.v_ks, o.projs)
    ev, U = np.linalg.eigh(H)
    tau = 2.0 / ev[-1]
    E = o.ground_state(300, tau)
    assert abs(E[-1] - 2 * ev[0]) < 1e-11
    u0 = U[:, 0] / np.sqrt(o.grid.dV)
    ov = abs(o.grid.dV * np.vdot(u0, o.psi[0, 0].ravel()))
    assert abs(ov - 1.0) < 1e-10
    # variational: the energy never rises while converging
    assert np.all(np.diff(E) <= 1e-13)


def test_self_consistent_fixed_point():
    s = tiny_periodic(n=8, L=4.0, n_orb=1, hartree=True, xc=True, seed=101)
    o = tdks.TDKS.from_system(s)
    H0 = _kron_hamiltonian(o.grid, s.kpts[0], o.v_ks, o.projs)
    tau = 2.0 / np.max(np.linalg.eigvalsh(H0))
    E = o.ground_state(400, tau)
    # h built from the final density (Hartree + LDA of the final orbital)
    H = _kron_hamiltonian(o.grid, s.kpts[0], o.v_ks, o.projs)
    psi = o.psi[0, 0].ravel()
    hpsi = H @ psi
    lam = o.grid.dV * np.vdot(psi, hpsi)
    res = np.sqrt(o.grid.dV) * np.linalg.norm(hpsi - lam * psi)
    assert res < 1e-9
    assert abs(E[-1] - E[-2]) < 1e-12
    # the energy settles from above, monotonically for this step size
    assert np.all(np.diff(E) <= 1e-13)
