"""Pins of the oracle's Becke-Johnson / Tran-Blaha exchange potential (Sec. 4.1).

* Becke-Roussel potential of the hydrogen 1s density: the model hole is exact
  for a one-electron density, so the potential equals the exact exchange
  potential, minus the Hartree potential of the density itself,
  -(1/r)(1 - (1 + r) e^(-2r)); r = 1 (where lap rho = 0, so x = 2) included;
* Q equals the curvature of the exact spherically averaged exchange hole of a
  set of orbitals, -h''(0)/2 with h(s) = -|sum_i phi_i(r) phi_i(r + s)|^2 / rho(r)
  (which fixes gamma = 1, the T = sum |grad phi|^2 convention and the 1/6),
  measured by finite differences of the hole itself;
* exchange scaling: rho_l(r) = l^3 rho(l r) gives v_l(r) = l v(l r);
* the spin split and the kinetic term: two electrons in the hydrogen 1s
  orbital give 2/3 of the exact potential at c = 2/3 and sqrt(5/12)/pi more
  at c = 1; for the uniform gas the kinetic term is -v_x(LDA)/2;
* the root of the Becke-Roussel equation for small |y| on the lower branch
  approaches -2y;
* tau of plane waves: sum (K1(theta)/h + kappa)^2 |w|^2 per orbital (K1 the
  symbol of the 9-point first derivative), with A entering through kappa in
  the velocity gauge only;
* g of rho0 (1 + a cos Gx): (K1/h)(1/pi) ln((1 + a)/(1 - a)) up to the
  quadrature error of the grid sum; c = alpha + beta sqrt(g);
* through the whole propagation with TB09: time reversal (Gamma, real
  inputs) and the static-A = k-shift identity still hold.
"""
import numpy as np
import pytest

from oracle import mgga, tdks
from oracle_helpers import tiny_periodic

C = 137.035999084
D1 = (4 / 5, -1 / 5, 4 / 105, -1 / 280)


def _k1(theta):
    return 2 * sum(D1[m - 1] * np.sin(m * theta) for m in range(1, 5))


def test_becke_roussel_is_exact_for_hydrogen():
    r = np.array([0.05, 0.3, 0.7, 1.0, 1.6, 3.0, 6.0])
    rho = np.exp(-2 * r) / np.pi            # one electron, one spin channel
    grad_sq = 4 * rho ** 2                  # |d rho / dr|^2
    lap = 4 * rho - 4 * rho / r             # rho'' + (2/r) rho'
    T = rho                                 # |grad psi|^2 with psi = e^(-r)/sqrt(pi)
    v = mgga.br89_potential(rho, grad_sq, lap, T)
    exact = -(1 - (1 + r) * np.exp(-2 * r)) / r
    assert np.max(np.abs(v - exact) / np.abs(exact)) < 1e-12


def test_spin_split_and_kinetic_term():
    """Two electrons in the hydrogen 1s orbital: each spin channel is the
    hydrogen density, so c = 2/3 leaves 2/3 of the exact hydrogen exchange
    potential and c = 1 adds sqrt(5/12)/pi; the uniform gas with its
    kinetic energy density (3/10)(3 pi^2)^(2/3) rho^(5/3) has the kinetic
    term -v_x(LDA)/2 = (3 rho/pi)^(1/3) / 2."""
    r = np.array([0.2, 0.8, 2.5])
    rh = np.exp(-2 * r) / np.pi
    rho, grad_sq, lap, tau = 2 * rh, 16 * rh ** 2, 2 * (4 * rh - 4 * rh / r), rh
    exact = -(1 - (1 + r) * np.exp(-2 * r)) / r
    assert np.max(np.abs(mgga.mbj_pointwise(rho, grad_sq, lap, tau, 2 / 3) - 2 / 3 * exact)) < 1e-12
    assert np.max(np.abs(mgga.mbj_pointwise(rho, grad_sq, lap, tau, 1.0) - exact - np.sqrt(5 / 12) / np.pi)) < 1e-12
    rho = np.array([1e-3, 0.03, 0.7])
    tau = 0.3 * (3 * np.pi ** 2) ** (2 / 3) * rho ** (5 / 3)
    z = np.zeros(3)
    K = mgga.mbj_pointwise(rho, z, z, tau, 1.0) - 1.5 * mgga.mbj_pointwise(rho, z, z, tau, 2 / 3)
    assert np.max(np.abs(K - 0.5 * (3 * rho / np.pi) ** (1 / 3)) / K) < 1e-13


def _gaussians(seed):
    rng = np.random.default_rng(seed)
    cen = rng.normal(size=(3, 3)) * 0.7
    alp = rng.uniform(0.5, 1.5, 3)
    amp = rng.normal(size=3)
    return cen, alp, amp


def _phi(P, cen, alp, amp):
    return np.stack([a * np.exp(-al * np.sum((P - c) ** 2, -1)) for c, al, a in zip(cen, alp, amp)])


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_q_is_the_exact_exchange_hole_curvature(seed):
    cen, alp, amp = _gaussians(seed)
    r = np.array([0.3, -0.2, 0.4])
    ph = _phi(r, cen, alp, amp)
    rho = np.sum(ph ** 2)
    # analytic derivatives of the Gaussians
    grads = np.stack([-2 * al * (r - c) * p for c, al, p in zip(cen, alp, ph)])
    lapl = np.array([(4 * al ** 2 * np.sum((r - c) ** 2) - 6 * al) * p for c, al, p in zip(cen, alp, ph)])
    grad_rho = 2 * np.sum(ph[:, None] * grads, 0)
    lap_rho = 2 * np.sum(grads ** 2) + 2 * np.sum(ph * lapl)
    T = np.sum(grads ** 2)
    Q = mgga.br89_q(rho, np.sum(grad_rho ** 2), lap_rho, T)

    # the hole h(r, r') = -(sum_i phi_i(r) phi_i(r'))^2 / rho(r); its spherical
    # average around r is h0 + (1/6) lap' h s^2 + ..., by central differences in r'
    def hole(rp):
        return -np.sum(ph * _phi(rp, cen, alp, amp)) ** 2 / rho

    def lap_h(e):
        return sum((hole(r + e * u) - 2 * hole(r) + hole(r - e * u)) / e ** 2 for u in np.eye(3))

    curvature = (4 * lap_h(1e-3) - lap_h(2e-3)) / 3 / 6.0     # Richardson: O(e^4)
    assert abs(curvature + Q) < 1e-7 * abs(Q)
    # gamma = 0.8 (the original energy fit) is visibly different
    assert abs(curvature + mgga.br89_q(rho, np.sum(grad_rho ** 2), lap_rho, T, gamma=0.8)) > 1e-3 * abs(Q)


def test_exchange_scaling():
    rng = np.random.default_rng(7)
    rho = rng.uniform(1e-3, 0.5, 200)
    grad_sq = rng.uniform(0, 2, 200) * rho ** (8 / 3)
    lap = rng.normal(size=200) * rho ** (5 / 3) * 3
    T = grad_sq / (4 * rho) + rng.uniform(0, 2, 200) * rho ** (5 / 3)
    v = mgga.br89_potential(rho, grad_sq, lap, T)
    for lam in (0.37, 1.7, 5.0):
        vl = mgga.br89_potential(lam ** 3 * rho, lam ** 8 * grad_sq, lam ** 5 * lap, lam ** 5 * T)
        assert np.max(np.abs(vl - lam * v) / np.abs(lam * v)) < 1e-12


def test_becke_roussel_root_limits():
    y = np.array([-1e-9, -1e-6])
    x = mgga.br89_x(y)
    assert np.all(np.abs(x / (-2 * y) - 1) < 10 * np.abs(y))
    assert np.all(mgga.br89_x(np.array([np.inf, -np.inf])) == 2.0)
    # both branches are monotone: larger y, smaller root on each side
    yn = -np.logspace(-3, 3, 20)
    yp = np.logspace(-3, 3, 20)
    assert np.all(np.diff(mgga.br89_x(yn)) > 0) and np.all(np.diff(mgga.br89_x(yp)) < 0)
    assert np.all(mgga.br89_x(yn) < 2) and np.all(mgga.br89_x(yp) > 2)


@pytest.mark.parametrize("gauge", ["velocity", "length"])
def test_tau_of_plane_waves(gauge):
    n, L = (8, 10, 12), (5.0, 6.0, 7.0)
    grid = tdks.Grid(n, L, "periodic")
    x, y, z = grid.r_fields()
    kpts = np.array([[0.1, -0.2, 0.05], [-0.3, 0.0, 0.2]])
    kw = np.array([0.25, 0.75])
    A = np.array([3.0, -2.0, 1.0])
    ms = [[(1, 0, 2), (0, -1, 1)], [(2, 1, 0), (-1, 0, -1)]]
    psi = np.zeros((2, 2) + grid.shape, dtype=np.complex128)
    expect = 0.0
    for ik in range(2):
        kap = kpts[ik] + (A / C if gauge == "velocity" else 0.0)
        for io, m in enumerate(ms[ik]):
            G = 2 * np.pi * np.array(m) / np.array(L)
            psi[ik, io] = np.exp(1j * (G[0] * x + G[1] * y + G[2] * z)) / np.sqrt(grid.volume)
            th = G * np.array(grid.h)
            expect += kw[ik] * np.sum((_k1(th) / np.array(grid.h) + kap) ** 2) / grid.volume
    tau = mgga.kinetic_energy_density(psi, kpts, kw, A, grid, gauge)
    assert np.max(np.abs(tau - expect)) < 1e-13 * expect


def test_tb09_g_and_c_closed_form():
    n, L = (96, 8, 8), (20.0, 4.0, 4.0)
    grid = tdks.Grid(n, L, "periodic")
    x, _, _ = grid.r_fields()
    G = 2 * np.pi / L[0]
    for a in (0.2, 0.6):
        rho = 0.03 * (1 + a * np.cos(G * x))
        g = mgga.tb09_g(rho, grid)
        expect = _k1(G * grid.h[0]) / grid.h[0] / np.pi * np.log((1 + a) / (1 - a))
        assert abs(g - expect) < 2e-3 * expect
        assert abs(mgga.tb09_c(rho, grid) - (-0.012 + 1.023 * np.sqrt(g))) < 1e-15
    assert mgga.tb09_g(np.full(grid.shape, 0.03), grid) == 0.0


def _run(s, xc, A=None, dt=None, psi0=None):
    o = tdks.TDKS(s.n, s.cell, s.boundary, s.kpts, s.kw, s.psi0 if psi0 is None else psi0,
                  s.dt if dt is None else dt, s.v_loc, s.projectors, hartree=s.hartree, xc=xc,
                  gauge=s.gauge)
    J = o.propagate(s.A if A is None else A)
    return o, J


@pytest.mark.parametrize("xc", ["tb09", "bj"])
def test_time_reversal_with_mgga(xc):
    s = tiny_periodic(nsteps=4)
    fwd, Jf = _run(s, xc)
    bwd, Jb = _run(s, xc, dt=-s.dt)
    assert np.max(np.abs(bwd.psi - np.conj(fwd.psi))) < 1e-13
    assert np.max(np.abs(Jb + Jf)) < 1e-15
    assert xc != "tb09" or 0.5 < fwd.mgga_c < 2.5
    # the potential differs from the LDA one
    lda, _ = _run(s, True)
    assert np.max(np.abs(fwd.v_xc - lda.v_xc)) > 1e-2


def test_static_A_is_a_k_shift_with_tb09():
    k = np.array([[0.05, 0.1, -0.2]])
    A0 = np.array([2.0, -1.0, 0.7])
    n = 3
    sa = tiny_periodic(kpts=k, nsteps=n, A=np.tile(A0, (n + 1, 1)))
    sb = tiny_periodic(kpts=k + A0 / C, nsteps=n, A=np.zeros((n + 1, 3)))
    # the constructor sees A = 0: start both from the same potential by a first
    # step under A0 in both runs' own gauge
    oa = tdks.TDKS(sa.n, sa.cell, sa.boundary, sa.kpts, sa.kw, sa.psi0, sa.dt, sa.v_loc, sa.projectors,
                   xc="tb09")
    oa.A_now = A0
    oa._update_potential(oa.psi, A0)
    ob = tdks.TDKS(sb.n, sb.cell, sb.boundary, sb.kpts, sb.kw, sa.psi0, sb.dt, sb.v_loc, sb.projectors,
                   xc="tb09")
    assert np.max(np.abs(oa.v_ks - ob.v_ks)) < 1e-13
    Ja = oa.propagate(sa.A)
    Jb = ob.propagate(sb.A)
    assert np.max(np.abs(oa.psi - ob.psi)) < 1e-13
    assert np.max(np.abs(Ja - Jb)) < 1e-15
