"""Pins of the oracle's time stepping and observables.

* time reversal (Gamma, real inputs): the run with -dt is the complex
  conjugate of the run with +dt, through the self-consistent loop;
* k -> -k with A -> -A and t -> -t conjugates the orbitals and flips the
  current (antiunitary time reversal at a general k-point);
* a static A is the same as the shift k -> k + A/c (velocity gauge);
* f-sum: the diamagnetic jump of the current after a kick is -N_e (A0/c)/Omega
  and the sigma(omega) integral returns sigma(0+) = n_e; isolated: the dipole
  velocity right after a kick is N_e F0;
* the current is -(1/Omega) dE/d(A/c) at fixed orbitals (nonlocal part included);
* energy-work theorem E(t) - E(0) = Omega int I . E dt: to fifth order in dt
  for a frozen Hamiltonian, first order with the potential frozen at rho(t_n);
* density bookkeeping and the linear regime.
"""
import numpy as np
import pytest

import synth
from oracle import spectra, tdks
from oracle_helpers import tiny_isolated, tiny_periodic

C = 137.035999084


def _run(s, A=None, dt=None, psi0=None):
    o = tdks.TDKS(s.n, s.cell, s.boundary, s.kpts, s.kw, s.psi0 if psi0 is None else psi0,
                  s.dt if dt is None else dt, s.v_loc, s.projectors, hartree=s.hartree, xc=s.xc,
                  gauge=s.gauge)
    J = o.propagate(s.A if A is None else A)
    return o, J


@pytest.mark.parametrize("iso", [False, True])
def test_time_reversal(iso):
    s = tiny_isolated(nsteps=5) if iso else tiny_periodic(nsteps=5)
    assert np.all(s.psi0.imag == 0)
    fwd, Jf = _run(s)
    bwd, Jb = _run(s, dt=-s.dt)
    assert np.max(np.abs(bwd.psi - np.conj(fwd.psi))) < 1e-13
    assert np.max(np.abs(bwd.rho - fwd.rho)) < 1e-13
    assert np.max(np.abs(Jb + Jf)) < 1e-15


def test_k_minus_k_conjugation():
    k = np.array([[0.21, -0.13, 0.08]])
    n = 5
    A = synth.cos2_pulse_table(n, 0.02, 0.02, 0.4, 0.1, 0.0, [1, 1, 0])
    A = A + np.array([0.3, -0.2, 0.5])
    sa = tiny_periodic(kpts=k, nsteps=n, A=A)
    sb = tiny_periodic(kpts=-k, nsteps=n, A=-A)
    oa, Ja = _run(sa, dt=-sa.dt)
    ob, Jb = _run(sb, psi0=np.conj(sa.psi0))
    assert np.max(np.abs(ob.psi - np.conj(oa.psi))) < 1e-13
    assert np.max(np.abs(Jb + Ja)) < 1e-14 * max(1.0, np.max(np.abs(Ja)) * 1e3)


def test_static_A_is_a_k_shift():
    k = np.array([[0.05, 0.1, -0.2]])
    A0 = np.array([2.0, -1.0, 0.7])
    n = 4
    sa = tiny_periodic(kpts=k, nsteps=n, A=np.tile(A0, (n + 1, 1)))
    sb = tiny_periodic(kpts=k + A0 / C, nsteps=n, A=np.zeros((n + 1, 3)))
    oa, Ja = _run(sa)
    ob, Jb = _run(sb, psi0=sa.psi0)
    assert np.max(np.abs(oa.psi - ob.psi)) < 1e-13
    assert np.max(np.abs(Ja - Jb)) < 1e-15


def test_diamagnetic_jump_and_spectral_fsum():
    A0 = np.array([C * 1e-3, 0, 0])
    n, dt = 60, 0.05
    s = tiny_periodic(nsteps=n, dt=dt, A=synth.kick_table(n, A0), n_proj=0, n_orb=4)
    o = tdks.TDKS.from_system(s)
    I_before = o.current(np.zeros(3))
    I_after = o.current(A0)
    N_e = 2 * s.n_orb
    Omega = o.grid.volume
    assert abs(I_before[0]) < 1e-15                      # real Gamma orbitals carry no current
    assert abs((I_after - I_before)[0] + N_e * 1e-3 / Omega) < 1e-15
    J = o.propagate(s.A)
    I = np.concatenate([I_after[None], J])[:, 0]
    # (2/pi) int_0^{pi/dt} Re sigma(omega) d omega = sigma(t = 0+) = n_e (no DC subtraction)
    om = np.linspace(0, np.pi / dt, 20001)
    sig = spectra.conductivity(I, dt, A0[0], om)
    integ = np.sum((sig.real[1:] + sig.real[:-1]) * 0.5 * np.diff(om))
    assert abs(2 / np.pi * integ - N_e / Omega) < 1e-6 * N_e / Omega


def test_isolated_kick_dipole_velocity():
    F0 = 1e-3
    s = tiny_isolated(n_proj=0, nsteps=1, dt=0.002, gauge="length")
    vels = []
    for F in (F0, 0.0):
        d = []
        for dt in (s.dt, -s.dt):
            o = tdks.TDKS(s.n, s.cell, s.boundary, s.kpts, s.kw, s.psi0, dt, s.v_loc, [],
                          hartree=True, xc=True, gauge="length")
            x, y, z = o.grid.r_fields()
            o.psi = o.psi * np.exp(-1j * F * z)[None, None]
            o.propagate(s.A)
            d.append(o.dipole())
        vels.append((d[0] - d[1]) / (2 * s.dt))
    vel = vels[0] - vels[1]           # the kick's share of the dipole velocity
    N_e = 2 * s.n_orb
    # continuum value N_e F0; the 9-point momentum differs at the grid's top modes
    assert abs(vel[2] - N_e * F0) < 1e-2 * N_e * F0
    assert abs(vel[0]) < 1e-3 * N_e * F0 and abs(vel[1]) < 1e-3 * N_e * F0


def test_current_is_energy_derivative():
    s = tiny_periodic(kpts=[[0.2, -0.15, 0.3], [-0.1, 0.05, 0.2]], nsteps=0, n_orb=3)
    o = tdks.TDKS.from_system(s)
    A = np.array([1.3, -0.4, 2.2])
    I = o.current(A)
    dA = 1e-4 * C            # step in A/c of 1e-4
    grad = np.zeros(3)
    for mu in range(3):
        e = np.zeros(3)
        e[mu] = dA
        f = [o.energy(A + m * e) for m in (-2, -1, 1, 2)]
        grad[mu] = (f[0] - 8 * f[1] + 8 * f[2] - f[3]) / (12 * dA / C)
    assert np.max(np.abs(I + grad / o.grid.volume)) < 1e-7 * np.max(np.abs(I))


def _energy_work_gap(dt, hx, pc=False):
    T = 2.0
    n = int(round(T / dt))
    A = synth.cos2_pulse_table(n, dt, 0.05, 0.5, T, 0.1, [1, 0.3, -0.2])
    s = tiny_periodic(kpts=[[0.1, 0.2, -0.1], [-0.3, 0.0, 0.2]], n_orb=3, dt=dt, nsteps=n, A=A,
                      hartree=hx, xc=hx, n=8, L=5.2)
    o = tdks.TDKS.from_system(s, predictor_corrector=pc)
    E0 = o.energy(A[0])
    Is = [o.current(A[0])]
    for m in range(n):
        o.step(A[m], A[m + 1])
        Is.append(o.current())
    W = spectra.work(np.array(Is), A, dt, o.grid.volume)
    return o.energy() - E0, W[-1]


def test_energy_work_theorem_linear():
    d1, w1 = _energy_work_gap(0.04, False)
    d2, w2 = _energy_work_gap(0.02, False)
    assert abs(d2 - w2) < 1e-3 * abs(w2)
    assert abs(d1 - w1) / abs(d2 - w2) > 16          # at least 4th order
    assert d2 * w2 > 0                               # energy gained = work done (sign)


def test_energy_work_theorem_selfconsistent_first_order():
    d1, w1 = _energy_work_gap(0.04, True)
    d2, w2 = _energy_work_gap(0.02, True)
    ratio = abs(d1 - w1) / abs(d2 - w2)
    assert 1.6 < ratio < 2.5                          # potential frozen over the step
    assert abs(w1 - w2) < 1e-2 * abs(w2)


def test_energy_work_theorem_predictor_corrector_second_order():
    """With the potential taken at the step midpoint (predictor-corrector),
    the self-consistent energy-work gap falls with the square of dt."""
    d1, w1 = _energy_work_gap(0.04, True, pc=True)
    d2, w2 = _energy_work_gap(0.02, True, pc=True)
    ratio = abs(d1 - w1) / abs(d2 - w2)
    assert ratio > 3.3
    e1, v1 = _energy_work_gap(0.04, True)
    assert abs(d1 - w1) < 0.5 * abs(e1 - v1)     # better than the frozen potential


def test_predictor_corrector_is_exact_without_self_consistency():
    """Without Hartree and xc the potential does not depend on rho, so the
    corrector repeats the plain step exactly."""
    s = tiny_periodic(kpts=[[0.1, 0.0, 0.2]], n_orb=2, nsteps=4, dt=0.03, hartree=False, xc=False,
                      A=synth.kick_table(4, [0.4, 0, 0]), n=8, L=5.2)
    a = tdks.TDKS.from_system(s)
    b = tdks.TDKS.from_system(s, predictor_corrector=True)
    Ja = a.propagate(s.A)
    Jb = b.propagate(s.A)
    assert np.max(np.abs(a.psi - b.psi)) < 1e-14
    assert np.max(np.abs(Ja - Jb)) < 1e-15


def test_density_bookkeeping():
    s = tiny_periodic(kpts=[[0.1, 0, 0], [0, 0.2, 0], [0, 0, 0.3]], nsteps=3, dt=0.03,
                      A=synth.kick_table(3, [0.5, 0, 0]))
    o = tdks.TDKS.from_system(s)
    assert abs(o.grid.dV * o.rho.sum() - 2 * s.n_orb) < 1e-12
    o.propagate(s.A)
    fn = 2 * np.einsum("k,kn->", s.kw, o.norms())
    assert abs(o.grid.dV * o.rho.sum() - fn) < 1e-12
    assert abs(fn - 2 * s.n_orb) < 1e-6


def test_linear_regime_superposition():
    n, dt = 20, 0.05
    A1 = synth.cos2_pulse_table(n, dt, 1.0, 0.6, n * dt, 0.0, [1, 0, 0])
    A2 = synth.cos2_pulse_table(n, dt, 1.0, 0.9, n * dt, 0.3, [0, 1, 1])
    res = []
    for lam in (1e-3, 5e-4):
        J = {}
        for key, A in (("0", 0 * A1), ("1", lam * A1), ("2", lam * A2), ("12", lam * (A1 + A2))):
            s = tiny_periodic(nsteps=n, dt=dt, A=A, n_orb=3, n=8, L=5.2)
            J[key] = _run(s)[1]
        res.append(np.max(np.abs(J["12"] - J["1"] - J["2"] + J["0"])))
        lin = np.max(np.abs(J["1"] - J["0"]))
        assert res[-1] < 1e-2 * lin
    assert 3.0 < res[0] / res[1] < 5.0               # residual is quadratic in the field


def test_excited_electrons_pins():
    """Zero against itself; invariant under a unitary mixing of the occupied
    orbitals of one k-point; one orbital rotated fully out of the reference
    space counts exactly 2 w_k / Omega; quadratic in a weak kick."""
    s = tiny_periodic(kpts=[[0.1, 0.0, 0.2], [0.0, -0.2, 0.1]], n_orb=3, nsteps=30, dt=0.03, n=8, L=5.2,
                      real=False)
    g = tdks.Grid(s.n, s.cell, s.boundary)
    ref = s.psi0
    assert abs(tdks.excited_electrons(ref, ref, s.kw, g)) < 1e-13
    rng = np.random.default_rng(7)
    M = rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3))
    U, _ = np.linalg.qr(M)
    mixed = ref.copy()
    mixed[1] = np.einsum("mn,nzyx->mzyx", U, ref[1])
    assert abs(tdks.excited_electrons(ref, mixed, s.kw, g)) < 1e-13
    # replace orbital 2 of k-point 0 by a normalised vector orthogonal to all references
    v = rng.normal(size=g.shape) + 1j * rng.normal(size=g.shape)
    for m in range(3):
        v = v - g.inner(ref[0, m], v) * ref[0, m]
    v = v / np.sqrt(np.real(g.inner(v, v)))
    out = ref.copy()
    out[0, 2] = v
    assert abs(tdks.excited_electrons(ref, out, s.kw, g) - 2 * s.kw[0] / g.volume) < 1e-13
    # weak kicks from exact eigenstates (no Hartree or xc, dense H per
    # k-point): nothing is excited without the kick, and n_ex grows as the
    # square of the kick
    from test_oracle_operators import _kron_hamiltonian
    s0 = tiny_periodic(kpts=[[0.1, 0.0, 0.2], [0.0, -0.2, 0.1]], n_orb=3, nsteps=30, dt=0.03, n=8, L=5.2,
                       hartree=False, xc=False)
    g0 = tdks.Grid(s0.n, s0.cell, s0.boundary)
    projs = [tdks.Projector(p.idx, p.x, p.beta, p.e_kb) for p in s0.projectors]
    eig = np.empty_like(s0.psi0)
    for ik, k in enumerate(s0.kpts):
        _, U = np.linalg.eigh(_kron_hamiltonian(g0, k, s0.v_loc, projs))
        for m in range(3):
            eig[ik, m] = (U[:, m] / np.sqrt(g0.dV)).reshape(g0.shape)
    vals = []
    for a0 in (0.0, 0.05, 0.1):
        o = tdks.TDKS.from_system(s0, psi0=eig)
        o.propagate(synth.kick_table(30, [a0, 0, 0]))
        vals.append(tdks.excited_electrons(eig, o.psi, s0.kw, o.grid))
    # without the kick only the Taylor step's tiny norm loss shows
    assert abs(vals[0]) < 1e-3 * vals[1]
    assert abs((vals[2] - vals[0]) / (vals[1] - vals[0]) - 4.0) < 0.01
