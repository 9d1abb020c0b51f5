"""Parity of the spectra and work entry points with the oracle's
post-processing (Sec. 3.1 Eq. distribution, Sec. 4.1 Eq. sigma_ft and W(t),
Sec. 4.2 DC subtraction), and of the excitation energy with the oracle's
energy difference.

Inputs are seeded synthetic series or series that the oracle itself produced;
sizes span several frequency blocks (256 per workgroup) and ragged sample
chunks."""
import numpy as np
import pytest

import synth
from gpu_helpers import announce
from oracle import spectra, tdks
from oracle_helpers import tiny_periodic

pytestmark = pytest.mark.gpu


def _series(n, seed):
    rng = np.random.default_rng(seed)
    t = np.arange(n) * 0.05
    return (2e-4 * np.exp(-0.004 * t) * np.cos(0.31 * t) + 6e-5 * np.sin(1.7 * t + 0.4) + 3e-6 * rng.standard_normal(n)
            + 4e-5)


@pytest.mark.parametrize("mask", [True, False])
@pytest.mark.parametrize("subtract_mean", [True, False])
@pytest.mark.parametrize("n_t,n_w", [(20001, 300), (37, 5), (2, 1)])
def test_conductivity_and_dielectric_match_oracle(mask, subtract_mean, n_t, n_w):
    from paper_1804_01404_amd import binding
    announce(f"conductivity n_t={n_t} n_w={n_w} mask={mask} mean={subtract_mean}")
    I = _series(n_t, 11)
    dt, A0 = 0.05, 0.137
    om = np.linspace(0.01, 2.5, n_w)
    sig, eps = binding.conductivity(I, dt, A0, om, mask=mask, subtract_mean=subtract_mean, dielectric=True)
    ref = spectra.conductivity(I, dt, A0, om, subtract_mean=subtract_mean, use_mask=mask)
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(sig - ref)) <= 1e-12 * scale
    eref = spectra.dielectric(ref, om)
    assert np.max(np.abs(eps - eref)) <= 1e-12 * np.max(np.abs(eref))
    # bitwise repeatable
    again = binding.conductivity(I, dt, A0, om, mask=mask, subtract_mean=subtract_mean)
    assert np.array_equal(again, sig)


def test_conductivity_of_an_oracle_kick_run():
    """sigma of the current that the oracle computes for a kicked cell."""
    from paper_1804_01404_amd import binding
    announce("conductivity of an oracle kick run")
    C = spectra.C_LIGHT
    A0 = np.array([C * 1e-3, 0, 0])
    n, dt = 120, 0.05
    s = tiny_periodic(nsteps=n, dt=dt, A=synth.kick_table(n, A0), n_orb=4)
    o = tdks.TDKS.from_system(s)
    I0 = o.current(A0)
    J = o.propagate(s.A)
    I = np.concatenate([I0[None], J])[:, 0]
    om = np.linspace(0.0, np.pi / dt, 513)
    for sub in (False, True):
        sig = binding.conductivity(I, dt, A0[0], om, subtract_mean=sub)
        ref = spectra.conductivity(I, dt, A0[0], om, subtract_mean=sub)
        assert np.max(np.abs(sig - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("n_t,n_E", [(5001, 700), (40, 3)])
def test_oscillator_strength_matches_oracle(n_t, n_E):
    from paper_1804_01404_amd import binding
    announce(f"oscillator strength n_t={n_t} n_E={n_E}")
    dt, F0 = 0.02, 1e-3
    t = np.arange(n_t) * dt
    rng = np.random.default_rng(5)
    d = F0 * (0.8 / 0.45 * np.sin(0.45 * t) + 0.3 / 1.2 * np.sin(1.2 * t)) + 1e-9 * rng.standard_normal(n_t)
    E = np.linspace(0.0, 4.0, n_E)
    got = binding.oscillator_strength(d, dt, F0, E)
    ref = spectra.oscillator_strength(d, dt, F0, E)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("n_t", [2, 1000, 5003])
def test_work_matches_oracle(n_t):
    from paper_1804_01404_amd import binding
    announce(f"work n_t={n_t}")
    dt = 0.02
    A = synth.cos2_pulse_table(n_t - 1, dt, 0.02, 0.6, dt * (n_t - 1), 0.2, [1.0, 0.4, -0.3])
    rng = np.random.default_rng(3)
    I = 1e-3 * rng.standard_normal((n_t, 3)) + 1e-4
    W = binding.work(I, A, dt, 1080.05)
    ref = spectra.work(I, A, dt, 1080.05)
    assert W[0] == 0.0
    assert np.max(np.abs(W - ref)) <= 1e-12 * max(np.max(np.abs(ref)), 1e-300)


def test_excitation_energy_matches_oracle_and_work():
    """E(t) - E(0) of a pulsed cell against the oracle's energy difference
    (complex128), and against the work of the field computed by the library
    from the recorded current (a frozen Hamiltonian, so the energy-work
    theorem holds to the Taylor error)."""
    from paper_1804_01404_amd import binding
    n, dt = 60, 0.02
    A = synth.cos2_pulse_table(n, dt, 0.05, 0.5, n * dt, 0.1, [1, 0.3, -0.2])
    s = tiny_periodic(kpts=[[0.1, 0.2, -0.1], [-0.3, 0.0, 0.2]], n_orb=3, dt=dt, nsteps=n, A=A,
                      hartree=False, xc=False, n=8, L=5.2)
    announce("excitation energy, 8^3 cell, 2 k-points, pulse")
    with binding.TDDFT(s, precision="c128") as t:
        t.set_potential()
        t.set_reference()
        I0 = t.density_current()[1]
        J = t.propagate(A)
        E_ex = t.excitation_energy()
    o = tdks.TDKS.from_system(s)
    E0 = o.energy(A[0])
    o.propagate(A)
    ref = o.energy() - E0
    assert abs(E_ex - ref) <= 1e-11 * abs(E0)
    W = binding.work(np.concatenate([I0[None], J]), A, dt, float(np.prod(s.cell)))
    assert abs(W[-1] - E_ex) <= 1e-3 * abs(E_ex)


def test_excitation_energy_refused_without_functional():
    from paper_1804_01404_amd import binding
    s = tiny_periodic(n=10, nsteps=2)
    s.xc = "tb09"
    with binding.TDDFT(s, precision="c128") as t:
        t.set_potential()
        t.set_reference()
        with pytest.raises(binding.TDDFTError) as e:
            t.excitation_energy()
        assert e.value.status == binding.ESTATE
