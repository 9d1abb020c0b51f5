"""Pins of the oracle's spectral post-processing and of the field energy.

* mask f(x) = 1 - 3x^2 + 2x^3 (Sec. 3.1): f(0) = 1, f(1) = 0, zero slope at
  both ends, f(1/2) = 1/2 and f(x) + f(1 - x) = 1;
* conductivity (Sec. 4.1, Eq. sigma_ft): a Drude current I(t) =
  -(n_e A0 / c) exp(-g t) after a kick A0 has sigma(w) = n_e / (g - i w) in the
  continuum; the trapezoid sum converges to it at second order in dt. This
  fixes the prefactor -c/A0, the sign of the exponent and the weights;
* DC subtraction (Sec. 4.2: I -> I - mean(I), so that a spurious constant
  current does not enter sigma): a constant series gives sigma = 0 at every w,
  adding a constant changes nothing, and a series whose sample mean is zero
  is left as it is;
* dielectric function (Sec. 4.1): eps = 1 + 4 pi i sigma / w turns the Drude
  sigma into the plasma form 1 - w_p^2 / (w (w + i g)), w_p^2 = 4 pi n_e;
* oscillator strength (Sec. 3.1, Eq. distribution): for the dipole of a kicked
  oscillator d(t) = F0 (f / w0) sin(w0 t) the distribution integrates to f
  (the sum rule int df/dE dE = d'(0) / F0 holds for the masked transform of any
  run length, since the mask is 1 at t = 0 and 0 with zero slope at T), and
  peaks at w0;
* field energy (Sec. 5, the energy monitor of the coupled run): closed forms
  for a uniform E and a uniform B; at Courant number 1 a pulse crossing a
  vacuum grid keeps exactly the energy of its profile, and the Mur end takes
  all of it out when the pulse leaves.
"""
import math

import numpy as np
import pytest

from oracle import maxwell, spectra

C = spectra.C_LIGHT


def test_mask_values_and_slopes():
    x = np.linspace(0.0, 1.0, 101)
    f = spectra.mask(x)
    assert f[0] == 1.0 and f[-1] == 0.0
    assert spectra.mask(0.5) == 0.5
    assert np.max(np.abs(f + f[::-1] - 1.0)) < 1e-15
    h = 1e-6
    for x0 in (0.0, 1.0):
        slope = (spectra.mask(x0 + h) - spectra.mask(x0 - h)) / (2 * h)
        assert abs(slope) < 1e-9
    # monotone decreasing in between
    assert np.all(np.diff(f) < 0)


def _drude(dt, T=600.0, n_e=0.03, g=0.05, A0=0.5):
    t = np.arange(int(round(T / dt)) + 1) * dt
    return t, -(n_e * A0 / C) * np.exp(-g * t), n_e, g, A0


def test_conductivity_drude_closed_form_second_order():
    om = np.array([0.1, 0.3, 1.0, 2.0])
    errs = []
    for dt in (0.02, 0.01):
        _, I, n_e, g, A0 = _drude(dt)
        sig = spectra.conductivity(I, dt, A0, om, use_mask=False)
        ref = n_e / (g - 1j * om)
        errs.append(np.max(np.abs(sig - ref) / np.abs(ref)))
    assert errs[1] < 5e-5
    assert 3.5 < errs[0] / errs[1] < 4.5           # trapezoid: second order


def test_dielectric_drude_plasma_form():
    om = np.array([0.1, 0.3, 1.0, 2.0])
    _, I, n_e, g, A0 = _drude(0.01)
    eps = spectra.dielectric(spectra.conductivity(I, 0.01, A0, om, use_mask=False), om)
    wp2 = 4 * np.pi * n_e
    ref = 1.0 - wp2 / (om * (om + 1j * g))
    assert np.max(np.abs(eps - ref) / np.abs(ref)) < 2e-5
    # a lossy medium: Im eps > 0 for the e^{+i w t} convention
    assert np.all(eps.imag > 0)


@pytest.mark.parametrize("use_mask", [True, False])
def test_conductivity_dc_subtraction(use_mask):
    dt, n = 0.05, 4000
    t = np.arange(n) * dt
    om = np.linspace(0.0, 3.0, 7)
    const = np.full(n, 2.5e-4)
    s0 = spectra.conductivity(const, dt, 0.1, om, subtract_mean=True, use_mask=use_mask)
    assert np.max(np.abs(s0)) < 1e-12 * np.max(np.abs(
        spectra.conductivity(const, dt, 0.1, om, use_mask=use_mask)))
    rng = np.random.default_rng(7)
    I = 1e-4 * np.cos(0.7 * t) * np.exp(-0.01 * t) + 1e-5 * rng.standard_normal(n)
    a = spectra.conductivity(I, dt, 0.1, om, subtract_mean=True, use_mask=use_mask)
    b = spectra.conductivity(I + 3e-3, dt, 0.1, om, subtract_mean=True, use_mask=use_mask)
    assert np.max(np.abs(a - b)) < 1e-9 * np.max(np.abs(a))
    # a series whose sample mean is zero is left unchanged (so the subtracted
    # value is the mean over the samples, not e.g. the first sample)
    z = np.cos(2 * np.pi * 5 * np.arange(n) / n)
    assert abs(z.mean()) < 1e-15 and z[0] == 1.0
    za = spectra.conductivity(z, dt, 0.1, om, subtract_mean=True, use_mask=use_mask)
    zb = spectra.conductivity(z, dt, 0.1, om, subtract_mean=False, use_mask=use_mask)
    assert np.max(np.abs(za - zb)) < 1e-12 * np.max(np.abs(zb))


@pytest.mark.parametrize("T", [60.0, 100.0])
def test_oscillator_strength_sum_rule_and_peak(T):
    w0, f0, F0, dt = 0.5, 2.0, 1e-3, 0.02
    t = np.arange(int(round(T / dt)) + 1) * dt
    d = F0 * (f0 / w0) * np.sin(w0 * t)
    E = np.linspace(0.0, 20.0, 4001)
    df = spectra.oscillator_strength(d, dt, F0, E)
    tot = np.sum(0.5 * (df[1:] + df[:-1]) * np.diff(E))
    assert abs(tot - f0) < 1e-6 * f0
    assert abs(E[np.argmax(df)] - w0) < 0.01
    # linear in the dipole, and per unit kick
    df2 = spectra.oscillator_strength(3.0 * d, dt, 3.0 * F0, E[::100])
    assert np.max(np.abs(df2 - df[::100])) < 1e-12 * np.max(np.abs(df))


def test_em_energy_uniform_fields():
    n, dx, dt = 50, 3.0, 0.01
    E0 = 2e-3
    A_now = np.full(n, -C * E0 * dt)           # A = -c E0 t: E = E0, B = 0
    A_prev = np.zeros(n)
    ref = E0 * E0 * n * dx / (8 * math.pi)
    assert abs(maxwell.em_energy(A_now, A_prev, dx, dt) - ref) < 1e-14 * ref
    beta = 5e-4
    A = beta * np.arange(n) * dx                # B = beta on n - 1 links, E = 0
    ref = beta * beta * (n - 1) * dx / (8 * math.pi)
    assert abs(maxwell.em_energy(A, A, dx, dt) - ref) < 1e-14 * ref


def _profile(u):
    v = np.where((u > 20.0) & (u < 40.0), np.sin(math.pi * (u - 20.0) / 20.0) ** 2, 0.0)
    return v * np.cos(0.4 * u)


def test_em_energy_conserved_and_absorbed_at_courant_one():
    n, dx = 300, 2.0
    dt = dx / C
    X = np.arange(n) * dx

    def exact(t):   # a left-moving pulse starting around j = 130
        return _profile((X + C * t) / dx - 100.0)
    A_prev, A_now = exact(-dt), exact(0.0)
    # E = B on every link for a one-way wave: 2 sum (dF)^2 / dx over 8 pi
    dF = np.diff(_profile(np.arange(-50, 400) * 1.0))
    ref = 2.0 * np.sum(dF ** 2) / dx / (8 * math.pi)
    assert abs(maxwell.em_energy(A_now, A_prev, dx, dt) - ref) < 1e-13 * ref
    I = np.zeros(n)
    energies = []
    for _ in range(200):
        A_new = maxwell.leapfrog(A_now, A_prev, I, dx, dt)
        maxwell.mur_ends(A_new, A_now, dx, dt)
        A_prev, A_now = A_now, A_new
        energies.append(maxwell.em_energy(A_now, A_prev, dx, dt))
    energies = np.array(energies)
    # inside the grid for the first 100 steps: conserved to rounding
    assert np.max(np.abs(energies[:100] - ref)) < 1e-13 * ref
    # after 200 steps the pulse has left through the left end: nothing remains
    assert energies[-1] < 1e-25 * ref
