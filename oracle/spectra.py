"""Spectra from real-time series (post-processing; test infrastructure).

* conductivity sigma(omega) = -(c / A0) int_0^T dt e^{i omega t} f(t/T) I(t)
  (Sec. 4.1, Eq. sigma_ft), dielectric function eps = 1 + 4 pi i sigma / omega;
* oscillator-strength distribution df/dE = (2 E / pi) Im int_0^T f(t/T) d(t)
  e^{i E t} dt for an impulsive kick of unit strength (Sec. 3.1,
  Eq. distribution), divided here by the kick strength F0;
* mask f(x) = 1 - 3 x^2 + 2 x^3 (Sec. 3.1).
Time integrals use the trapezoid rule on the step grid t_n = n dt.
"""
import numpy as np

C_LIGHT = 137.035999084


def mask(x):
    """Cubic window f(x) = 1 - 3x^2 + 2x^3 (f(0) = 1, f(1) = 0, flat ends)."""
    x = np.asarray(x, dtype=np.float64)
    return 1.0 - 3.0 * x ** 2 + 2.0 * x ** 3


def _trapz_weights(n, dt):
    w = np.full(n, dt)
    w[0] = w[-1] = 0.5 * dt
    return w


def conductivity(I, dt, A0, omegas, subtract_mean=False, use_mask=True):
    """sigma(omega) from I(t_n), n = 0..N-1 (I[0] = current just after the kick).

    subtract_mean: replace I by I - mean(I) first, the DC correction that
    makes sigma(0) vanish for insulators (Sec. 4.2)."""
    I = np.asarray(I, dtype=np.float64)
    if subtract_mean:
        I = I - I.mean()
    n = I.shape[0]
    t = np.arange(n) * dt
    T = t[-1]
    f = mask(t / T) if use_mask else np.ones(n)
    w = _trapz_weights(n, dt) * f * I
    ph = np.exp(1j * np.outer(np.asarray(omegas), t))
    return -(C_LIGHT / A0) * ph @ w


def dielectric(sigma, omegas):
    """eps(omega) = 1 + 4 pi i sigma(omega) / omega."""
    return 1.0 + 4j * np.pi * np.asarray(sigma) / np.asarray(omegas)


def oscillator_strength(d, dt, F0, energies):
    """df/dE = (2E/pi) Im int f(t/T) d(t) e^{iEt} dt / F0 (dipole after a kick F0)."""
    d = np.asarray(d, dtype=np.float64)
    n = d.shape[0]
    t = np.arange(n) * dt
    T = t[-1]
    w = _trapz_weights(n, dt) * mask(t / T) * d
    E = np.asarray(energies)
    return 2.0 * E / np.pi * np.imag(np.exp(1j * np.outer(E, t)) @ w) / F0


def work(I, A, dt, volume):
    """Work done by the field on the electrons in the cell,
    W_n = volume * sum_{m<n} dt (I_m + I_{m+1})/2 . E_m, E_m = -(A_{m+1} - A_m)/(c dt).
    I[m] is the current at t_m (m = 0..N), A the vector-potential table."""
    I = np.asarray(I, dtype=np.float64)
    A = np.asarray(A, dtype=np.float64)
    E = -(A[1:] - A[:-1]) / (C_LIGHT * dt)
    inc = dt * np.sum(0.5 * (I[:-1] + I[1:]) * E, axis=1)
    return volume * np.concatenate([[0.0], np.cumsum(inc)])
