"""Named synthetic workloads.

Each workload stands in for one of the paper's computations by its shape:

* ``diamond-16^3-gamma``    8-atom cubic cell, 16^3 grid, 16 orbitals, Gamma,
                            s projectors, dt 0.02, 200 steps, x kick (c128).
* ``diamond-20^3-k512``     same cell, 20^3 grid, 8^3 Monkhorst-Pack k-points,
                            16 orbitals, s+p projectors, x kick; the Si
                            linear-response run of Sec. 4.2 (16^3, 8^3 k) in shape.
* ``cluster-96^3-256at``    isolated cluster: 256 atoms on jittered fcc sites
                            in a 96^3 box (h 0.45), 512 orbitals, s+p, length
                            gauge, Gaussian-envelope 1.55 eV pulse; the
                            core-shell clusters of Sec. 3.3 in shape.
* ``batch-64cells``         64 independent periodic cells of uneven size.
* ``multiscale-256X``       256 macroscopic points, each a 16^3 diamond cell
                            with 16 orbitals and 4^3 k-points (Sec. 5).

Seeds: ``SeedSequence([1804, 1404, index])`` with the index below (cells of a
batch add their cell number).
"""
from __future__ import annotations

import math

import numpy as np

from .systems import (C_AU, System, build_system, cos2_pulse_table, diamond_positions,
                      fcc_cluster, gauss_pulse_table, kick_table, mp_kgrid, rng_for)

CONFIG_NAMES = {
    0: "diamond-16^3-gamma",
    1: "diamond-20^3-k512",
    2: "cluster-96^3-256at",
    3: "batch-64cells",
    4: "multiscale-256X",
}

EV = 1.0 / 27.211386245988  # Hartree per eV
DIAMOND_L = 10.26
KICK_MOMENTUM = 1e-3          # |A0| / c, bohr^-1 (the impulse F0 of Sec. 3.1)


def single_cell_config(index: int, *, n=None, nk=None, n_orb=None, nsteps=None, dt=None,
                       precision=None, n_fcc=None, with_orbitals=True, kick=KICK_MOMENTUM,
                       hartree=True, xc=True, n_proj=None) -> System:
    """Build workload 0, 1 or 2, optionally shrunk for tests (grid, k-grid,
    orbitals, steps). The random stream depends only on ``index``."""
    rng = rng_for(index)
    if index in (0, 1):
        N = n or (16 if index == 0 else 20)
        q = nk or (1 if index == 0 else 8)
        L = DIAMOND_L
        kpts, kw = mp_kgrid((q, q, q), (L, L, L))
        steps = nsteps if nsteps is not None else (200 if index == 0 else 6000)
        return build_system(
            name=CONFIG_NAMES[index], n=(N, N, N), cell=(L, L, L), boundary="periodic",
            n_orb=n_orb or 16, kpts=kpts, kw=kw, atoms=diamond_positions(L), rng=rng,
            n_proj=n_proj if n_proj is not None else (1 if index == 0 else 4),
            dt=dt or (0.02 if index == 0 else 0.04), nsteps=steps,
            A=kick_table(steps, [C_AU * kick, 0.0, 0.0]), hartree=hartree, xc=xc,
            precision=precision or ("c128" if index == 0 else "mixed"),
            with_orbitals=with_orbitals, seed_index=index)
    if index == 2:
        N = n or 96
        h = 0.45
        L = N * h
        ncell = n_fcc or 4
        atoms = fcc_cluster(ncell, 7.72, 0.1, rng)
        steps = nsteps if nsteps is not None else 1000
        ddt = dt or 0.02
        kpts = np.zeros((1, 3))
        kw = np.ones(1)
        A = gauss_pulse_table(steps, ddt, 1e-3, 1.55 * EV, 10.0, 5.0, [0.0, 0.0, 1.0])
        return build_system(
            name=CONFIG_NAMES[2], n=(N, N, N), cell=(L, L, L), boundary="isolated",
            n_orb=n_orb or 512, kpts=kpts, kw=kw, atoms=atoms, rng=rng,
            n_proj=n_proj if n_proj is not None else 4, dt=ddt, nsteps=steps, A=A,
            hartree=hartree, xc=xc, gauge="length", precision=precision or "mixed",
            with_orbitals=with_orbitals, seed_index=2)
    raise ValueError(f"no single-cell workload with index {index}")


def _random_atoms(rng, n_at, L, min_sep=1.5):
    pts = []
    while len(pts) < n_at:
        p = rng.uniform(0.0, L, size=3)
        ok = True
        for q in pts:
            d = p - q
            d -= L * np.round(d / L)
            if np.sqrt((d * d).sum()) < min_sep:
                ok = False
                break
        if ok:
            pts.append(p)
    return np.array(pts)


def batch_cells(n_cells: int = 64, *, nsteps=500, dt=0.02, with_orbitals=True,
                max_orb=64, max_k=64, grids=(12, 16, 20, 24, 32), precision="mixed",
                cells=None) -> list:
    """Workload 3: independent periodic cells with uneven grids, orbital and
    k-point counts, atoms and pulses (cos^2 pulse, T = 10 a.u.)."""
    out = []
    for c in (range(n_cells) if cells is None else cells):
        rng = rng_for(3, c)
        N = int(rng.choice(grids))
        h = 0.55
        L = N * h
        n_orb = int(rng.integers(8, max_orb + 1))
        n_k = int(rng.integers(1, max_k + 1))
        n_at = int(rng.integers(2, 17))
        kpts = rng.uniform(-np.pi / L, np.pi / L, size=(n_k, 3))
        kw = np.full(n_k, 1.0 / n_k)
        atoms = _random_atoms(rng, n_at, L)
        E0 = float(np.exp(rng.uniform(np.log(1e-4), np.log(1e-2))))
        omega = float(rng.uniform(0.5, 3.0)) * EV
        cep = float(rng.uniform(0.0, 1.0))
        pol = rng.normal(size=3)
        A = cos2_pulse_table(nsteps, dt, E0, omega, 10.0, cep, pol)
        out.append(build_system(
            name=f"{CONFIG_NAMES[3]}/cell{c}", n=(N, N, N), cell=(L, L, L), boundary="periodic",
            n_orb=n_orb, kpts=kpts, kw=kw, atoms=atoms, rng=rng, n_proj=4, dt=dt,
            nsteps=nsteps, A=A, precision=precision, with_orbitals=with_orbitals,
            seed_index=3))
    return out


def multiscale_cell(*, nk=4, n=16, n_orb=16, dt=0.08, nsteps=0, with_orbitals=True,
                    precision="mixed") -> System:
    """Workload 4's microscopic cell: 16^3 diamond, 16 orbitals, 4^3 k-points,
    s+p projectors. The same initial orbitals sit at every macroscopic point."""
    rng = rng_for(4)
    L = DIAMOND_L
    kpts, kw = mp_kgrid((nk, nk, nk), (L, L, L))
    return build_system(
        name=CONFIG_NAMES[4], n=(n, n, n), cell=(L, L, L), boundary="periodic", n_orb=n_orb,
        kpts=kpts, kw=kw, atoms=diamond_positions(L), rng=rng, n_proj=4, dt=dt,
        nsteps=nsteps, A=np.zeros((nsteps + 1, 3)), precision=precision,
        with_orbitals=with_orbitals, seed_index=4)


def surrogate_init(window: int, hidden: int, seed: int) -> np.ndarray:
    """Seeded initial parameters of the current surrogate, float32, in the
    library's flat layout W1 [H][W], b1 [H], W2 [H][H], b2 [H], w3 [H], b3,
    ws [W]: Glorot-uniform dense weights, zero biases, zero skip weights."""
    rng = rng_for(7, seed)
    W, H = int(window), int(hidden)

    def glorot(fan_out, fan_in):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        return rng.uniform(-lim, lim, size=(fan_out, fan_in))
    parts = [glorot(H, W), np.zeros(H), glorot(H, H), np.zeros(H), glorot(1, H)[0], np.zeros(1), np.zeros(W)]
    return np.concatenate([np.ravel(p) for p in parts]).astype(np.float32)


def random_pulse_tables(n_traj: int, n_macro: int, dt_macro: float, seed: int, *,
                        e0_range=(1e-4, 1e-2), ev_range=(0.5, 3.0), t_range=(40.0, 200.0)):
    """Seeded training fields for the surrogate: per trajectory a cos^2
    pulse (log-uniform peak field, uniform photon energy in eV, duration in
    a.u., carrier-envelope phase) sampled at the macroscopic times
    t_0 .. t_{n_macro - 1}; returns A [n_traj][n_macro] along one axis and
    the pulse parameters."""
    rng = rng_for(8, seed)
    out = np.empty((n_traj, n_macro))
    params = []
    for i in range(n_traj):
        E0 = float(np.exp(rng.uniform(np.log(e0_range[0]), np.log(e0_range[1]))))
        omega = float(rng.uniform(*ev_range)) * EV
        T = float(rng.uniform(*t_range))
        cep = float(rng.uniform(0.0, 1.0))
        tab = cos2_pulse_table(n_macro - 1, dt_macro, E0, omega, T, cep, [1.0, 0.0, 0.0])
        out[i] = tab[:, 0]
        params.append((E0, omega, T, cep))
    return out, params


def random_field_tables(n_traj: int, n_macro: int, dt_macro: float, seed: int, *, a_max=10.0,
                        ev_range=(0.3, 4.0)):
    """Seeded, varied training fields for the surrogate, A [n_traj][n_macro]
    along one axis at the macroscopic times: in turn a cos^2 pulse of random
    duration (10..150 a.u.), photon energy, phase and peak; a smoothed step
    (an impulsive kick) at a random time; and a superposition of 12 random
    short pulses (a broadband field). Peaks of |A| are log-uniform in
    [a_max / 100, a_max]; every field is zero at t_0."""
    rng = rng_for(9, seed)
    t = np.arange(n_macro) * dt_macro
    out = np.zeros((n_traj, n_macro))
    for i in range(n_traj):
        kind = i % 3
        if kind == 0:
            T = float(rng.uniform(10.0, 150.0))
            om = float(rng.uniform(*ev_range)) * EV
            t0 = float(rng.uniform(0.0, 0.3)) * t[-1]
            env = np.where((t > t0) & (t < t0 + T), np.sin(np.pi * (t - t0) / T) ** 2, 0.0)
            a = env * np.sin(om * (t - t0) + 2 * np.pi * rng.uniform())
        elif kind == 1:
            t0 = float(rng.uniform(0.05, 0.6)) * t[-1]
            w = float(rng.uniform(0.5, 3.0))
            a = 0.5 * (1.0 + np.tanh((t - t0) / w))
            a -= a[0]
        else:
            a = np.zeros(n_macro)
            for _ in range(12):
                T = float(rng.uniform(5.0, 40.0))
                om = float(rng.uniform(*ev_range)) * EV
                t0 = float(rng.uniform(0.0, 0.9)) * t[-1]
                env = np.where((t > t0) & (t < t0 + T), np.sin(np.pi * (t - t0) / T) ** 2, 0.0)
                a += rng.normal() * env * np.sin(om * (t - t0) + 2 * np.pi * rng.uniform())
        peak = float(np.exp(rng.uniform(np.log(a_max / 100.0), np.log(a_max))))
        m = np.max(np.abs(a))
        out[i] = a * (peak / m) if m > 0 else a
    return out


def cos2_pulse_potential(tau, E0, omega, T):
    """A(tau) = -c int_0^tau E for E(t) = E0 sin^2(pi t/T) sin(omega t) on
    0 < t < T (Eq. pulse of Sec. 3.1 with a sine carrier), constant after T,
    zero before 0; closed form of the integral."""
    p = math.pi / T
    tau = np.clip(np.asarray(tau, dtype=np.float64), 0.0, T)

    def prim(t):
        out = -0.5 * np.cos(omega * t) / omega
        out = out + 0.25 * np.cos((omega + 2 * p) * t) / (omega + 2 * p)
        wm = omega - 2 * p
        if abs(wm) > 1e-12:
            out = out + 0.25 * np.cos(wm * t) / wm
        return out
    return -C_AU * E0 * (prim(tau) - prim(0.0))


def incident_table(n_macro, dt, dx, delay, E0, omega, T):
    """Incident A at X_0 = 0 and X_1 = dX for t_0 .. t_{n_macro}: the pulse
    travels towards +X and reaches X = 0 at t = delay."""
    t = np.arange(n_macro + 1) * dt
    out = np.empty((n_macro + 1, 2))
    out[:, 0] = cos2_pulse_potential(t - delay, E0, omega, T)
    out[:, 1] = cos2_pulse_potential(t - delay - dx / C_AU, E0, omega, T)
    return out
