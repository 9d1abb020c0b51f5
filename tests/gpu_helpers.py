"""Shared helpers of the GPU tests: run a system through the C ABI and
through the oracle on the same seeded inputs."""
import sys

import numpy as np

from oracle import tdks


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def gpu_run(system, nsteps=None, precision=None, flags=0, A=None):
    from paper_1804_01404_amd.binding import TDDFT
    A = system.A if A is None else A
    if nsteps is not None:
        A = A[: nsteps + 1]
    announce(f"{system.name} n={system.n} n_orb={system.n_orb} n_k={system.n_k} "
             f"steps={A.shape[0] - 1} prec={precision or system.precision}")
    with TDDFT(system, precision=precision, flags=flags) as t:
        t.set_potential()
        J = t.propagate(A)
        rho, Jnow = t.density_current()
        psi = t.orbitals()
        E = t.energy()
        norms = t.norms()
        d = t.dipole()
    return dict(J=J, rho=rho, psi=psi, E=E, norms=norms, dipole=d, Jnow=Jnow)


def oracle_run(system, nsteps=None, A=None):
    A = system.A if A is None else A
    if nsteps is not None:
        A = A[: nsteps + 1]
    o = tdks.TDKS.from_system(system)
    J = o.propagate(A)
    return dict(J=J, rho=o.rho, psi=o.psi, E=o.energy(), norms=o.norms(), dipole=o.dipole(),
                obj=o)


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def max_rel_series(a, b):
    """max_t |a - b| / max_t |b| per component, maximised over components."""
    scale = np.max(np.abs(b), axis=0)
    scale = np.where(scale > 0, scale, 1.0)
    return float(np.max(np.max(np.abs(a - b), axis=0) / scale))
