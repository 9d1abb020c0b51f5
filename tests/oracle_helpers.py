"""Small seeded systems shared by the oracle pin tests (inputs only)."""
import numpy as np

import synth
from synth.systems import build_system, rng_for


def tiny_periodic(n=10, L=6.4, n_orb=4, kpts=None, n_atoms=3, n_proj=4, dt=0.02, nsteps=4,
                  A=None, hartree=True, xc=True, seed=101, real=True):
    """A small periodic cell with random atoms, s+p projectors and k-points."""
    rng = rng_for(seed)
    atoms = rng.uniform(0.0, L, size=(n_atoms, 3))
    if kpts is None:
        kpts = np.zeros((1, 3))
    kpts = np.asarray(kpts, dtype=np.float64)
    kw = np.full(kpts.shape[0], 1.0 / kpts.shape[0])
    if A is None:
        A = np.zeros((nsteps + 1, 3))
    s = build_system(name="tiny", n=(n, n, n), cell=(L, L, L), boundary="periodic", n_orb=n_orb,
                     kpts=kpts, kw=kw, atoms=atoms, rng=rng, n_proj=n_proj, dt=dt,
                     nsteps=nsteps, A=A, hartree=hartree, xc=xc)
    if not real:
        # give the Gamma-point orbitals a random complex phase pattern
        ph = np.exp(1j * rng.uniform(0, 2 * np.pi, size=s.psi0.shape[:2]))
        s.psi0 = s.psi0 * ph[:, :, None, None, None]
    return s


def tiny_isolated(n=12, h=0.5, n_orb=4, n_atoms=2, n_proj=4, dt=0.02, nsteps=4, A=None,
                  hartree=True, xc=True, seed=202, gauge="length"):
    rng = rng_for(seed)
    L = n * h
    atoms = rng.uniform(-0.15 * L, 0.15 * L, size=(n_atoms, 3))
    if A is None:
        A = np.zeros((nsteps + 1, 3))
    return build_system(name="tiny-iso", n=(n, n, n), cell=(L, L, L), boundary="isolated",
                        n_orb=n_orb, kpts=np.zeros((1, 3)), kw=np.ones(1), atoms=atoms, rng=rng,
                        n_proj=n_proj, dt=dt, nsteps=nsteps, A=A, hartree=hartree, xc=xc,
                        gauge=gauge)
