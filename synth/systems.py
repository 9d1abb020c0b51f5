"""System description and seeded generators (inputs only, no propagation math).

Conventions shared by every consumer:

* atomic units (Hartree, bohr, hbar = m = e = 1); ``C_AU`` is the speed of
  light, 1/alpha (CODATA 2018);
* a grid array has numpy shape ``(n3, n2, n1)`` with x (axis 2) fastest; the
  flat index of point (i1, i2, i3) is ``(i3 * n2 + i2) * n1 + i1``;
* periodic grids sit at ``r_j = j h``; isolated grids are centred on the box,
  ``r_j = (j - (N - 1) / 2) h``, and the orbitals vanish outside the box;
* orbitals are stored ``[n_k][n_orb][n3][n2][n1]`` complex128 and normalised
  to one over the box with the weight ``h1 h2 h3``.

The synthetic pseudopotential replaces the paper's norm-conserving files
(Sec. 2.1; Kleinman-Bylander form, Sec. 3.1): each atom carries a Gaussian
local well and separable projectors of s (and optionally p) symmetry on a
sphere of radius ``r_c``.
"""
from __future__ import annotations

import dataclasses
import os
from typing import List, Optional, Sequence

import numpy as np
import scipy.fft as sfft

C_AU = 137.035999084  # speed of light in atomic units


def rng_for(index: int, *extra: int) -> np.random.Generator:
    """PCG64 generator seeded by SeedSequence([1804, 1404, index, *extra])."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([1804, 1404, int(index), *map(int, extra)])))


@dataclasses.dataclass
class AtomProjector:
    """Kleinman-Bylander projectors of one atom restricted to its sphere.

    idx   int32 [npts]        flat grid index of each sphere point (ascending)
    x     float64 [npts, 3]   offset r - R_a of that point (minimum image)
    beta  float64 [n_proj, npts] real projector values, h^3 sum beta^2 = 1
    e_kb  float64 [n_proj]    KB energies (Ha)
    """

    idx: np.ndarray
    x: np.ndarray
    beta: np.ndarray
    e_kb: np.ndarray

    @property
    def npts(self) -> int:
        return int(self.idx.shape[0])

    @property
    def n_proj(self) -> int:
        return int(self.beta.shape[0])


@dataclasses.dataclass
class System:
    """Everything one cell of the TDKS time step needs, in plain arrays."""

    name: str
    n: tuple                      # (n1, n2, n3) grid points along x, y, z
    cell: tuple                   # (L1, L2, L3) box lengths, bohr
    boundary: str                 # 'periodic' | 'isolated'
    n_orb: int
    kpts: np.ndarray              # [n_k, 3] bohr^-1
    kw: np.ndarray                # [n_k] weights, sum 1
    atoms: np.ndarray             # [n_at, 3] positions (grid frame)
    depth: np.ndarray             # [n_at] Gaussian well depth U (Ha)
    width: np.ndarray             # [n_at] Gaussian well width w (bohr)
    v_loc: np.ndarray             # [n3, n2, n1] local potential (Ha)
    projectors: List[AtomProjector]
    psi0: Optional[np.ndarray]    # [n_k, n_orb, n3, n2, n1] complex128
    dt: float
    nsteps: int
    A: np.ndarray                 # [nsteps + 1, 3] vector potential at t_n = n dt
    hartree: bool = True
    xc: bool = True               # PZ81 LDA
    gauge: str = "velocity"       # 'velocity' | 'length' (isolated only)
    precision: str = "c128"       # 'c128' | 'mixed'
    r_c: float = 2.0
    sigma: float = 1.0
    seed_index: int = 0

    @property
    def h(self) -> tuple:
        return tuple(self.cell[i] / self.n[i] for i in range(3))

    @property
    def n_k(self) -> int:
        return int(self.kpts.shape[0])

    @property
    def n_grid(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def og(self) -> int:
        """orbital x k-point x grid-point count of one step."""
        return self.n_orb * self.n_k * self.n_grid

    @property
    def n_proj(self) -> int:
        return self.projectors[0].n_proj if self.projectors else 0


# --------------------------------------------------------------------------
# geometry


def mp_kgrid(nk: Sequence[int], cell: Sequence[float]) -> tuple:
    """Unshifted Monkhorst-Pack grid: k = (2i - q - 1) / (2q) * 2 pi / L,
    i = 1..q per axis, equal weights. q = 1 gives the Gamma point."""
    axes = []
    for q, L in zip(nk, cell):
        i = np.arange(1, q + 1)
        axes.append((2 * i - q - 1) / (2.0 * q) * 2 * np.pi / L)
    kz, ky, kx = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    k = np.stack([kx.ravel(), ky.ravel(), kz.ravel()], axis=1)
    w = np.full(k.shape[0], 1.0 / k.shape[0])
    return k, w


def diamond_positions(L: float) -> np.ndarray:
    """8 atoms of the conventional diamond cell, in bohr (periodic frame)."""
    f = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0],
                  [.25, .25, .25], [.25, .75, .75], [.75, .25, .75], [.75, .75, .25]])
    return f * L


def fcc_cluster(ncell: int, a: float, jitter: float, rng: np.random.Generator) -> np.ndarray:
    """ncell^3 conventional fcc cells (4 atoms each) centred on the origin,
    each atom displaced by N(0, jitter) per component."""
    base = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
    pts = []
    for i in range(ncell):
        for j in range(ncell):
            for k in range(ncell):
                pts.append((base + np.array([i, j, k])) * a)
    pts = np.concatenate(pts, axis=0)
    pts -= pts.mean(axis=0)
    pts += rng.normal(0.0, jitter, size=pts.shape)
    return pts


def grid_coords(n: Sequence[int], cell: Sequence[float], boundary: str) -> list:
    """1-D coordinate arrays (x, y, z) of the grid points."""
    out = []
    for N, L in zip(n, cell):
        h = L / N
        j = np.arange(N, dtype=np.float64)
        out.append(j * h if boundary == "periodic" else (j - (N - 1) / 2.0) * h)
    return out


def _offsets(n, cell, boundary, R):
    """Offsets r - R over the whole grid (minimum image when periodic)."""
    xs = grid_coords(n, cell, boundary)
    d = []
    for ax in range(3):
        v = xs[ax] - R[ax]
        if boundary == "periodic":
            v = v - cell[ax] * np.round(v / cell[ax])
        d.append(v)
    return d


def gaussian_vloc(n, cell, boundary, atoms, depth, width, cut: float = 10.0) -> np.ndarray:
    """V_loc(r) = sum_a sum_images -U_a exp(-|x|^2 / (2 w_a^2)) for |x| <= cut*w_a."""
    xs = grid_coords(n, cell, boundary)
    V = np.zeros((n[2], n[1], n[0]))
    for R, U, w in zip(atoms, depth, width):
        rc = cut * w
        if boundary == "periodic":
            ranges = [range(-int(np.ceil(rc / L)) - 1, int(np.ceil(rc / L)) + 2) for L in cell]
        else:
            ranges = [range(0, 1)] * 3
        for i3 in ranges[2]:
            dz = xs[2] - R[2] - i3 * cell[2]
            for i2 in ranges[1]:
                dy = xs[1] - R[1] - i2 * cell[1]
                for i1 in ranges[0]:
                    dx = xs[0] - R[0] - i1 * cell[0]
                    r2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
                    m = r2 <= rc * rc
                    if m.any():
                        V[m] += -U * np.exp(-r2[m] / (2 * w * w))
    return V


def build_projectors(n, cell, boundary, atoms, e_kb, r_c: float = 2.0, sigma: float = 1.0) -> List[AtomProjector]:
    """Sphere tables of s (+p) projectors, normalised on the grid.

    g(r) = exp(-r^2 / 2 sigma^2) (1 - r^2 / r_c^2)^2 on r < r_c (strict);
    s: beta = N_s g, p_mu: beta = N_p (x_mu / r_c) g, with h^3 sum beta^2 = 1.
    """
    h = [cell[i] / n[i] for i in range(3)]
    dV = h[0] * h[1] * h[2]
    out = []
    n_proj = e_kb.shape[1]
    for a, R in enumerate(atoms):
        d = _offsets(n, cell, boundary, R)
        r2 = d[2][:, None, None] ** 2 + d[1][None, :, None] ** 2 + d[0][None, None, :] ** 2
        sel = np.nonzero((r2 < r_c * r_c).ravel())[0]
        i3, i2, i1 = np.unravel_index(sel, (n[2], n[1], n[0]))
        x = np.stack([d[0][i1], d[1][i2], d[2][i3]], axis=1)
        rr = (x ** 2).sum(axis=1)
        g = np.exp(-rr / (2 * sigma * sigma)) * (1 - rr / (r_c * r_c)) ** 2
        betas = [g]
        if n_proj == 4:
            betas += [x[:, m] / r_c * g for m in range(3)]
        beta = np.stack(betas, axis=0)
        beta /= np.sqrt(dV * (beta ** 2).sum(axis=1, keepdims=True))
        out.append(AtomProjector(idx=sel.astype(np.int32), x=x, beta=beta,
                                 e_kb=np.asarray(e_kb[a], dtype=np.float64).copy()))
    return out


# --------------------------------------------------------------------------
# initial orbitals


def _orthonormalise(W: np.ndarray, dV: float) -> np.ndarray:
    """Gram-Schmidt in orbital order, written as Cholesky-QR applied twice.

    W is [n_orb, npts]; returns L^-1 W with S = dV W W^H = L L^H, which is the
    Gram-Schmidt result (lower-triangular map with positive diagonal)."""
    import scipy.linalg as sla
    for _ in range(2):
        S = dV * (W @ W.conj().T)
        S = 0.5 * (S + S.conj().T)
        L = np.linalg.cholesky(S)
        # L^-1 W as a product with the small inverse (one threaded GEMM)
        Linv = sla.solve_triangular(L, np.eye(L.shape[0], dtype=L.dtype), lower=True)
        W = Linv @ W
    return W


def random_orbitals(n, cell, boundary, kpts, n_orb, rng, ecut: float = 4.0,
                    real_gamma: bool = True) -> np.ndarray:
    """Seeded smooth orthonormal orbitals, [n_k, n_orb, n3, n2, n1] complex128.

    Periodic: complex normal plane-wave coefficients on 0.5|G+k|^2 <= ecut
    (the cutoff grows until it holds at least 2 n_orb waves). Isolated:
    the same filter on the box, times a sin^2 window vanishing at the walls.
    Gamma-only periodic and isolated sets are real-valued when ``real_gamma``.
    """
    from concurrent.futures import ThreadPoolExecutor
    from threadpoolctl import threadpool_limits
    h = [cell[i] / n[i] for i in range(3)]
    dV = h[0] * h[1] * h[2]
    gs = [2 * np.pi * np.fft.fftfreq(n[i], d=1.0 / n[i]) / cell[i] for i in range(3)]
    out = np.empty((kpts.shape[0], n_orb, n[2], n[1], n[0]), dtype=np.complex128)
    ncpu = os.cpu_count() or 1
    # the random coefficients are drawn k-point by k-point in order; the
    # transforms and orthonormalisations of the k-points then run side by side
    draws = []
    for ik, k in enumerate(kpts):
        ec = ecut
        while True:
            g2 = ((gs[2][:, None, None] + k[2]) ** 2 + (gs[1][None, :, None] + k[1]) ** 2
                  + (gs[0][None, None, :] + k[0]) ** 2)
            mask = 0.5 * g2 <= ec
            if mask.sum() >= 2 * n_orb:
                break
            ec *= 1.5
        real = real_gamma and (boundary == "isolated" or not np.any(k))
        # coefficients drawn orbital by orbital (real parts, then imaginary
        # parts), then one batched inverse FFT on all host cores
        W = np.zeros((n_orb, n[2], n[1], n[0]), dtype=np.complex128)
        m = int(mask.sum())
        for j in range(n_orb):
            W[j][mask] = rng.normal(size=m) + 1j * rng.normal(size=m)
        draws.append([W, real])

    def finish(ik, workers):
        W, real = draws[ik]
        draws[ik] = None
        W = sfft.ifftn(W, axes=(1, 2, 3), overwrite_x=True, workers=workers)
        if real:
            W = W.real.astype(np.complex128)
        if boundary == "isolated":
            win = [np.sin(np.pi * (np.arange(N) + 1) / (N + 1)) ** 2 for N in n]
            W *= win[2][:, None, None] * win[1][None, :, None] * win[0][None, None, :]
        W = _orthonormalise(W.reshape(n_orb, -1), dV).reshape(W.shape)
        if real:
            W = W.real.astype(np.complex128)
        out[ik] = W

    if len(draws) > 1 and ncpu > 1:
        with threadpool_limits(limits=1), ThreadPoolExecutor(max_workers=min(ncpu, len(draws))) as ex:
            list(ex.map(lambda ik: finish(ik, 1), range(len(draws))))
    else:
        for ik in range(len(draws)):
            finish(ik, ncpu)
    return out


# --------------------------------------------------------------------------
# vector-potential tables (A at t_n = n dt, n = 0..nsteps)


def kick_table(nsteps: int, A0: Sequence[float]) -> np.ndarray:
    """Impulsive kick A(t) = A0 theta(t) (Sec. 4.1, Eq. impulsive_A):
    A_n = A0 for every n >= 0 (the step function has already switched on)."""
    return np.tile(np.asarray(A0, dtype=np.float64), (nsteps + 1, 1))


def cos2_pulse_table(nsteps: int, dt: float, E0: float, omega: float, T: float,
                     cep: float, pol: Sequence[float]) -> np.ndarray:
    """A(t) = Im{A0 cos^2[pi (t - T/2) / T] exp[-i omega (t - T/2) - 2 pi i cep]}
    on 0 < t < T (Eq. pulse), A0 = (c E0 / omega) * pol with a real unit pol."""
    t = np.arange(nsteps + 1) * dt
    pol = np.asarray(pol, dtype=np.float64)
    pol = pol / np.linalg.norm(pol)
    env = np.where((t > 0) & (t < T), np.cos(np.pi * (t - T / 2) / T) ** 2, 0.0)
    ph = np.exp(-1j * omega * (t - T / 2) - 2j * np.pi * cep)
    a = C_AU * E0 / omega * env * ph.imag
    return a[:, None] * pol[None, :]


def gauss_pulse_table(nsteps: int, dt: float, E0: float, omega: float, t0: float,
                      tau: float, pol: Sequence[float], sub: int = 32) -> np.ndarray:
    """A(t) = -c int_0^t E dt' for E(t) = E0 exp(-(t-t0)^2 / 2 tau^2) cos(omega (t - t0)),
    integrated with composite Simpson on ``sub`` sub-intervals per step."""
    pol = np.asarray(pol, dtype=np.float64)
    pol = pol / np.linalg.norm(pol)
    Ef = lambda t: E0 * np.exp(-(t - t0) ** 2 / (2 * tau * tau)) * np.cos(omega * (t - t0))
    s = np.linspace(0.0, dt, 2 * sub + 1)
    wts = np.ones(2 * sub + 1)
    wts[1:-1:2] = 4
    wts[2:-1:2] = 2
    wts *= (dt / (2 * sub)) / 3.0
    inc = np.array([np.dot(wts, Ef(n * dt + s)) for n in range(nsteps)])
    a = np.concatenate([[0.0], -C_AU * np.cumsum(inc)])
    return a[:, None] * pol[None, :]


# --------------------------------------------------------------------------


def build_system(*, name, n, cell, boundary, n_orb, kpts, kw, atoms, rng, n_proj,
                 dt, nsteps, A, hartree=True, xc=True, gauge="velocity", precision="c128",
                 r_c=2.0, sigma=1.0, with_orbitals=True, seed_index=0,
                 depth_range=(1.0, 3.0), width_range=(0.8, 1.2), ekb_range=(0.5, 2.0)) -> System:
    n = tuple(int(v) for v in n)
    cell = tuple(float(v) for v in cell)
    n_at = atoms.shape[0]
    depth = rng.uniform(*depth_range, size=n_at)
    width = rng.uniform(*width_range, size=n_at)
    e_kb = rng.uniform(*ekb_range, size=(n_at, n_proj)) if n_proj else np.zeros((n_at, 0))
    v_loc = gaussian_vloc(n, cell, boundary, atoms, depth, width)
    projs = build_projectors(n, cell, boundary, atoms, e_kb, r_c=r_c, sigma=sigma) if n_proj else []
    psi0 = random_orbitals(n, cell, boundary, kpts, n_orb, rng) if with_orbitals else None
    return System(name=name, n=n, cell=cell, boundary=boundary, n_orb=n_orb, kpts=kpts, kw=kw,
                  atoms=atoms, depth=depth, width=width, v_loc=v_loc, projectors=projs,
                  psi0=psi0, dt=dt, nsteps=nsteps, A=A, hartree=hartree, xc=xc, gauge=gauge,
                  precision=precision, r_c=r_c, sigma=sigma, seed_index=seed_index)
