"""Pins of the oracle's Hartree, LDA and pseudopotential tables.

* periodic Hartree: rho = cos(G.r) gives V_H = 4 pi / G^2 cos(G.r);
* isolated Hartree (doubled-box FFT) equals the pair-by-pair sum; a Gaussian
  charge gives erf(r / sqrt 2 s) / r far away; the self-cell average of 1/r
  equals an independent quadrature and the cube constant;
* PZ81: v = d(rho eps)/d rho by finite differences, exchange closed form,
  the branch values at r_s = 1 (Perdew-Zunger 1981);
* the potential and projector tables the input generator hands to both sides
  equal the oracle's own derivation from the atom parameters.
"""
import numpy as np
import pytest
from scipy import integrate, special

import synth
from oracle import tdks
from oracle_helpers import tiny_isolated, tiny_periodic


def test_hartree_periodic_cosine():
    grid = tdks.Grid((12, 10, 16), (7.0, 6.5, 9.0), "periodic")
    x, y, z = grid.r_fields()
    for m in [(1, 0, 0), (2, -3, 1), (0, 0, 5)]:
        G = np.array([2 * np.pi * m[i] / grid.cell[i] for i in range(3)])
        rho = np.cos(G[0] * x + G[1] * y + G[2] * z)
        V = tdks.hartree_periodic(rho, grid)
        assert np.max(np.abs(V - 4 * np.pi / (G @ G) * rho)) < 1e-12 * 4 * np.pi / (G @ G)
    assert np.max(np.abs(tdks.hartree_periodic(np.ones(grid.shape), grid))) < 1e-13


def test_self_cell_average_of_inverse_r():
    # unit cube: 2.38007736...; independent check by the Duffy split into three
    # pyramids, each with a smooth integrand after t-scaling
    assert abs(tdks.coulomb_self_cell((1.0, 1.0, 1.0)) - 2.3800773639795523) < 1e-13

    def duffy(a, b, c):
        tot = 0.0
        for (p, q, r) in [(a, b, c), (b, c, a), (c, a, b)]:
            v, _ = integrate.dblquad(lambda u, s: 1 / np.sqrt(1 + s * s + u * u), 0, q / p, 0, r / p,
                                     epsabs=1e-13, epsrel=1e-13)
            tot += p * p / 2 * v
        return tot
    h = (0.4, 0.55, 0.7)
    ref = 8 * duffy(h[0] / 2, h[1] / 2, h[2] / 2) / (h[0] * h[1] * h[2])
    assert abs(tdks.coulomb_self_cell(h) - ref) < 1e-10 * ref


def test_hartree_isolated_equals_pairwise_sum():
    rng = np.random.default_rng(5)
    grid = tdks.Grid((9, 8, 7), (4.5, 4.8, 4.9), "isolated")
    rho = rng.uniform(0, 1, size=grid.shape)
    V = tdks.hartree_isolated(rho, grid)
    Vd = tdks.hartree_isolated_direct(rho, grid)
    assert np.max(np.abs(V - Vd)) < 1e-11 * np.max(np.abs(Vd))


def test_hartree_isolated_gaussian_far_field():
    grid = tdks.Grid((40, 40, 40), (20.0, 20.0, 20.0), "isolated")
    x, y, z = grid.r_fields()
    s = 1.2
    r2 = x ** 2 + y ** 2 + z ** 2
    rho = np.exp(-r2 / (2 * s * s)) / (2 * np.pi * s * s) ** 1.5
    V = tdks.hartree_isolated(rho, grid)
    r = np.sqrt(r2)
    ref = special.erf(r / (np.sqrt(2) * s)) / np.where(r > 0, r, 1)
    far = r > 5.0
    assert np.max(np.abs(V[far] - ref[far]) / ref[far]) < 1e-4


def test_pz81_derivative_and_branches():
    rho = np.geomspace(1e-6, 50.0, 400)
    v, e = tdks.lda_pz81(rho)
    d = 1e-6
    f = lambda r: r * tdks.lda_pz81(r)[1]
    num = (f(rho * (1 + d)) - f(rho * (1 - d))) / (2 * d * rho)
    rs = (3 / (4 * np.pi * rho)) ** (1 / 3)
    away = np.abs(rs - 1) > 1e-3        # the two branches meet (with a small kink) at r_s = 1
    assert np.max(np.abs(num[away] - v[away]) / np.abs(v[away])) < 1e-8
    # exchange alone: eps_x = -(3/4)(3/pi)^(1/3) rho^(1/3) = -0.4581652932831429 / r_s
    ex = -0.75 * (3 / np.pi) ** (1 / 3) * rho ** (1 / 3)
    assert np.allclose(ex, -0.4581652932831429 / rs, rtol=1e-14)
    # correlation at r_s = 1 from the two sides: gamma/(1+b1+b2) and B + D
    rho1 = 3 / (4 * np.pi)
    e_hi = tdks.lda_pz81(np.array([rho1]))[1][0] - (-0.4581652932831429)
    assert abs(e_hi - (-0.1423 / (1 + 1.0529 + 0.3334))) < 1e-12
    e_lo = tdks.lda_pz81(np.array([rho1 * (1 + 1e-12)]))[1][0] + 0.4581652932831429 * (1 + 1e-12) ** (1 / 3)
    assert abs(e_lo - (-0.048 - 0.0116)) < 1e-9
    assert np.all(tdks.lda_pz81(np.array([0.0, 1e-31]))[0] == 0)


@pytest.mark.parametrize("which", ["periodic", "isolated", "diamond"])
def test_generated_tables_match_oracle_derivation(which):
    if which == "periodic":
        s = tiny_periodic()
    elif which == "isolated":
        s = tiny_isolated()
    else:
        s = synth.single_cell_config(1, nk=1, with_orbitals=False, nsteps=0)
    grid = tdks.Grid(s.n, s.cell, s.boundary)
    V = tdks.local_potential(grid, s.atoms, s.depth, s.width)
    assert np.max(np.abs(V - s.v_loc)) < 1e-13
    for R, pr in zip(s.atoms, s.projectors):
        idx, x, beta = tdks.projector_table(grid, R, pr.n_proj, s.r_c, s.sigma)
        assert np.array_equal(idx, pr.idx.astype(np.int64))
        assert np.max(np.abs(x - pr.x)) < 1e-13
        assert np.max(np.abs(beta - pr.beta)) < 1e-12


def test_sphere_sizes_of_the_diamond_cells():
    # r_c = 2 bohr spheres: 123 points at h = 0.641 and 251 at h = 0.513
    s16 = synth.single_cell_config(0, with_orbitals=False, nsteps=0)
    s20 = synth.single_cell_config(1, nk=1, with_orbitals=False, nsteps=0)
    assert {p.npts for p in s16.projectors} == {123}
    assert {p.npts for p in s20.projectors} == {251}
