"""GPU parity of the Becke-Johnson / Tran-Blaha exchange (Sec. 4.1) against the
FP64 oracle, through the C ABI.

* TB09 (c from the density at every update) and BJ (c = 1) on a periodic cell
  with projectors, two k-points and a vector-potential pulse, so that the
  kinetic energy density carries kappa = k + A/c; both the fused and the
  per-stage path; complex128 within 1e-10 (orbitals, density) and 1e-8 of
  the current's maximum, the mixing parameter c within 1e-12;
* the mixed path within the mixed-precision bounds of the LDA tests;
* BJ on an isolated box in the length gauge (zero halo in grad rho, lap rho
  and tau);
* the predictor-corrector step and the imaginary-time ground state with TB09;
* 20 orbital k-points, so that the density and tau partial sums run in
  three chunks (the last ragged) and are reduced; the full 20^3 x 512-k cell
  (512 chunks): density against the downloaded orbitals, c against the
  oracle's c of that density;
* a batch of TB09 cells equals their solo runs bit for bit.
"""
import numpy as np
import pytest

import synth
from oracle import tdks
from oracle_helpers import tiny_isolated, tiny_periodic
from gpu_helpers import announce, max_rel_series, rel_l2

pytestmark = pytest.mark.gpu
STREAMING = 8
PC = 32
PATHS = [pytest.param(0, id="fused"), pytest.param(STREAMING, id="streaming")]


def _pulse_system(xc, nsteps=8):
    k = np.array([[0.0, 0.0, 0.0], [0.17, -0.11, 0.23]])
    A = synth.cos2_pulse_table(nsteps, 0.02, 0.05, 0.6, 0.16, 0.0, [1.0, 0.5, 0.0])
    s = tiny_periodic(n=12, L=6.0, n_orb=4, kpts=k, nsteps=nsteps, A=A, dt=0.02, real=False, seed=7701)
    s.xc = xc
    return s


def _gpu(s, precision, flags=0, A=None):
    from paper_1804_01404_amd.binding import TDDFT
    A = s.A if A is None else A
    announce(f"mgga xc={s.xc} {s.boundary} n={s.n} prec={precision} flags={flags} steps={A.shape[0] - 1}")
    with TDDFT(s, precision=precision, flags=flags) as t:
        t.set_potential()
        c0 = t.xc_parameter()
        J = t.propagate(A)
        rho, _ = t.density_current()
        psi = t.orbitals()
        c1 = t.xc_parameter()
    return dict(J=J, rho=rho, psi=psi, c0=c0, c1=c1)


def _oracle(s, A=None, pc=False):
    o = tdks.TDKS.from_system(s, predictor_corrector=pc)
    c0 = o.mgga_c
    J = o.propagate(s.A if A is None else A)
    return dict(J=J, rho=o.rho, psi=o.psi, c0=c0, c1=o.mgga_c)


@pytest.mark.parametrize("flags", PATHS)
@pytest.mark.parametrize("xc", ["tb09", "bj"])
def test_periodic_pulse_matches_oracle(xc, flags):
    s = _pulse_system(xc)
    g = _gpu(s, "c128", flags)
    o = _oracle(s)
    assert abs(g["c0"] - o["c0"]) < 1e-12 and abs(g["c1"] - o["c1"]) < 1e-12
    if xc == "bj":
        assert g["c1"] == 1.0
    assert rel_l2(g["rho"], o["rho"]) < 1e-10
    assert np.max(np.abs(g["psi"] - o["psi"])) < 1e-10
    assert max_rel_series(g["J"], o["J"]) < 1e-8


@pytest.mark.parametrize("flags", PATHS)
@pytest.mark.parametrize("prec", ["c128", "mixed"])
def test_tb09_several_density_chunks(prec, flags):
    """20 orbital k-points: the density and tau partial sums run in three
    chunks of 8 (the last one ragged) and are reduced, instead of being
    written in place."""
    k = np.array([[0.0, 0.0, 0.0], [0.17, -0.11, 0.23], [-0.2, 0.1, 0.05], [0.3, 0.3, -0.1], [0.0, -0.25, 0.15]])
    nsteps = 5
    A = synth.cos2_pulse_table(nsteps, 0.02, 0.05, 0.6, 0.1, 0.0, [0.5, 1.0, 0.0])
    s = tiny_periodic(n=12, L=6.0, n_orb=4, kpts=k, nsteps=nsteps, A=A, dt=0.02, real=False, seed=7705)
    s.xc = "tb09"
    g = _gpu(s, prec, flags)
    o = _oracle(s)
    if prec == "c128":
        assert abs(g["c1"] - o["c1"]) < 1e-12
        assert rel_l2(g["rho"], o["rho"]) < 1e-10
        assert np.max(np.abs(g["psi"] - o["psi"])) < 1e-10
        assert max_rel_series(g["J"], o["J"]) < 1e-8
    else:
        assert abs(g["c1"] - o["c1"]) < 1e-6
        assert rel_l2(g["rho"], o["rho"]) < 2e-6 * np.sqrt(nsteps)
        assert max_rel_series(g["J"], o["J"]) < 1e-5


@pytest.mark.parametrize("flags", PATHS)
def test_full_size_tb09_density_and_c(flags):
    """The 20^3 cell with 512 k-points and TB09, one step: the density, summed
    over 512 chunks of 16 orbitals beside the kinetic energy density and then
    reduced, equals the density of the downloaded orbitals, and c equals the
    oracle's c of that density."""
    from oracle import mgga
    s = synth.single_cell_config(1, nsteps=1)
    s.xc = "tb09"
    grid = tdks.Grid(s.n, s.cell, s.boundary)
    for prec in ("c128", "mixed"):
        g = _gpu(s, prec, flags)
        rho_host = tdks.density(g["psi"], s.kw, grid)
        assert rel_l2(g["rho"], rho_host) < (1e-13 if prec == "c128" else 1e-7)
        assert abs(g["c1"] - mgga.tb09_c(rho_host, grid)) < (1e-10 if prec == "c128" else 1e-7)


def test_mixed_path_tb09():
    s = _pulse_system("tb09")
    g = _gpu(s, "mixed")
    o = _oracle(s)
    n = s.A.shape[0] - 1
    assert rel_l2(g["rho"], o["rho"]) < 2e-6 * np.sqrt(n)
    assert abs(g["c1"] - o["c1"]) < 1e-6
    assert max_rel_series(g["J"], o["J"]) < 1e-5


def test_isolated_length_gauge_bj():
    A = synth.cos2_pulse_table(6, 0.02, 0.02, 0.6, 0.12, 0.0, [0.0, 0.0, 1.0])
    s = tiny_isolated(n=12, nsteps=6, A=A, seed=7702)
    s.xc = "bj"
    g = _gpu(s, "c128")
    o = _oracle(s)
    assert rel_l2(g["rho"], o["rho"]) < 1e-10
    assert np.max(np.abs(g["psi"] - o["psi"])) < 1e-10


@pytest.mark.parametrize("flags", PATHS)
def test_predictor_corrector_tb09(flags):
    s = _pulse_system("tb09", nsteps=5)
    g = _gpu(s, "c128", flags | PC)
    o = _oracle(s, pc=True)
    assert rel_l2(g["rho"], o["rho"]) < 1e-10
    assert np.max(np.abs(g["psi"] - o["psi"])) < 1e-10
    assert abs(g["c1"] - o["c1"]) < 1e-12


def test_ground_state_tb09():
    from paper_1804_01404_amd.binding import TDDFT
    s = tiny_periodic(n=12, L=6.0, n_orb=4, kpts=np.array([[0.0, 0.0, 0.0], [0.2, 0.1, -0.1]]), seed=7703)
    s.xc = "tb09"
    announce("mgga ground state tb09")
    with TDDFT(s, precision="c128") as t:
        t.set_potential()
        E = t.ground_state(15, 0.02)
        psi = t.orbitals()
        c = t.xc_parameter()
    o = tdks.TDKS.from_system(s)
    Eo = o.ground_state(15, 0.02)
    assert np.max(np.abs(E - Eo)) < 1e-10 * np.max(np.abs(Eo))
    assert np.max(np.abs(psi - o.psi)) < 1e-9
    assert abs(c - o.mgga_c) < 1e-12


def test_batch_of_tb09_cells_equals_solo_runs():
    from paper_1804_01404_amd.binding import TDDFT, TDDFTBatch
    cells = []
    for i, xc in enumerate(["tb09", "tb09", "bj"]):
        s = _pulse_system(xc, nsteps=4)
        s.psi0 = s.psi0 * np.exp(0.3j * i)
        cells.append(s)
    announce("mgga batch vs solo")
    with TDDFTBatch(cells, precision="mixed") as b:
        Jb = b.propagate([c.A for c in cells])
    for s, J in zip(cells, Jb):
        with TDDFT(s, precision="mixed") as t:
            t.set_potential()
            Js = t.propagate(s.A)
        assert np.array_equal(J, Js)
