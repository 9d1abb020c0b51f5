"""GPU checks of uneven batches: every cell of a batch equals its own solo
run bit for bit (the persistent fused kernel computes each (cell, orbital)
item exactly as the one-orbital-per-workgroup kernel; 24^3 cells take the
per-stage kernels in both), the tuner's steps change nothing, and cells agree
with the FP64 oracle."""
import numpy as np
import pytest

import synth
from gpu_helpers import announce, gpu_run, oracle_run, rel_l2, max_rel_series

pytestmark = pytest.mark.gpu


def _cells(precision):
    cells = synth.batch_cells(cells=range(7), nsteps=7, max_orb=12, max_k=3,
                              grids=(12, 16, 20, 24), precision=precision)
    return cells


@pytest.mark.parametrize("prec", ["c128", "mixed"])
def test_batch_cells_equal_solo_runs(prec):
    from paper_1804_01404_amd.binding import TDDFTBatch
    cells = _cells(prec)
    announce(f"batch of {len(cells)} cells, grids {[c.n[0] for c in cells]}, {prec}")
    with TDDFTBatch(cells, precision=prec) as b:
        Js = b.propagate([c.A for c in cells])
        psis = [b.orbitals(i) for i in range(len(cells))]
        rep = b.report()
    announce(f"batch plan {rep}")
    assert sum(g["cells"] for g in rep["groups"]) + len(rep["per_stage_cells"]) == len(cells)
    for i, c in enumerate(cells):
        solo = gpu_run(c, precision=prec)
        assert np.array_equal(Js[i], solo["J"]), i
        assert np.array_equal(psis[i], solo["psi"]), i


@pytest.mark.parametrize("switches", ["same", "mixed"])
def test_one_grid_batch_equals_solo_runs(switches):
    """Cells of one grid size form one persistent group. With the same Hartree
    and xc switches the group runs the ends of its step as one launch per
    kernel (some cells with several density chunks); with one cell without
    Hartree and one without xc every cell keeps its own. Either way each cell
    equals its solo run bit for bit."""
    from paper_1804_01404_amd.binding import TDDFTBatch
    cells = synth.batch_cells(cells=range(4), nsteps=5, max_orb=24, max_k=8, grids=(16,), precision="mixed")
    if switches == "mixed":
        cells[1].hartree = False
        cells[2].xc = False
    announce(f"one-grid batch, {switches} switches, orbitals x k {[c.n_orb * len(c.kw) for c in cells]}")
    with TDDFTBatch(cells, precision="mixed") as b:
        Js = b.propagate([c.A for c in cells])
        psis = [b.orbitals(i) for i in range(len(cells))]
        rep = b.report()
    assert len(rep["groups"]) == 1
    assert rep["groups"][0]["grouped_tail"] == (switches == "same")
    for i, c in enumerate(cells):
        solo = gpu_run(c, precision="mixed")
        assert np.array_equal(Js[i], solo["J"]), i
        assert np.array_equal(psis[i], solo["psi"]), i


def test_batch_cells_match_oracle():
    from paper_1804_01404_amd.binding import TDDFTBatch
    cells = _cells("c128")[:3]
    announce("batch vs oracle")
    with TDDFTBatch(cells, precision="c128") as b:
        Js = b.propagate([c.A for c in cells])
        psis = [b.orbitals(i) for i in range(len(cells))]
    for i, c in enumerate(cells):
        o = oracle_run(c)
        assert rel_l2(psis[i], o["psi"]) < 1e-10, i
        assert max_rel_series(Js[i], o["J"]) < 1e-8, i


def test_batch_second_propagate_reuses_graph():
    """Two propagate calls (tuning then graph replay) continue the same run."""
    from paper_1804_01404_amd.binding import TDDFTBatch
    cells = _cells("mixed")[:4]
    for c in cells:
        c.A = c.A  # 7 steps
    announce("batch two calls")
    with TDDFTBatch(cells, precision="mixed") as b:
        J1 = b.propagate([c.A[:4] for c in cells])
        J2 = b.propagate([c.A[3:] for c in cells])
        psi_a = [b.orbitals(i) for i in range(len(cells))]
    with TDDFTBatch(cells, precision="mixed") as b:
        J = b.propagate([c.A for c in cells])
        psi_b = [b.orbitals(i) for i in range(len(cells))]
    for i in range(len(cells)):
        assert np.array_equal(np.concatenate([J1[i], J2[i]]), J[i])
        assert np.array_equal(psi_a[i], psi_b[i])


def test_mixed_batch_with_32_cubed_cells_matches_oracle():
    """A complex FP32 batch whose cells include two 32^3 cells (per-stage
    lanes with the tuned decomposition) beside 16^3 and 20^3 cells (persistent
    fused groups), each with its own k-points, atoms and pulse, against the
    oracle: orbitals and density within 2e-6 sqrt(n), current within 1e-4 of
    its maximum (these cells start from random orbitals at random k-points
    under weak pulses, so the current is a small difference of the momentum
    and kappa-norm terms, each rounded at the FP32 level)."""
    from paper_1804_01404_amd.binding import TDDFTBatch
    n = 6
    cells = synth.batch_cells(cells=[0, 1, 2, 3], nsteps=n, max_orb=8, max_k=2, grids=(32,), precision="mixed")
    cells[1] = synth.batch_cells(cells=[1], nsteps=n, max_orb=8, max_k=2, grids=(16,), precision="mixed")[0]
    cells[3] = synth.batch_cells(cells=[3], nsteps=n, max_orb=8, max_k=2, grids=(20,), precision="mixed")[0]
    announce(f"mixed batch with 32^3 cells, grids {[c.n[0] for c in cells]}")
    with TDDFTBatch(cells, precision="mixed") as b:
        Js = b.propagate([c.A for c in cells])
        psis = [b.orbitals(i) for i in range(len(cells))]
        rhos = [b.density(i) for i in range(len(cells))]
        rep = b.report()
    assert sorted(rep["per_stage_cells"]) == [0, 2]
    assert len(rep["per_stage_tiles"]) >= 1
    for i, c in enumerate(cells):
        o = oracle_run(c)
        assert rel_l2(psis[i], o["psi"]) < 2e-6 * np.sqrt(n), i
        assert rel_l2(rhos[i], o["rho"]) < 2e-6 * np.sqrt(n), i
        err = max_rel_series(Js[i], o["J"])
        announce(f"  cell {i} ({c.n[0]}^3) current error {err:.3e}")
        assert err < 1e-4, i
