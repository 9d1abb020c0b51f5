"""Seeded synthetic inputs for the real-time TDKS time step.

This package only *describes* systems: grids, k-point sets, atom positions,
synthetic Gaussian pseudopotential parameters sampled onto the grid, initial
orbitals and vector-potential tables. It holds none of the propagation
arithmetic (no finite-difference operator, no Taylor series, no density,
current, Hartree or exchange-correlation evaluation). Both the CPU oracle and
the GPU library consume what it produces, so the two sides start from the same
bytes.

Every random number is drawn from ``numpy.random.Generator(PCG64)`` seeded by
``numpy.random.SeedSequence([1804, 1404, index])``.
"""
from .systems import (  # noqa: F401
    C_AU,
    System,
    AtomProjector,
    mp_kgrid,
    diamond_positions,
    grid_coords,
    gaussian_vloc,
    build_projectors,
    random_orbitals,
    kick_table,
    cos2_pulse_table,
    gauss_pulse_table,
    build_system,
)
from .configs import (  # noqa: F401
    single_cell_config,
    batch_cells,
    multiscale_cell,
    surrogate_init,
    random_pulse_tables,
    random_field_tables,
    cos2_pulse_potential,
    incident_table,
    CONFIG_NAMES,
)
