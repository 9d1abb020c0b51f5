"""CPU oracle of the real-time TDKS time step — TEST INFRASTRUCTURE ONLY.

Plain FP64 NumPy, written from the paper's equations. Only ``tests/``,
``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg may
import it. The HIP library never calls it and it never calls the library.
"""
from . import tdks  # noqa: F401
