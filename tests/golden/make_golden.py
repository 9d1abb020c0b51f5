"""Write the stored oracle trajectory used as a regression guard.

Calls only ``synth`` (inputs) and ``oracle`` (the CPU reference); no value
here comes from the GPU library. Run from the repository root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import tdks  # noqa: E402

NSTEPS = 20


def trajectory():
    s = synth.single_cell_config(0, nsteps=NSTEPS)
    o = tdks.TDKS.from_system(s)
    J = o.propagate(s.A)
    return {
        "workload": "diamond-16^3-gamma, first %d steps, dt 0.02, x kick |A0|/c = 1e-3" % NSTEPS,
        "J": J.tolist(),
        "energy_end": o.energy(),
        "rho_sum_end": float(o.grid.dV * o.rho.sum()),
    }


if __name__ == "__main__":
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_diamond16_20steps.json")
    with open(out, "w") as f:
        json.dump(trajectory(), f, indent=1)
    print("wrote", out)
