"""The per-stage tuner (tddft_report): every decomposition it may choose gives
the same bits, its choice is kept per shape for the process and in the JSON
file named by TDDFT_TUNE_CACHE, and a plan in that file is taken as given.

Forced plans run in child processes (one at a time; the file is read once per
process)."""
import hashlib
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import synth
from gpu_helpers import announce
from oracle_helpers import tiny_isolated, tiny_periodic

pytestmark = pytest.mark.gpu
STREAMING, NO_TUNE = 8, 16
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(s, flags, prec="mixed"):
    from paper_1804_01404_amd.binding import TDDFT
    with TDDFT(s, precision=prec, flags=flags) as t:
        t.set_potential()
        rep = t.report()
        J = t.propagate(s.A)
        rho, _ = t.density_current()
        psi = t.orbitals()
    return rep, J, rho, psi


def _systems():
    A = synth.cos2_pulse_table(6, 0.02, 0.02, 0.6, 0.12, 0.0, [0.3, 0.2, 1.0])
    iso = tiny_isolated(n=40, h=0.45, n_orb=6, nsteps=6, A=A, seed=4041)
    per = tiny_periodic(n=20, L=10.26, n_orb=5, kpts=[[0.1, 0.0, 0.2], [-0.2, 0.1, 0.0]], nsteps=6,
                        A=synth.kick_table(6, [0.137, 0.0, 0.0]), seed=4042)
    return {"isolated40": iso, "periodic20": per}


@pytest.mark.parametrize("name", ["isolated40", "periodic20"])
@pytest.mark.parametrize("prec", ["mixed", "c128"])
def test_tuned_decomposition_gives_the_default_bits(name, prec):
    s = _systems()[name]
    announce(f"tuner {name} {prec}")
    rep_t, J_t, rho_t, psi_t = _run(s, STREAMING, prec)
    rep_d, J_d, rho_d, psi_d = _run(s, STREAMING | NO_TUNE, prec)
    assert rep_t["source"] in ("tuned", "cache") and rep_d["source"] == "default"
    if rep_t["source"] == "tuned":
        assert len(rep_t["candidates"]) >= 2
    announce(f"  chosen {rep_t['stage']}")
    assert np.array_equal(psi_t, psi_d)
    assert np.array_equal(rho_t, rho_d)
    assert np.array_equal(J_t, J_d)
    # a second context of the same shape reuses the choice
    rep2, _, _, _ = _run(s, STREAMING, prec)
    assert rep2["source"] == "cache" and rep2["stage"] == rep_t["stage"]


_CHILD = r"""
import hashlib, json, sys
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
import numpy as np, torch
torch.cuda.set_device(0)
from test_gpu_tuner import _systems, _run
s = _systems()[{name!r}]
rep, J, rho, psi = _run(s, 8)
print(json.dumps({{"report": {{k: rep[k] for k in ("key", "source", "stage")}},
                  "sha": hashlib.sha256(psi.tobytes() + J.tobytes() + rho.tobytes()).hexdigest()}}))
"""


def _child(name, cache):
    env = dict(os.environ, TDDFT_TUNE_CACHE=str(cache))
    code = _CHILD.format(root=ROOT, tests=os.path.join(ROOT, "tests"), name=name)
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


@pytest.mark.parametrize("name", ["isolated40", "periodic20"])
def test_cache_file_is_written_read_and_obeyed(name, tmp_path):
    cache = tmp_path / "tune.json"
    announce(f"tuner cache file {name}: tune")
    first = _child(name, cache)
    assert first["report"]["source"] == "tuned"
    text = cache.read_text()
    key = first["report"]["key"]
    assert key in text and json.loads(text)[key]["TX"] == first["report"]["stage"]["TX"]
    announce(f"tuner cache file {name}: reuse")
    second = _child(name, cache)
    assert second["report"]["source"] == "cache" and second["sha"] == first["sha"]
    # forced plans: each one that fits runs as given and gives the same bits
    iso = name.startswith("isolated")
    plans = ([(2, 40, 8, 1, 0), (2, 8, 40, 2, 1), (2, 20, 20, 4, 1), (2, 40, 20, 1, 1)] if iso else
             [(0, 20, 20, 1, 0), (1, 20, 10, 1, 1), (1, 10, 20, 2, 0), (1, 20, 20, 4, 1)])
    for bc, tx, ty, zs, xm in plans:
        cache.write_text(json.dumps({key: {"bc": bc, "TX": tx, "TY": ty, "zs": zs, "xmap": xm, "ms": 0.0}}))
        announce(f"tuner cache file {name}: forced {(bc, tx, ty, zs, xm)}")
        got = _child(name, cache)
        st = got["report"]["stage"]
        assert got["report"]["source"] == "cache"
        assert (st["bc"], st["TX"], st["TY"], st["zs"], st["xmap"]) == (bc, tx, ty, zs, xm)
        assert got["sha"] == first["sha"]
