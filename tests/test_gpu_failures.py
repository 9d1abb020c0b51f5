"""Failure handling through the C ABI, forced from the host so that every
kernel exits normally:

* ENOMEM: the caller's allocator returns NULL at the k-th request; init
  fails cleanly, frees everything it had taken, and a later init works;
* ENUMERIC: NaN orbitals installed with tddft_set_orbitals poison the context
  at the next propagate (fused and per-stage paths); afterwards only
  last_error and free work;
* the norm watchdog (TDDFT_FLAG_NORM_WATCHDOG) stops a run whose step is
  outside the Taylor stability bound (allowed with ALLOW_UNSTABLE) as soon as
  a norm leaves 1 by 1e-3, while the same run without the watchdog goes on.
"""
import ctypes as C

import numpy as np
import pytest

import synth
from gpu_helpers import announce
from oracle_helpers import tiny_periodic

pytestmark = pytest.mark.gpu
STREAMING = 8


@pytest.mark.parametrize("fail_at", [0, 1, 5, 17])
def test_enomem_from_the_allocator_callback(fail_at):
    import torch
    from paper_1804_01404_amd import binding
    lib = binding.load_library()
    s = tiny_periodic(n=12, nsteps=1)
    announce(f"ENOMEM at allocation {fail_at}")
    dev = torch.cuda.current_device()
    stream = torch.cuda.Stream(device=dev)
    live = {}
    calls = [0]

    def alloc(nbytes, _u):
        calls[0] += 1
        if calls[0] - 1 == fail_at:
            return None
        p = int(torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream.cuda_stream))
        live[p] = nbytes
        return p

    def free(ptr, _u):
        assert int(ptr) in live
        del live[int(ptr)]
        torch.cuda.caching_allocator_delete(int(ptr))
    a_cb, f_cb = binding.ALLOC_FN(alloc), binding.FREE_FN(free)
    cfg, keep = binding._config_for(s, "c128", 0)
    cfg.stream = C.c_void_p(stream.cuda_stream)
    cfg.dev_alloc = a_cb
    cfg.dev_free = f_cb
    psi = np.ascontiguousarray(s.psi0, dtype=np.complex128)
    h = C.c_void_p()
    st = lib.tddft_init(C.byref(cfg), psi.ctypes.data_as(C.POINTER(C.c_double)), C.byref(h))
    assert st == binding.ENOMEM
    assert not h.value
    assert not live                      # everything taken before the failure was given back
    # the same configuration with a working allocator
    with binding.TDDFT(s) as t:
        t.set_potential()
        assert np.all(np.isfinite(t.propagate(s.A)))


@pytest.mark.parametrize("flags", [0, STREAMING])
def test_nan_orbitals_poison_the_context(flags):
    from paper_1804_01404_amd import binding
    s = tiny_periodic(n=12, nsteps=3)
    announce(f"ENUMERIC from NaN orbitals flags={flags}")
    with binding.TDDFT(s, flags=flags) as t:
        t.set_potential()
        psi = s.psi0.copy()
        psi[0, 1, 3, 4, 5] = np.nan
        t.set_orbitals(psi)
        with pytest.raises(binding.TDDFTError) as e:
            t.propagate(s.A)
        assert e.value.status == binding.ENUMERIC
        for call in (lambda: t.propagate(s.A), t.energy, t.orbitals, t.density_current):
            with pytest.raises(binding.TDDFTError) as e:
                call()
            assert e.value.status == binding.ESTATE
            assert "poisoned" in str(e.value)


def test_nan_cell_poisons_a_batch():
    """A NaN orbital in one cell of a batch: the batch's propagate (which takes
    every cell's NaN flag back with one copy) returns ENUMERIC naming that
    cell, and the poisoned batch refuses further steps."""
    from paper_1804_01404_amd import binding
    cells = synth.batch_cells(cells=range(3), nsteps=3, max_orb=8, max_k=2, grids=(12, 16), precision="mixed")
    psi = cells[1].psi0.copy()
    psi.reshape(-1)[7] = np.nan
    cells[1].psi0 = psi
    announce("ENUMERIC from a NaN cell in a batch")
    with binding.TDDFTBatch(cells, precision="mixed") as b:
        with pytest.raises(binding.TDDFTError) as e:
            b.propagate([c.A for c in cells])
        assert e.value.status == binding.ENUMERIC
        assert "cell 1" in str(e.value)
        with pytest.raises(binding.TDDFTError) as e:
            b.propagate([c.A for c in cells])
        assert e.value.status == binding.ESTATE


def test_norm_watchdog_stops_an_unstable_run():
    from paper_1804_01404_amd import binding
    # 20^3 cell at dt = 0.08: |lambda| dt = 2.97 > 2 sqrt 2, the top modes grow
    s = synth.single_cell_config(1, nk=1, n_orb=4, nsteps=400, dt=0.08, precision="c128")
    announce("norm watchdog, 20^3 at dt 0.08")
    flags = binding.FLAG_ALLOW_UNSTABLE | binding.FLAG_NO_GRAPH
    with binding.TDDFT(s, precision="c128", flags=flags) as t:
        t.set_potential()
        J = t.propagate(s.A[:21])                    # 20 steps: no watchdog, still finite
        assert np.all(np.isfinite(J))
    with binding.TDDFT(s, precision="c128", flags=flags | binding.FLAG_NORM_WATCHDOG) as t:
        t.set_potential()
        tripped = None
        for n in range(0, 400, 20):
            try:
                t.propagate(s.A[n:n + 21])
            except binding.TDDFTError as e:
                tripped = (n, e)
                break
        assert tripped is not None, "the watchdog never tripped"
        assert tripped[1].status == binding.ENUMERIC and "watchdog" in str(tripped[1])
    # a stable run with the watchdog on is unaffected
    s2 = synth.single_cell_config(1, nk=1, n_orb=4, nsteps=40, dt=0.04, precision="c128")
    with binding.TDDFT(s2, precision="c128", flags=binding.FLAG_NORM_WATCHDOG) as t:
        t.set_potential()
        assert np.all(np.isfinite(t.propagate(s2.A)))
