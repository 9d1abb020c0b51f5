"""The allocation-free conductivity (for callers that cannot allocate) gives
the same bits as the allocating entry point, on two calls in a row, the
second smaller, through the C ABI with device arrays from torch."""
import ctypes as C

import numpy as np
import pytest

from gpu_helpers import announce

pytestmark = pytest.mark.gpu


def _noalloc(lib, I_dev, dt, A0, om_dev, flags, sig_dev, eps_dev, stream):
    fn = lib.tddft_conductivity_noalloc
    fn.argtypes = [C.c_int32, C.c_void_p, C.c_double, C.c_double, C.c_int32, C.c_void_p, C.c_uint32,
                   C.c_void_p, C.c_void_p, C.c_void_p]
    fn.restype = C.c_int
    return fn(I_dev.shape[0], I_dev.data_ptr(), dt, A0, om_dev.shape[0], om_dev.data_ptr(), flags,
              sig_dev.data_ptr(), eps_dev.data_ptr() if eps_dev is not None else None, stream)


def test_noalloc_conductivity_equals_allocating_entry_point():
    import torch
    from paper_1804_01404_amd import binding
    lib = binding.load_library()
    dev = torch.device("cuda", 0)
    stream = torch.cuda.Stream(device=dev)
    rng = np.random.default_rng(21)
    for n_t, n_w, flags in ((30001, 700, binding.SPECTRUM_SUBTRACT_MEAN), (999, 37, 0)):
        announce(f"conductivity_noalloc n_t={n_t} n_w={n_w} flags={flags}")
        t = np.arange(n_t) * 0.04
        I = 1e-4 * np.exp(-0.003 * t) * np.cos(0.5 * t) + 1e-6 * rng.standard_normal(n_t) + 2e-5
        om = np.linspace(0.02, 3.0, n_w)
        ref, eref = binding.conductivity(I, 0.04, 0.2, om, mask=not (flags & binding.SPECTRUM_NO_MASK),
                                         subtract_mean=bool(flags & binding.SPECTRUM_SUBTRACT_MEAN),
                                         dielectric=True)
        I_d = torch.tensor(I, dtype=torch.float64, device=dev)
        om_d = torch.tensor(om, dtype=torch.float64, device=dev)
        sig_d = torch.full((n_w, 2), float("nan"), dtype=torch.float64, device=dev)
        eps_d = torch.full((n_w, 2), float("nan"), dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        st = _noalloc(lib, I_d, 0.04, 0.2, om_d, flags, sig_d, eps_d, C.c_void_p(stream.cuda_stream))
        assert st == binding.OK, lib.tddft_last_error(None)
        stream.synchronize()
        sig = sig_d.cpu().numpy()
        eps = eps_d.cpu().numpy()
        assert np.array_equal(sig[:, 0] + 1j * sig[:, 1], ref)
        assert np.array_equal(eps[:, 0] + 1j * eps[:, 1], eref)


def test_noalloc_rejects_sizes_beyond_the_workspace():
    import torch
    from paper_1804_01404_amd import binding
    lib = binding.load_library()
    dev = torch.device("cuda", 0)
    I_d = torch.zeros(20000, dtype=torch.float64, device=dev)
    om_d = torch.zeros(9000, dtype=torch.float64, device=dev)
    sig_d = torch.zeros((9000, 2), dtype=torch.float64, device=dev)
    st = _noalloc(lib, I_d, 0.04, 0.2, om_d, 0, sig_d, None, None)
    assert st == binding.EINVAL
    assert b"workspace" in lib.tddft_last_error(None)
