"""ctypes binding of libtddft.so (argument marshalling only).

Every computation runs in the library's HIP kernels. PyTorch supplies the
device memory (its caching allocator, through the allocator callbacks of
``tddft_config``) and the stream; nothing here falls back to a CPU path: if
the library is not built, loading fails with an error.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtddft.so")

ABI_VERSION = 1
OK, EINVAL, ENOMEM, EDEVICE, EUNSTABLE, ESTATE, ENUMERIC = range(7)
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "EUNSTABLE", 5: "ESTATE",
                6: "ENUMERIC"}
PERIODIC, ISOLATED = 0, 1
C128, MIXED = 0, 1
VELOCITY, LENGTH = 0, 1
XC_NONE, XC_PZ81, XC_TB09, XC_BJ = 0, 1, 2, 3
_XC_CODES = {None: XC_NONE, False: XC_NONE, True: XC_PZ81, "lda": XC_PZ81, "tb09": XC_TB09, "bj": XC_BJ}


def xc_code(xc) -> int:
    """Library code of a system's xc choice: False/None, True or "lda", "tb09", "bj"."""
    try:
        return _XC_CODES[xc]
    except (KeyError, TypeError):
        raise ValueError(f"unknown xc choice {xc!r}") from None

FLAG_ALLOW_UNSTABLE, FLAG_DEBUG_SYNC, FLAG_NO_GRAPH, FLAG_STREAMING, FLAG_NO_TUNE = 1, 2, 4, 8, 16
FLAG_PREDICTOR_CORRECTOR, FLAG_NORM_WATCHDOG = 32, 64

EXPORTED = ["tddft_abi_version", "tddft_init", "tddft_set_potential", "tddft_propagate",
            "tddft_density_current", "tddft_get_orbitals", "tddft_set_orbitals", "tddft_energy",
            "tddft_norms", "tddft_xc_parameter", "tddft_dipole", "tddft_kick", "tddft_ground_state",
            "tddft_set_reference",
            "tddft_excited_electrons", "tddft_last_timing", "tddft_time_kernel",
            "tddft_last_error", "tddft_free", "tddft_batch_create", "tddft_batch_set_potential",
            "tddft_batch_propagate", "tddft_batch_cell", "tddft_batch_last_timing", "tddft_batch_report",
            "tddft_batch_last_error", "tddft_batch_free", "tddft_nn_num_params", "tddft_nn_create",
            "tddft_nn_get_params", "tddft_nn_set_params", "tddft_nn_forward", "tddft_nn_loss_grad",
            "tddft_nn_adam_step", "tddft_nn_train", "tddft_nn_last_error", "tddft_nn_free",
            "tddft_ms_create", "tddft_ms_attach_surrogate", "tddft_ms_step", "tddft_ms_status",
            "tddft_ms_last_error", "tddft_ms_free", "tddft_excitation_energy", "tddft_conductivity",
            "tddft_oscillator_strength", "tddft_work", "tddft_conductivity_noalloc", "tddft_report",
            "tddft_nn_train_ex", "tddft_nn_fit_linear", "tddft_ms_energy"]
KERNEL_STAGE, KERNEL_PROJECT, KERNEL_OBSERVE, KERNEL_DENSITY, KERNEL_FUSED = 0, 1, 2, 3, 4

ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)
_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class Config(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("struct_size", C.c_uint32), ("n", C.c_int32 * 3),
                ("cell", C.c_double * 3), ("boundary", C.c_int32), ("n_orb", C.c_int32),
                ("n_k", C.c_int32), ("kpt", _dp), ("kw", _dp), ("dt", C.c_double),
                ("precision", C.c_int32), ("hartree", C.c_int32), ("xc", C.c_int32),
                ("gauge", C.c_int32), ("flags", C.c_uint32), ("stream", C.c_void_p),
                ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN), ("alloc_user", C.c_void_p)]


class Atom(C.Structure):
    _fields_ = [("npts", C.c_int32), ("n_proj", C.c_int32), ("idx", _ip), ("x", _dp),
                ("beta", _dp), ("e_kb", _dp)]


class NNConfig(C.Structure):
    _fields_ = [("window", C.c_int32), ("hidden", C.c_int32), ("a_scale", C.c_double),
                ("j_scale", C.c_double), ("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float)]


class MSConfig(C.Structure):
    _fields_ = [("n_x", C.c_int32), ("x0", C.c_int32), ("n_mat", C.c_int32), ("dx", C.c_double),
                ("dt", C.c_double), ("n_sub", C.c_int32), ("axis", C.c_int32)]


class TDDFTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libtddft.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run python -m paper_1804_01404_amd.build)")
    # One HIP runtime per process: torch carries its own libamdhip64, so it is
    # brought up first and the library's libamdhip64.so.7 dependency then
    # resolves to the copy already loaded (same soname).
    import torch
    if torch.cuda.is_available():
        torch.cuda.init()
    lib = C.CDLL(path)
    lib.tddft_abi_version.restype = C.c_uint32
    lib.tddft_init.argtypes = [C.POINTER(Config), _dp, C.POINTER(C.c_void_p)]
    lib.tddft_set_potential.argtypes = [C.c_void_p, _dp, C.c_int32, C.POINTER(Atom)]
    lib.tddft_propagate.argtypes = [C.c_void_p, C.c_int32, _dp, _dp]
    lib.tddft_density_current.argtypes = [C.c_void_p, _dp, _dp]
    lib.tddft_get_orbitals.argtypes = [C.c_void_p, _dp]
    lib.tddft_set_orbitals.argtypes = [C.c_void_p, _dp]
    lib.tddft_energy.argtypes = [C.c_void_p, _dp]
    lib.tddft_norms.argtypes = [C.c_void_p, _dp]
    lib.tddft_xc_parameter.argtypes = [C.c_void_p, _dp]
    lib.tddft_dipole.argtypes = [C.c_void_p, _dp]
    lib.tddft_kick.argtypes = [C.c_void_p, C.c_double, C.c_int32]
    lib.tddft_ground_state.argtypes = [C.c_void_p, C.c_int32, C.c_double, _dp]
    lib.tddft_set_reference.argtypes = [C.c_void_p]
    lib.tddft_excited_electrons.argtypes = [C.c_void_p, _dp]
    lib.tddft_last_timing.argtypes = [C.c_void_p, _dp]
    lib.tddft_time_kernel.argtypes = [C.c_void_p, C.c_int32, C.c_int32, _dp]
    lib.tddft_last_error.argtypes = [C.c_void_p]
    lib.tddft_last_error.restype = C.c_char_p
    lib.tddft_free.argtypes = [C.c_void_p]
    lib.tddft_free.restype = None
    for name in ("tddft_init", "tddft_set_potential", "tddft_propagate", "tddft_density_current",
                 "tddft_get_orbitals", "tddft_set_orbitals", "tddft_energy", "tddft_norms", "tddft_xc_parameter",
                 "tddft_dipole", "tddft_kick", "tddft_last_timing", "tddft_time_kernel"):
        getattr(lib, name).restype = C.c_int
    lib.tddft_batch_create.argtypes = [C.c_int32, C.POINTER(Config), C.POINTER(_dp), C.POINTER(C.c_void_p)]
    lib.tddft_batch_set_potential.argtypes = [C.c_void_p, C.c_int32, _dp, C.c_int32, C.POINTER(Atom)]
    lib.tddft_batch_propagate.argtypes = [C.c_void_p, C.c_int32, C.POINTER(_dp), C.POINTER(_dp)]
    lib.tddft_batch_cell.argtypes = [C.c_void_p, C.c_int32]
    lib.tddft_batch_cell.restype = C.c_void_p
    lib.tddft_batch_last_timing.argtypes = [C.c_void_p, _dp]
    lib.tddft_batch_report.argtypes = [C.c_void_p, C.c_char_p, C.c_size_t]
    lib.tddft_batch_last_error.argtypes = [C.c_void_p]
    lib.tddft_batch_last_error.restype = C.c_char_p
    lib.tddft_batch_free.argtypes = [C.c_void_p]
    lib.tddft_batch_free.restype = None
    for name in ("tddft_batch_create", "tddft_batch_set_potential", "tddft_batch_propagate",
                 "tddft_batch_last_timing", "tddft_batch_report"):
        getattr(lib, name).restype = C.c_int
    # learned surrogate and multiscale
    _fp = C.POINTER(C.c_float)
    lib.tddft_nn_num_params.argtypes = [C.c_int32, C.c_int32]
    lib.tddft_nn_num_params.restype = C.c_int64
    lib.tddft_nn_create.argtypes = [C.POINTER(NNConfig), _fp, C.POINTER(C.c_void_p)]
    lib.tddft_nn_get_params.argtypes = [C.c_void_p, _fp]
    lib.tddft_nn_set_params.argtypes = [C.c_void_p, _fp]
    lib.tddft_nn_forward.argtypes = [C.c_void_p, C.c_int32, _fp, _fp]
    lib.tddft_nn_loss_grad.argtypes = [C.c_void_p, C.c_int32, _fp, _fp, _fp, _fp]
    lib.tddft_nn_adam_step.argtypes = [C.c_void_p]
    lib.tddft_nn_train.argtypes = [C.c_void_p, C.c_int32, C.c_int32, _dp, _dp, C.c_int32, C.c_int32,
                                   C.c_uint64, _fp]
    lib.tddft_nn_train_ex.argtypes = [C.c_void_p, C.c_int32, C.c_int32, _dp, _dp, C.c_int32, C.c_int32,
                                      C.c_uint64, C.c_uint32, _fp]
    lib.tddft_nn_train_ex.restype = C.c_int
    lib.tddft_nn_fit_linear.argtypes = [C.c_void_p, C.c_int32, C.c_int32, _dp, _dp, C.c_double, C.c_double]
    lib.tddft_nn_fit_linear.restype = C.c_int
    lib.tddft_nn_last_error.argtypes = [C.c_void_p]
    lib.tddft_nn_last_error.restype = C.c_char_p
    lib.tddft_nn_free.argtypes = [C.c_void_p]
    lib.tddft_nn_free.restype = None
    lib.tddft_ms_create.argtypes = [C.POINTER(MSConfig), C.POINTER(Config), _dp, _dp, C.c_int32,
                                    C.POINTER(Atom), C.POINTER(C.c_void_p)]
    lib.tddft_ms_attach_surrogate.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_int32,
                                              C.POINTER(C.c_int32), C.c_int32, C.c_double]
    lib.tddft_ms_step.argtypes = [C.c_void_p, C.c_int32, _dp, _dp, _dp]
    lib.tddft_ms_status.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_double), C.POINTER(C.c_int32)]
    lib.tddft_ms_energy.argtypes = [C.c_void_p, _dp, _dp]
    lib.tddft_ms_energy.restype = C.c_int
    lib.tddft_ms_last_error.argtypes = [C.c_void_p]
    lib.tddft_ms_last_error.restype = C.c_char_p
    lib.tddft_ms_free.argtypes = [C.c_void_p]
    lib.tddft_ms_free.restype = None
    for name in ("tddft_nn_create", "tddft_nn_get_params", "tddft_nn_set_params", "tddft_nn_forward",
                 "tddft_nn_loss_grad", "tddft_nn_adam_step", "tddft_nn_train", "tddft_ms_create",
                 "tddft_ms_attach_surrogate", "tddft_ms_step", "tddft_ms_status"):
        getattr(lib, name).restype = C.c_int
    # spectra and work (no context)
    lib.tddft_excitation_energy.argtypes = [C.c_void_p, _dp]
    lib.tddft_report.argtypes = [C.c_void_p, C.c_char_p, C.c_size_t]
    lib.tddft_report.restype = C.c_int
    lib.tddft_conductivity.argtypes = [C.c_int32, _dp, C.c_double, C.c_double, C.c_int32, _dp, C.c_uint32,
                                       _dp, _dp]
    lib.tddft_oscillator_strength.argtypes = [C.c_int32, _dp, C.c_double, C.c_double, C.c_int32, _dp, _dp]
    lib.tddft_work.argtypes = [C.c_int32, _dp, _dp, C.c_double, C.c_double, _dp]
    for name in ("tddft_excitation_energy", "tddft_conductivity", "tddft_oscillator_strength", "tddft_work"):
        getattr(lib, name).restype = C.c_int
    if lib.tddft_abi_version() != ABI_VERSION:
        raise RuntimeError("libtddft.so ABI version mismatch")
    _lib = lib
    return lib


def _ptr(a: np.ndarray, ctype=C.c_double):
    return a.ctypes.data_as(C.POINTER(ctype))


class _TorchMemory:
    """Allocator callbacks backed by torch's caching allocator on one stream."""

    def __init__(self, device: int, stream):
        import torch
        self.torch = torch
        self.device = device
        self.stream = stream
        self.alloc_cb = ALLOC_FN(self._alloc)
        self.free_cb = FREE_FN(self._free)

    def _alloc(self, nbytes, _user):
        try:
            return int(self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream))
        except Exception:  # reported to the library as a NULL allocation (ENOMEM)
            return None

    def _free(self, ptr, _user):
        self.torch.cuda.caching_allocator_delete(int(ptr))


class TDDFT:
    """One TDKS cell on the GPU, driven through the C ABI."""

    def __init__(self, system, *, precision: Optional[str] = None, flags: int = 0,
                 torch_memory: bool = True, psi0: Optional[np.ndarray] = None):
        self.lib = load_library()
        s = system
        self.system = s
        prec = precision or s.precision
        self.n = tuple(s.n)
        self.n_orb, self.n_k = s.n_orb, s.n_k
        self._kpt = np.ascontiguousarray(s.kpts, dtype=np.float64)
        self._kw = np.ascontiguousarray(s.kw, dtype=np.float64)
        self._mem = None
        self._stream = None
        cfg = Config()
        cfg.abi_version = ABI_VERSION
        cfg.struct_size = C.sizeof(Config)
        cfg.n[:] = list(s.n)
        cfg.cell[:] = list(s.cell)
        cfg.boundary = PERIODIC if s.boundary == "periodic" else ISOLATED
        cfg.n_orb = s.n_orb
        cfg.n_k = s.n_k
        cfg.kpt = _ptr(self._kpt)
        cfg.kw = _ptr(self._kw)
        cfg.dt = s.dt
        cfg.precision = MIXED if prec == "mixed" else C128
        cfg.hartree = int(bool(s.hartree))
        cfg.xc = xc_code(s.xc)
        cfg.gauge = LENGTH if s.gauge == "length" else VELOCITY
        cfg.flags = flags
        if torch_memory:
            import torch
            dev = torch.cuda.current_device()
            self._stream = torch.cuda.Stream(device=dev)
            self._mem = _TorchMemory(dev, self._stream.cuda_stream)
            cfg.stream = C.c_void_p(self._stream.cuda_stream)
            cfg.dev_alloc = self._mem.alloc_cb
            cfg.dev_free = self._mem.free_cb
        self._cfg = cfg
        psi = np.ascontiguousarray(s.psi0 if psi0 is None else psi0, dtype=np.complex128)
        assert psi.shape == (s.n_k, s.n_orb, s.n[2], s.n[1], s.n[0])
        h = C.c_void_p()
        st = self.lib.tddft_init(C.byref(cfg), _ptr(psi.view(np.float64)), C.byref(h))
        if st != OK:
            raise TDDFTError(st, "tddft_init failed (invalid configuration or device error)")
        self.h = h

    # -----------------------------------------------------------------
    def _check(self, st):
        if st != OK:
            msg = self.lib.tddft_last_error(self.h)
            raise TDDFTError(st, msg.decode() if msg else "")

    def set_potential(self, v_loc=None, projectors=None):
        s = self.system
        v = np.ascontiguousarray(s.v_loc if v_loc is None else v_loc, dtype=np.float64)
        projs = s.projectors if projectors is None else projectors
        keep = []
        atoms = (Atom * max(1, len(projs)))()
        for i, p in enumerate(projs):
            idx = np.ascontiguousarray(p.idx, dtype=np.int32)
            x = np.ascontiguousarray(p.x, dtype=np.float64)
            beta = np.ascontiguousarray(p.beta, dtype=np.float64)
            ekb = np.ascontiguousarray(p.e_kb, dtype=np.float64)
            keep += [idx, x, beta, ekb]
            atoms[i].npts = idx.shape[0]
            atoms[i].n_proj = beta.shape[0]
            atoms[i].idx = _ptr(idx, C.c_int32)
            atoms[i].x = _ptr(x)
            atoms[i].beta = _ptr(beta)
            atoms[i].e_kb = _ptr(ekb)
        self._check(self.lib.tddft_set_potential(self.h, _ptr(v), len(projs),
                                                 atoms if projs else None))
        return self

    def propagate(self, A: np.ndarray) -> np.ndarray:
        A = np.ascontiguousarray(A, dtype=np.float64)
        nsteps = A.shape[0] - 1
        J = np.zeros((max(nsteps, 0), 3))
        self._check(self.lib.tddft_propagate(self.h, nsteps, _ptr(A), _ptr(J)))
        return J

    def density_current(self):
        rho = np.empty((self.n[2], self.n[1], self.n[0]))
        J = np.empty(3)
        self._check(self.lib.tddft_density_current(self.h, _ptr(rho), _ptr(J)))
        return rho, J

    def orbitals(self) -> np.ndarray:
        psi = np.empty((self.n_k, self.n_orb, self.n[2], self.n[1], self.n[0]), dtype=np.complex128)
        self._check(self.lib.tddft_get_orbitals(self.h, _ptr(psi.view(np.float64))))
        return psi

    def set_orbitals(self, psi: np.ndarray):
        psi = np.ascontiguousarray(psi, dtype=np.complex128)
        self._check(self.lib.tddft_set_orbitals(self.h, _ptr(psi.view(np.float64))))

    def energy(self) -> float:
        e = C.c_double()
        self._check(self.lib.tddft_energy(self.h, C.byref(e)))
        return e.value

    def xc_parameter(self) -> float:
        """The BJ / TB09 mixing parameter c of the last potential update."""
        v = C.c_double()
        self._check(self.lib.tddft_xc_parameter(self.h, C.byref(v)))
        return v.value

    def norms(self) -> np.ndarray:
        out = np.empty((self.n_k, self.n_orb))
        self._check(self.lib.tddft_norms(self.h, _ptr(out)))
        return out

    def dipole(self) -> np.ndarray:
        d = np.empty(3)
        self._check(self.lib.tddft_dipole(self.h, _ptr(d)))
        return d

    def ground_state(self, n_iter: int, tau: float, energies: bool = True) -> np.ndarray:
        """Imaginary-time preparation of the initial state; energy per
        iteration (or, with energies=False, none: no host round trip per
        iteration)."""
        E = np.empty(max(int(n_iter), 1))
        self._check(self.lib.tddft_ground_state(self.h, int(n_iter), float(tau), _ptr(E) if energies else None))
        return E[: int(n_iter)] if energies else np.empty(0)

    def set_reference(self):
        """Keep the current orbitals as the reference of excited_electrons."""
        self._check(self.lib.tddft_set_reference(self.h))

    def excited_electrons(self) -> float:
        """Number density of excited electron-hole pairs (bohr^-3)."""
        v = C.c_double()
        self._check(self.lib.tddft_excited_electrons(self.h, C.byref(v)))
        return v.value

    def excitation_energy(self) -> float:
        """E(t) - E(reference) in Ha per cell (LDA; see tddft_work for BJ / TB09)."""
        v = C.c_double()
        self._check(self.lib.tddft_excitation_energy(self.h, C.byref(v)))
        return v.value

    def kick(self, F0: float, axis: int):
        self._check(self.lib.tddft_kick(self.h, float(F0), int(axis)))

    def report(self) -> dict:
        """How the step runs: the fused path, or the tuned per-stage decomposition."""
        import json
        buf = C.create_string_buffer(1 << 16)
        self._check(self.lib.tddft_report(self.h, buf, len(buf)))
        return json.loads(buf.value.decode())

    def last_timing_ms(self) -> float:
        ms = C.c_double()
        self._check(self.lib.tddft_last_timing(self.h, C.byref(ms)))
        return ms.value

    def time_kernel(self, which: int, reps: int = 50) -> float:
        """Mean duration (ms) of one kernel of the step, launched alone
        ``reps`` times on the context's stream between HIP events."""
        ms = C.c_double()
        self._check(self.lib.tddft_time_kernel(self.h, int(which), int(reps), C.byref(ms)))
        return ms.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.tddft_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


SPECTRUM_NO_MASK, SPECTRUM_SUBTRACT_MEAN = 1, 2
NN_COSINE_LR, NN_FREEZE_LINEAR = 1, 2


def _stateless_check(lib, st):
    if st != OK:
        msg = lib.tddft_last_error(None)
        raise TDDFTError(st, msg.decode() if msg else "")


def conductivity(I, dt: float, A0: float, omegas, *, mask: bool = True, subtract_mean: bool = False,
                 dielectric: bool = False):
    """sigma(omega) (complex) of one current component after a kick A0, and
    optionally eps(omega), computed by the library's kernels."""
    lib = load_library()
    I = np.ascontiguousarray(I, dtype=np.float64)
    om = np.ascontiguousarray(omegas, dtype=np.float64)
    sig = np.empty(om.shape[0], dtype=np.complex128)
    eps = np.empty(om.shape[0], dtype=np.complex128) if dielectric else None
    flags = (0 if mask else SPECTRUM_NO_MASK) | (SPECTRUM_SUBTRACT_MEAN if subtract_mean else 0)
    _stateless_check(lib, lib.tddft_conductivity(I.shape[0], _ptr(I), float(dt), float(A0), om.shape[0],
                                                 _ptr(om), flags, _ptr(sig.view(np.float64)),
                                                 _ptr(eps.view(np.float64)) if dielectric else None))
    return (sig, eps) if dielectric else sig


def oscillator_strength(d, dt: float, F0: float, energies):
    """df/dE of one dipole component after a kick F0 (library kernels)."""
    lib = load_library()
    d = np.ascontiguousarray(d, dtype=np.float64)
    E = np.ascontiguousarray(energies, dtype=np.float64)
    out = np.empty(E.shape[0])
    _stateless_check(lib, lib.tddft_oscillator_strength(d.shape[0], _ptr(d), float(dt), float(F0), E.shape[0],
                                                        _ptr(E), _ptr(out)))
    return out


def work(I, A, dt: float, volume: float):
    """W(t_n) of the field on the electrons of one cell (library kernels)."""
    lib = load_library()
    I = np.ascontiguousarray(I, dtype=np.float64)
    A = np.ascontiguousarray(A, dtype=np.float64)
    assert I.shape == A.shape and I.ndim == 2 and I.shape[1] == 3
    W = np.empty(I.shape[0])
    _stateless_check(lib, lib.tddft_work(I.shape[0], _ptr(I), _ptr(A), float(dt), float(volume), _ptr(W)))
    return W


def mfma_layout_check(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Run one v_mfma_f64_16x16x4f64 with the lane layout the projector
    kernel assumes; returns D (16 x 16) for comparison with A @ B."""
    lib = load_library()
    fn = lib.tddft_test_mfma_layout
    fn.argtypes = [_dp, _dp, _dp]
    fn.restype = C.c_int
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    D = np.zeros((16, 16))
    if fn(_ptr(A), _ptr(B), _ptr(D)) != 0:
        raise RuntimeError("mfma layout check failed to run")
    return D


def mfma44_layout_check(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Run one v_mfma_f64_4x4x4f64 (four blocks) with the lane layout the
    stage projection assumes; A, B [4][4][4]; returns D [4][4][4] for
    comparison with A[b] @ B[b]."""
    lib = load_library()
    fn = lib.tddft_test_mfma44_layout
    fn.argtypes = [_dp, _dp, _dp]
    fn.restype = C.c_int
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    D = np.zeros((4, 4, 4))
    if fn(_ptr(A), _ptr(B), _ptr(D)) != 0:
        raise RuntimeError("mfma layout check failed to run")
    return D


def _config_for(system, precision, flags):
    s = system
    cfg = Config()
    cfg.abi_version = ABI_VERSION
    cfg.struct_size = C.sizeof(Config)
    cfg.n[:] = list(s.n)
    cfg.cell[:] = list(s.cell)
    cfg.boundary = PERIODIC if s.boundary == "periodic" else ISOLATED
    cfg.n_orb = s.n_orb
    cfg.n_k = s.n_k
    kpt = np.ascontiguousarray(s.kpts, dtype=np.float64)
    kw = np.ascontiguousarray(s.kw, dtype=np.float64)
    cfg.kpt = _ptr(kpt)
    cfg.kw = _ptr(kw)
    cfg.dt = s.dt
    cfg.precision = MIXED if precision == "mixed" else C128
    cfg.hartree = int(bool(s.hartree))
    cfg.xc = xc_code(s.xc)
    cfg.gauge = LENGTH if s.gauge == "length" else VELOCITY
    cfg.flags = flags
    return cfg, (kpt, kw)


def _atoms_for(projs):
    keep = []
    atoms = (Atom * max(1, len(projs)))()
    for i, p in enumerate(projs):
        idx = np.ascontiguousarray(p.idx, dtype=np.int32)
        x = np.ascontiguousarray(p.x, dtype=np.float64)
        beta = np.ascontiguousarray(p.beta, dtype=np.float64)
        ekb = np.ascontiguousarray(p.e_kb, dtype=np.float64)
        keep += [idx, x, beta, ekb]
        atoms[i].npts = idx.shape[0]
        atoms[i].n_proj = beta.shape[0]
        atoms[i].idx = _ptr(idx, C.c_int32)
        atoms[i].x = _ptr(x)
        atoms[i].beta = _ptr(beta)
        atoms[i].e_kb = _ptr(ekb)
    return atoms, keep


class TDDFTBatch:
    """Many independent cells advanced together (tddft_batch_* entry points).

    Device memory comes from the library's own allocator; the stream is a
    torch stream so that torch work can be ordered against the batch."""

    def __init__(self, systems, *, precision: str = "mixed", flags: int = 0):
        import torch
        self.lib = load_library()
        self.systems = list(systems)
        n = len(self.systems)
        self._stream = torch.cuda.Stream()
        cfgs = (Config * n)()
        keep = []
        psis = []
        for i, s in enumerate(self.systems):
            cfg, k = _config_for(s, precision, flags)
            keep.append(k)
            cfgs[i] = cfg
            psi = np.ascontiguousarray(s.psi0, dtype=np.complex128)
            psis.append(psi)
        cfgs[0].stream = C.c_void_p(self._stream.cuda_stream)
        ptrs = (_dp * n)(*[_ptr(p.view(np.float64)) for p in psis])
        h = C.c_void_p()
        st = self.lib.tddft_batch_create(n, cfgs, ptrs, C.byref(h))
        if st != OK:
            raise TDDFTError(st, "tddft_batch_create failed")
        self.h = h
        for i, s in enumerate(self.systems):
            atoms, kp = _atoms_for(s.projectors)
            v = np.ascontiguousarray(s.v_loc, dtype=np.float64)
            self._check(self.lib.tddft_batch_set_potential(self.h, i, _ptr(v), len(s.projectors),
                                                           atoms if s.projectors else None))

    def _check(self, st):
        if st != OK:
            msg = self.lib.tddft_batch_last_error(self.h)
            raise TDDFTError(st, msg.decode() if msg else "")

    def propagate(self, tables):
        """tables: one A table [nsteps + 1, 3] per cell; returns the J tables."""
        n = len(self.systems)
        tabs = [np.ascontiguousarray(t, dtype=np.float64) for t in tables]
        nsteps = tabs[0].shape[0] - 1
        assert all(t.shape == (nsteps + 1, 3) for t in tabs)
        Js = [np.zeros((nsteps, 3)) for _ in range(n)]
        A = (_dp * n)(*[_ptr(t) for t in tabs])
        Jp = (_dp * n)(*[_ptr(j) for j in Js])
        self._check(self.lib.tddft_batch_propagate(self.h, nsteps, A, Jp))
        return Js

    def orbitals(self, cell):
        s = self.systems[cell]
        c = self.lib.tddft_batch_cell(self.h, cell)
        psi = np.empty((s.n_k, s.n_orb, s.n[2], s.n[1], s.n[0]), dtype=np.complex128)
        st = self.lib.tddft_get_orbitals(c, _ptr(psi.view(np.float64)))
        if st != OK:
            raise TDDFTError(st, self.lib.tddft_last_error(c).decode())
        return psi

    def density(self, cell):
        s = self.systems[cell]
        c = self.lib.tddft_batch_cell(self.h, cell)
        rho = np.empty((s.n[2], s.n[1], s.n[0]))
        st = self.lib.tddft_density_current(c, _ptr(rho), None)
        if st != OK:
            raise TDDFTError(st, self.lib.tddft_last_error(c).decode())
        return rho

    def last_timing_ms(self) -> float:
        ms = C.c_double()
        self._check(self.lib.tddft_batch_last_timing(self.h, C.byref(ms)))
        return ms.value

    def report(self) -> dict:
        import json
        buf = C.create_string_buffer(1 << 16)
        self._check(self.lib.tddft_batch_report(self.h, buf, len(buf)))
        return json.loads(buf.value.decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.tddft_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


# ---------------------------------------------------------------------------
# learned current surrogate and multiscale light propagation


def nn_num_params(window: int, hidden: int) -> int:
    return int(load_library().tddft_nn_num_params(int(window), int(hidden)))


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class Surrogate:
    """The current surrogate (tddft_nn_* entry points): FP32 network on the
    device, trained by the library's forward, backward and Adam kernels."""

    def __init__(self, window, hidden, params, *, a_scale=1.0, j_scale=1.0, lr=1e-3, beta1=0.9,
                 beta2=0.999, eps=1e-8):
        self.lib = load_library()
        self.window, self.hidden = int(window), int(hidden)
        self.n_params = nn_num_params(window, hidden)
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.shape != (self.n_params,):
            raise ValueError(f"expected {self.n_params} parameters, got {p.shape}")
        cfg = NNConfig(window=self.window, hidden=self.hidden, a_scale=float(a_scale),
                       j_scale=float(j_scale), lr=lr, beta1=beta1, beta2=beta2, eps=eps)
        self.a_scale, self.j_scale = float(a_scale), float(j_scale)
        h = C.c_void_p()
        st = self.lib.tddft_nn_create(C.byref(cfg), _fptr(p), C.byref(h))
        if st != OK:
            raise TDDFTError(st, "tddft_nn_create failed")
        self.h = h

    def _check(self, st):
        if st != OK:
            msg = self.lib.tddft_nn_last_error(self.h)
            raise TDDFTError(st, msg.decode() if msg else "")

    def params(self) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        self._check(self.lib.tddft_nn_get_params(self.h, _fptr(out)))
        return out

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        self._check(self.lib.tddft_nn_set_params(self.h, _fptr(p)))

    def forward(self, x) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.empty(x.shape[0], dtype=np.float32)
        self._check(self.lib.tddft_nn_forward(self.h, x.shape[0], _fptr(x), _fptr(y)))
        return y

    def loss_grad(self, x, target):
        x = np.ascontiguousarray(x, dtype=np.float32)
        t = np.ascontiguousarray(target, dtype=np.float32)
        loss = np.zeros(1, dtype=np.float32)
        g = np.empty(self.n_params, dtype=np.float32)
        self._check(self.lib.tddft_nn_loss_grad(self.h, x.shape[0], _fptr(x), _fptr(t), _fptr(loss), _fptr(g)))
        return float(loss[0]), g

    def adam_step(self):
        self._check(self.lib.tddft_nn_adam_step(self.h))

    def train(self, A, J, *, epochs, batch, seed=0, cosine=False, freeze_linear=False):
        A = np.ascontiguousarray(A, dtype=np.float64)
        J = np.ascontiguousarray(J, dtype=np.float64)
        assert A.shape == J.shape and A.ndim == 2
        losses = np.zeros(max(int(epochs), 1), dtype=np.float32)
        flags = (NN_COSINE_LR if cosine else 0) | (NN_FREEZE_LINEAR if freeze_linear else 0)
        self._check(self.lib.tddft_nn_train_ex(self.h, A.shape[0], A.shape[1], _ptr(A), _ptr(J), int(epochs),
                                               int(batch), int(seed), flags, _fptr(losses)))
        return losses[: int(epochs)]

    def fit_linear(self, A, J, *, a_fit, lambda_rel=1e-10):
        """Least-squares skip weights and output bias on the trajectories
        whose largest |A| is within a_fit (device FP64); w3 := 0."""
        A = np.ascontiguousarray(A, dtype=np.float64)
        J = np.ascontiguousarray(J, dtype=np.float64)
        assert A.shape == J.shape and A.ndim == 2
        self._check(self.lib.tddft_nn_fit_linear(self.h, A.shape[0], A.shape[1], _ptr(A), _ptr(J), float(a_fit),
                                                 float(lambda_rel)))

    def close(self):
        if getattr(self, "h", None):
            self.lib.tddft_nn_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


class Multiscale:
    """Coupled 1-D Maxwell + cells (tddft_ms_* entry points). ``cell`` is a
    System whose dt is the cell step (dt / n_sub); ``psi0`` its orbitals."""

    def __init__(self, cell, psi0, *, n_x, x0, n_mat, dx, dt, n_sub, axis=2, precision="mixed", flags=0):
        self.lib = load_library()
        self.n_x = int(n_x)
        cfg = MSConfig(n_x=int(n_x), x0=int(x0), n_mat=int(n_mat), dx=float(dx), dt=float(dt),
                       n_sub=int(n_sub), axis=int(axis))
        ccfg, keep = _config_for(cell, precision, flags)
        psi = np.ascontiguousarray(psi0, dtype=np.complex128)
        v = np.ascontiguousarray(cell.v_loc, dtype=np.float64)
        atoms, kp = _atoms_for(cell.projectors)
        h = C.c_void_p()
        st = self.lib.tddft_ms_create(C.byref(cfg), C.byref(ccfg), _ptr(psi.view(np.float64)), _ptr(v),
                                      len(cell.projectors), atoms if cell.projectors else None, C.byref(h))
        if st != OK:
            raise TDDFTError(st, "tddft_ms_create failed")
        self.h = h

    def _check(self, st):
        if st != OK:
            msg = self.lib.tddft_ms_last_error(self.h)
            raise TDDFTError(st, msg.decode() if msg else "")

    def attach_surrogate(self, nn, *, a_max, sentinels=(), check_every=50, tol=1e-3):
        sen = np.ascontiguousarray(sentinels, dtype=np.int32)
        self._nn = nn
        self._check(self.lib.tddft_ms_attach_surrogate(self.h, nn.h, float(a_max), sen.shape[0],
                                                       _ptr(sen, C.c_int32) if sen.shape[0] else None,
                                                       int(check_every), float(tol)))

    def step(self, n_macro, inc=None):
        A = np.zeros((int(n_macro), self.n_x))
        I = np.zeros((int(n_macro), self.n_x))
        incp = None
        if inc is not None:
            inc = np.ascontiguousarray(inc, dtype=np.float64)
            assert inc.shape == (int(n_macro) + 1, 2)
            incp = _ptr(inc)
        self._check(self.lib.tddft_ms_step(self.h, int(n_macro), incp, _ptr(A), _ptr(I)))
        return A, I

    def energy(self):
        """(field energy, work on the medium) per unit area at the current step."""
        em, w = C.c_double(), C.c_double()
        self._check(self.lib.tddft_ms_energy(self.h, C.byref(em), C.byref(w)))
        return em.value, w.value

    def status(self) -> dict:
        mode, fb, steps = C.c_int32(), C.c_int32(), C.c_int32()
        last = C.c_double()
        self._check(self.lib.tddft_ms_status(self.h, C.byref(mode), C.byref(fb), C.byref(last),
                                             C.byref(steps)))
        return {"mode": "network" if mode.value == 1 else "cells", "fallbacks": fb.value,
                "last_check": last.value, "steps": steps.value}

    def close(self):
        if getattr(self, "h", None):
            self.lib.tddft_ms_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
