"""MI355X-native real-time TDKS time step (hand-written HIP kernels for gfx950).

The compute path is libtddft.so (C ABI in include/tddft.h); this package
holds its sources (csrc/), the build step (build.py) and the ctypes binding
(binding.py). Importing the package does not load the library.
"""


def __getattr__(name):
    if name in ("TDDFT", "TDDFTError", "load_library"):
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
