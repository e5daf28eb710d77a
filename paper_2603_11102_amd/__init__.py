"""MI355X-native high-order gas-kinetic scheme step (S2O4, isothermal, WENO-JS, ALM + IBM body forces).

The compute path is libgks.so (hand-written HIP for gfx950, C ABI in include/gks.h); this package holds
the HIP sources (csrc/), the in-tree build script and a thin ctypes binding. Import of the binding is
lazy so that the build step and CPU-only tooling do not need a GPU.
"""


def __getattr__(name):
    if name == "GksSolver":
        from .solver import GksSolver
        return GksSolver
    raise AttributeError(name)
