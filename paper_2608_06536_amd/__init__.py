"""MI355X (gfx950) engine for the Cholesky-decomposed Coulomb/exchange build
with non-symmetric densities, its derivative, batched and mixed-precision
forms.  The kernels are in ``csrc/`` (HIP), behind the C ABI of
``include/jk.h``; ``jk`` is the Python binding and ``synth`` the seeded input
generator.  The library loads lazily on first use and raises if missing."""
import importlib

__all__ = ["jk", "synth"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
