"""MI355X-native lattice scalar-field evolution (CosmoLattice 2.0 hot path).

The product is the HIP library libcl_lattice.so behind the C ABI of
include/cl_lattice.h; this package holds its sources (csrc/), its build
script and a thin ctypes binding with the same call names.  The binding
(`Lattice`, `Ensemble`, `lib`, ...) is loaded on first attribute access and
raises ImportError when the library has not been built.
"""
import importlib
import importlib.util


def __getattr__(name):
    if name.startswith("_"):
        raise AttributeError(name)
    if importlib.util.find_spec(__name__ + "." + name) is not None:
        return importlib.import_module(__name__ + "." + name)  # a submodule (e.g. build)
    return getattr(importlib.import_module(__name__ + "._lib"), name)
