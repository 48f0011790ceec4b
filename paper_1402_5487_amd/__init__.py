"""libplbm: the parametric lattice Boltzmann method (arXiv:1402.5487) on
MI355X.  The compute path is the HIP library libplbm.so behind the C ABI in
include/plbm.h; this package holds its ctypes binding (_plbm), torch-backed
lattice objects (lattice), and the seeded initial fields (inputs).

The binding is imported lazily so that the input generators stay importable
on machines where the library is not built.
"""

__all__ = ["Lattice", "inputs"]


def __getattr__(name):
    if name == "Lattice":
        from .lattice import Lattice
        return Lattice
    raise AttributeError(name)
