"""MI355X-native moment-represented regularized lattice Boltzmann step.

The hot path (fused collide-reconstruct-pull-project-correct step of
arXiv 2609.09160, Eqs. (7)-(9)) is hand-written HIP for gfx950 in
`csrc/`, built into `liblbfast.so` behind the C ABI of `include/lbfast.h`.
`Solver` is the thin Python front end (torch provides device memory and the
stream).  `inputs` holds the seeded synthetic input recipes.
"""
from ._lib import LbfastError, declared_functions, load  # noqa: F401


def __getattr__(name):
    if name == "Solver":
        from .solver import Solver
        return Solver
    raise AttributeError(name)
