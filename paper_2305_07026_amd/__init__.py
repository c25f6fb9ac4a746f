"""MI355X (gfx950) implementation of the DABA iteration (decentralized,
accelerated bundle adjustment) behind the C ABI of include/daba.h.

Importing the package loads libdaba.so and fails if it is not built."""

from . import binding  # noqa: F401  (loads the library; raises if missing)
from .solver import DabaObjective, DabaPartSolver, DabaSolver, daba_objective  # noqa: F401

__all__ = ["DabaSolver", "DabaPartSolver", "DabaObjective", "daba_objective", "binding"]
