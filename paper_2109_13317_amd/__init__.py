"""MI355X-native SU(2) pseudofermion-FRG flow engine (arXiv:2109.13317).

The flow right-hand side, Runge-Kutta steps and correlations run in HIP
kernels behind the C ABI of include/pffrg.h (libpffrg.so, built in this
directory).  This package holds the Python binding (``flow.Context`` for one flow,
``flow.Batch`` for many flows in lockstep), the
lattice front end that produces the ABI's symmetry-reduced tables
(``lattice.build_tables``), flow checkpoints (``checkpoint``), the breakdown
detector for chi_max(Lambda) (``breakdown``), task and resource files in the
paper's XML layout (``taskfile``) and the build script.
"""

from .lattice import LatticeTables, build_tables

__all__ = ["LatticeTables", "build_tables", "Context", "Batch"]


def __getattr__(name):
    if name in ("Context", "Batch"):
        from . import flow
        return getattr(flow, name)
    raise AttributeError(name)
