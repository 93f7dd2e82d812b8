"""MI355X (gfx950) graph-PEPS simple update for the kicked-Ising circuit.

The compute path is libgpeps.so (HIP kernels behind a C ABI, include/gpeps.h);
this package only marshals arguments to it.
"""

from ._lib import GpepsError, load  # noqa: F401

__all__ = ["GpepsError", "load", "Simulator", "from_workload"]


def __getattr__(name):
    if name in ("Simulator", "from_workload"):
        from . import simulator
        return getattr(simulator, name)
    raise AttributeError(name)
