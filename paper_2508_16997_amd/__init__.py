"""MI355X-native coupled viscoelastic lattice Boltzmann step (arXiv:2508.16997).

The compute path is the HIP library ``libvlb.so`` (C ABI in ``include/vlb.h``); this
package only marshals arguments and provides device memory and streams via PyTorch.
"""
from ._lib import EXPORTS, LIB_PATH, VlbError, load  # noqa: F401

__all__ = ["Simulation", "Batch", "host_geometry", "params_from_groups", "load", "VlbError", "EXPORTS", "LIB_PATH"]


def __getattr__(name):
    if name in ("Simulation", "Batch", "host_geometry", "params_from_groups"):
        from . import sim

        return getattr(sim, name)
    raise AttributeError(name)
