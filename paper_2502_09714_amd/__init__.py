"""MI355X-native ADER-DG for 3D seismic waves in the continuum-damage rheology.

The compute path is the HIP library ``libdgd.so`` (C interface in
``include/dgd.h``); this package only marshals arguments to it.
"""
from ._lib import BF16, FP32, FP64, DGDError, lib  # noqa: F401


def Simulation(*args, **kw):
    from .api import Simulation as _S
    return _S(*args, **kw)


def from_workload(*args, **kw):
    from .api import from_workload as _f
    return _f(*args, **kw)
