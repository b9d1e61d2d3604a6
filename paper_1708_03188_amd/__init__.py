"""MI355X (gfx950) spectral-Galerkin hot path: Python binding over libsgm.so.

The binding only marshals arguments; transforms, solves and time steps run in
the HIP kernels of libsgm.so.  Importing the package does not load the
library; the first Plan (or other object) does, and raises SgmError if the
library has not been built.
"""
from ._lib import SgmError, load  # noqa: F401


def __getattr__(name):
    if name in ("Plan", "GLBatch", "FNO"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
