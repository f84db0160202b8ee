"""DoGIP (double-grid quadrature with interpolation-projection) operator on MI355X.

The compute path is libdogip.so (HIP kernels for gfx950 behind the C interface
of include/dogip.h); this package holds its sources, the ctypes binding and thin
handles that take device memory and streams from torch.
"""

from .capi import DogipError, lib  # noqa: F401
from .dogip import Batch, Mesh, Operator, Space, quadrature_rule, stream_ptr  # noqa: F401

__all__ = ["Mesh", "Space", "Operator", "Batch", "DogipError", "lib", "stream_ptr", "quadrature_rule"]
