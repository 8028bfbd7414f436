"""Device FP64 arrays owned through the library's own allocator (fde_device_alloc).

For processes that run without torch (FDE_NO_TORCH=1): a ``DeviceArray`` is accepted
wherever the binding takes a device tensor.  Copies are synchronous; nothing here touches
the data beyond moving it.
"""
from __future__ import annotations

import ctypes as C
import sys

import numpy as np

from . import _native as N


class DeviceArray:
    """A C-contiguous float64 array in device memory (freed by ``free`` or on collection)."""

    is_cuda = True

    def __init__(self, shape):
        self.shape = tuple(int(d) for d in (shape if isinstance(shape, (tuple, list)) else (shape,)))
        self.size = int(np.prod(self.shape)) if self.shape else 1
        p = C.c_void_p()
        N.check(N.lib().fde_device_alloc(max(1, self.size) * 8, C.byref(p)))
        self._ptr = p.value

    @classmethod
    def from_numpy(cls, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        d = cls(a.shape)
        if a.size:
            N.check(N.lib().fde_memcpy(C.c_void_p(d._ptr), a.ctypes.data_as(C.c_void_p), a.nbytes,
                                       N.FDE_COPY_H2D))
        return d

    def numpy(self):
        out = np.empty(self.shape, dtype=np.float64)
        if self.size:
            N.check(N.lib().fde_memcpy(out.ctypes.data_as(C.c_void_p), C.c_void_p(self._ptr), out.nbytes,
                                       N.FDE_COPY_D2H))
        return out

    def copy_from(self, other: "DeviceArray"):
        if other.size != self.size:
            raise ValueError("size mismatch")
        N.check(N.lib().fde_memcpy(C.c_void_p(self._ptr), C.c_void_p(other._ptr), self.size * 8,
                                   N.FDE_COPY_D2D))

    def data_ptr(self) -> int:
        return self._ptr

    def numel(self) -> int:
        return self.size

    def free(self):
        if getattr(self, "_ptr", None):
            N.lib().fde_device_free(C.c_void_p(self._ptr))
            self._ptr = None

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.free()
        except Exception:
            pass


def synchronize():
    N.check(N.lib().fde_device_synchronize())
