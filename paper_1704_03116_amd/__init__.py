"""MI355X (gfx950) implementation of the DOPE ADMM hot path: C-ABI library libdope.so (include/dope.h)
with hand-written HIP kernels, and a thin ctypes binding."""
from . import _native  # noqa: F401
from ._native import DopeError  # noqa: F401

__all__ = ["_native", "DopeError", "Dope"]


def __getattr__(name):
    if name == "Dope":
        from .solver import Dope
        return Dope
    raise AttributeError(name)
