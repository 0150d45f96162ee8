"""MI355X (gfx950) library for the JFNK solution of high-order cell-centred
finite-volume solid mechanics: a C ABI (include/hofv.h, libhofv.so built
in-tree) and a thin ctypes binding (``api``).  There is no CPU fallback: the
binding raises if libhofv.so has not been built."""
from . import _lib  # noqa: F401
from .api import Context, HofvError, context_for  # noqa: F401

__all__ = ["Context", "HofvError", "context_for"]
