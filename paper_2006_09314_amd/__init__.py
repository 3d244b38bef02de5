"""fracctl: rank-truncated PCG for the fractional control equation on MI355X.

The compute path lives in the native library libfracctl.so (HIP kernels for
gfx950 behind a C ABI, declared in include/fracctl.h).  This package is a
thin ctypes binding over it: `lib()` loads the library, `api` marshals torch
device tensors into the C calls.  Nothing here computes any part of the
method.
"""
from ._lib import lib, LibraryMissing, FcError, STATUS  # noqa: F401

__all__ = ["lib", "LibraryMissing", "FcError", "STATUS"]
