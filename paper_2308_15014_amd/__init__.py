"""CAPS filtered partitioned search (arXiv 2308.15014) on MI355X.

The compute lives in libcaps.so (hand-written HIP for gfx950, C ABI in
include/caps.h); this package marshals arguments to it.
"""
from ._lib import CapsError, lib, profile_enable, profile_read  # noqa: F401
from .index import Index, bliss_assign  # noqa: F401
from .server import Server  # noqa: F401

__all__ = ["Index", "Server", "CapsError", "lib", "bliss_assign"]
