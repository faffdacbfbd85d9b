"""MI355X (gfx950) implementation of the online energy + polarisation RFI screen
of arXiv 2412.14775: HIP kernels behind the C ABI in include/rfi.h (librfi.so),
with a thin ctypes binding (``rfi``, which also wraps the serving loop of
csrc/serve.hip as ``rfi.Server``) and a detection-quality harness (``detection``)."""
from . import rfi  # noqa: F401

__all__ = ["rfi"]
