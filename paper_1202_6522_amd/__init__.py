"""shtn: Gauss-Legendre spherical harmonic transforms on AMD MI355X (gfx950).

Method: Schaeffer, arXiv 1202.6522.  The transforms run in hand-written HIP
kernels behind the C interface of include/shtn.h (libshtn.so); `shtn.Plan`
is the torch-facing binding and `autograd` wraps it for differentiation.
Importing the package does not load the library.
"""
from . import inputs  # noqa: F401

__all__ = ["inputs", "shtn", "autograd"]


def __getattr__(name):
    if name in ("shtn", "autograd", "batch"):
        import importlib
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
