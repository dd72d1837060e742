"""DAWN shortest paths on one MI355X: a HIP library (``libdawn.so``) behind a C ABI.

``paper_2208_04514_amd.dawn`` is the Python binding (same names as the C
entry points); ``paper_2208_04514_amd.build`` compiles the library.
"""
from . import dawn  # noqa: F401
from .dawn import DawnError, load  # noqa: F401

__all__ = ["dawn", "DawnError", "load"]
