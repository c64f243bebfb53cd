"""libjacobi: partitioned synchronous Jacobi for AMD MI355X (gfx950).

The compute path lives in the C-ABI shared library ``libjacobi.so`` built
from ``csrc/``; ``binding`` loads it with ctypes and exposes its entry points
under the same names.  Importing this package loads nothing: the library is
opened on first use, and a missing library raises instead of falling back.
"""
__all__ = ["binding", "workloads"]
