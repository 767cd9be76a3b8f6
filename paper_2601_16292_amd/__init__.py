"""MI355X (gfx950) hot path of columnar agent-based modelling (arXiv 2601.16292).

The compute lives in ``libamber.so`` (hand-written HIP kernels behind a C ABI,
``include/amber.h``); ``paper_2601_16292_amd.amber`` is a thin ctypes binding
with the same names, and ``Population`` allocates the caller-owned device
buffers with PyTorch.  Importing the package loads nothing; the binding raises
if the library has not been built.
"""

__all__ = ["amber", "workloads"]
