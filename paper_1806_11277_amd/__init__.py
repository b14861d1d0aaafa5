"""MI355X (gfx950) elastic Helmholtz hybrid shifted-Laplacian multigrid / domain
decomposition solver: HIP kernels behind the C ABI of include/ehh.h (libehh.so)
and a thin ctypes binding (``paper_1806_11277_amd.ehh``)."""

__all__ = ["ehh"]
