"""PACO (exact bounded-radix Cooley-Tukey DFT: LocalFFT -> one fused global
permutation -> LocalFFT) as a gfx950 HIP library behind a C ABI.

``paco`` is the ctypes binding of ``libpaco.so``; ``torch_api`` wraps it for
torch tensors (PyTorch provides device memory and streams only).
"""
from . import inputs  # noqa: F401  (seeded synthetic inputs; no transform arithmetic)

__all__ = ["inputs"]
