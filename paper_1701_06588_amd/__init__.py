"""MI355X-native engine for contracted solid-harmonic-Gaussian (SHG) integrals.

The compute path lives in ``libshg.so`` (HIP for gfx950, C ABI declared in
``include/shg.h``); ``paper_1701_06588_amd.shg`` is the thin ctypes binding
that marshals torch device tensors into it.
"""
__all__ = ["inputs"]
