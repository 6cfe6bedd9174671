"""MI355X-native A-tSNE high-dimensional similarity path (arXiv:1512.01655).

The compute lives in ``libatsne.so`` (hand-written HIP for gfx950 behind a C
ABI declared in ``include/atsne.h``); ``paper_1512_01655_amd.atsne`` is the
thin ctypes binding over it.  Importing the package does not load the
library; the binding does, and fails loudly when it is missing.
"""
__all__ = ["atsne", "datagen"]
