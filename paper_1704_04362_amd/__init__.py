"""MI355X (gfx950) library for the Fourier-domain t-product pipeline of
Tarzanagh & Michailidis, "Fast randomized algorithms for t-product based
tensor operations and decompositions" (rt-product, t-SVD, t-CX/t-CUR,
t-SVT completion).

The compute lives in the HIP shared library ``libtprod.so`` (C ABI declared
in include/tprod.h). ``paper_1704_04362_amd.api`` is a thin binding that
marshals torch device tensors and the current HIP stream into those calls.
Importing this package does not load the library; the first API call does,
and fails loudly if it has not been built (``python -m
paper_1704_04362_amd.build``).
"""

__all__ = ["api"]
