"""MI355X (gfx950) splitter for the Mandelbrot polynomials p_n and q_{l,n}
(Mihalache & Vigneron, "How to split a tera-polynomial", arXiv 2402.06083).

The hot path lives in ``libmsplit.so`` (HIP kernels behind the C ABI of
``include/msplit.h``); :mod:`paper_2402_06083_amd.msplit` is its ctypes
binding.
"""
from . import msplit  # noqa: F401
from .msplit import (certify, expected_count, hyperbolic, misiurewicz, split,  # noqa: F401
                     workspace_size)
