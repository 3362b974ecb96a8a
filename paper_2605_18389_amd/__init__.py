"""Heat-kernel (spherical-harmonic) Sinkhorn on S^2 for AMD Instinct MI355X.

Implements the hot path of arXiv 2605.18389: HeatConv (Sec. 3.2) as a row FFT,
per-order Legendre transform, spectral multiply and inverse, inside the
balanced and unbalanced Sinkhorn loop of Alg. 1, the Sinkhorn divergence
(Def. 2.3) and its gradient (Sec. 4.2.2).  All arithmetic runs in the HIP
kernels of ``libshot.so`` (C ABI in ``include/shot.h``); this package only
marshals arguments.  ``synth`` holds seeded input generators.
"""

from .binding import (Plan, ShotError, load_library, status_string, LIB_PATH, EXPORTS,
                      GRID_GAUSS_LEGENDRE, GRID_CLENSHAW_CURTIS, FP64, FP32, BF16_MFMA,
                      LEG_AUTO, LEG_TABLE, LEG_RECURRENCE, OK, E_INVALID, E_BREAKDOWN,
                      W_NOT_CONVERGED, E_UNSUPPORTED)

__all__ = ["Plan", "ShotError", "load_library", "status_string", "LIB_PATH", "EXPORTS"]
