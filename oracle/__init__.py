"""FP64 CPU oracle for spherical-harmonic Sinkhorn (heat-kernel Sinkhorn on S^2).

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain, obviously-correct
reference that the HIP path is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with ``paper_2605_18389_amd`` and imports nothing
from it; the two meet only through seeded input arrays.

Everything is float64 NumPy, written step by step from the paper:

* ``grids``      -- Gauss-Legendre, Gauss-Lobatto and Clenshaw-Curtis (equiangular with poles)
                    latitude quadrature and area weights (App. C.1 "Discretizations
                    of S^2", App. C.2 "Discrete OT on the Sphere").
* ``legendre``   -- orthonormal associated Legendre functions P̄_l^m (App. B,
                    definition of Y_lm and N_lm).
* ``sht``        -- semi-naive SHT (rFFT in longitude, per-order Legendre
                    projection) and HeatConv (Sec. 3.2, "Algorithm" paragraph).
* ``healpix``    -- HEALPix rings (equal-area pixels, App. C.1) and the
                    pseudo-spectral SHT written as direct sums over each ring.
* ``dense``      -- the same operator written as a dense radial kernel via the
                    addition theorem (Prop. 3.4 / Thm. 3.3); a test pin only.
* ``sinkhorn``   -- Algorithm 1 (balanced and unbalanced branches), potentials,
                    cost (App. C.2 eq. for OT^tau_{C,eps}), convergence check
                    (App. C.3), divergence (Def. 2.3), envelope gradient (Sec. 4.2.2).
* ``attribution`` -- centred gradient field and its area-weighted RMS per
                    latitude band (Sec. 4.2.2, regional attribution).
* ``convolution`` -- heat versus matrix convolution of a measure (appendix on
                    convolution on S^2): C(eps), the dense geodesic-Gaussian
                    convolution, the rescaled mean absolute error.

Where the paper is silent or inconsistent, each module's docstring states the
reading it takes (heat time t = eps/4 everywhere, band limit l < L, Alg. 1
taken literally, ...).
"""

from .grids import Grid, gauss_legendre, gauss_lobatto, clenshaw_curtis, make_grid
from .healpix import HealpixGrid, ring_geometry
from .legendre import legendre_table, normalised_legendre_column
from .sht import analysis, synthesis, heat_apply, heat_multipliers
from .dense import dense_heat_matrix, dense_heat_apply
from .sinkhorn import sinkhorn, divergence, envelope_gradient, fd_directional
from .attribution import regional_rms, latitudes
from .convolution import geodesic_kernel_integral, matrix_convolution, heat_convolution, rescaled_mae, heat_vs_matrix

__all__ = [
    "Grid", "gauss_legendre", "gauss_lobatto", "clenshaw_curtis", "make_grid", "HealpixGrid", "ring_geometry",
    "legendre_table", "normalised_legendre_column",
    "analysis", "synthesis", "heat_apply", "heat_multipliers",
    "dense_heat_matrix", "dense_heat_apply",
    "sinkhorn", "divergence", "envelope_gradient", "fd_directional", "regional_rms", "latitudes",
    "geodesic_kernel_integral", "matrix_convolution", "heat_convolution", "rescaled_mae", "heat_vs_matrix",
]
