"""Dense radial-kernel form of the truncated heat operator (oracle pin; tiny grids only).

By Prop. 3.4 a radial kernel operator is a spherical convolution, and the
addition theorem for spherical harmonics (sum_m Y_lm(x) conj(Y_lm(y)) =
(2l+1)/(4 pi) P_l(x.y)) turns the band-limited HeatConv into a dense kernel
    HeatConv(v)_i = sum_j H_L(x_i . x_j) a_j v_j,
    H_L(c) = sum_{l<L} (2l+1)/(4 pi) exp(-t l(l+1)) P_l(c),
with P_l the plain Legendre polynomials, evaluated here by numpy's
``legendre.legval`` -- a library routine independent of the oracle's own
associated-Legendre recurrence.  The identity is exact whenever nlon >= 2L-1.
"""

import numpy as np
from numpy.polynomial import legendre as npleg


def kernel_profile(L, t):
    """Legendre-series coefficients of H_L."""
    l = np.arange(L, dtype=np.float64)
    return (2.0 * l + 1.0) / (4.0 * np.pi) * np.exp(-t * l * (l + 1.0))


def dense_heat_matrix(grid, t):
    """K with (K v)_i = sum_j H_L(x_i . x_j) a_j v_j, shape (n, n); rows/cols in grid order."""
    X = grid.points().reshape(-1, 3)
    c = np.clip(X @ X.T, -1.0, 1.0)
    H = npleg.legval(c, kernel_profile(grid.L, t))
    return H * grid.area.reshape(1, -1)


def dense_heat_apply(v, grid, t, K=None):
    if K is None:
        K = dense_heat_matrix(grid, t)
    v = np.asarray(v, dtype=np.float64)
    shp = v.shape
    return (v.reshape(-1, grid.n) @ K.T).reshape(shp)
