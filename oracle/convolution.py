"""Heat versus matrix convolution on the sphere (oracle; test infrastructure only).

The appendix on convolution on S^2 compares two ways of smoothing a measure f:

* the matrix convolution with the unnormalised geodesic Gaussian
  K_eps(x, y) = exp(-d(x, y)^2 / eps), d the great-circle distance, evaluated
  on the grid as (K_eps f)(x_i) = sum_j a_j K_eps(x_i, x_j) f_j with the grid's
  area weights a_j;
* the heat convolution H_t f at t = eps / 4 (HeatConv of Sec. 3.2), whose
  kernel integrates to one.

By Varadhan's formula H_{eps/4}(x, y) is close to K_eps(x, y) / C(eps) for small
eps, with C(eps) the integral of K_eps(x, .) over the sphere,
    C(eps) = 2 pi int_0^pi exp(-gamma^2 / eps) sin(gamma) d gamma
(the kernel depends on the angle gamma between x and y only, and the area of
the band at angle gamma is 2 pi sin(gamma) d gamma).  The error measure is the
mean over grid points of |C(eps) (H_{eps/4} f) - (K_eps f)|.
"""

import numpy as np

from .sht import heat_apply


def geodesic_kernel_integral(eps, nodes=64, pieces=64):
    """C(eps) by composite Gauss-Legendre quadrature in gamma.

    The integrand is concentrated within a few sqrt(eps) of gamma = 0 for small
    eps, so [0, pi] is cut at gamma = min(pi, 40 sqrt(eps)) (beyond it the
    integrand is below exp(-1600)) and that range split into ``pieces`` equal
    panels of ``nodes`` points each.
    """
    eps = float(eps)
    top = min(np.pi, 40.0 * np.sqrt(eps))
    u, wu = np.polynomial.legendre.leggauss(nodes)
    edges = np.linspace(0.0, top, pieces + 1)
    total = 0.0
    for lo, hi in zip(edges[:-1], edges[1:]):
        g = 0.5 * (hi - lo) * u + 0.5 * (hi + lo)
        total += 0.5 * (hi - lo) * float(np.sum(wu * np.exp(-g * g / eps) * np.sin(g)))
    return 2.0 * np.pi * total


def _flat_points(grid):
    return grid.points().reshape(-1, 3)


def matrix_convolution(f, grid, eps, block=2048):
    """(K_eps f)(x_i) = sum_j a_j exp(-d(x_i, x_j)^2 / eps) f_j; f shaped like a field."""
    X = _flat_points(grid)
    af = (grid.area * np.asarray(f, dtype=np.float64).reshape(grid.area.shape)).reshape(-1)
    out = np.empty(X.shape[0])
    for s in range(0, X.shape[0], block):
        cosd = np.clip(X[s:s + block] @ X.T, -1.0, 1.0)
        d = np.arccos(cosd)
        out[s:s + block] = np.exp(-d * d / eps) @ af
    return out.reshape(grid.area.shape)


def heat_convolution(f, grid, eps):
    """H_t f at t = eps / 4, through the grid's SHT (HeatConv)."""
    f = np.asarray(f, dtype=np.float64).reshape(grid.area.shape)
    return heat_apply(f, grid, eps / 4.0)


def rescaled_mae(heat, matrix, eps):
    """Mean over points of |C(eps) heat - matrix|."""
    return float(np.mean(np.abs(geodesic_kernel_integral(eps) * np.asarray(heat) - np.asarray(matrix))))


def heat_vs_matrix(f, grid, eps_list):
    """MAE of the rescaled heat convolution against the matrix convolution, per eps."""
    return np.array([rescaled_mae(heat_convolution(f, grid, e), matrix_convolution(f, grid, e), e)
                     for e in eps_list])
