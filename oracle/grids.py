"""Latitude quadratures and area weights (oracle; test infrastructure only).

Follows App. C.1 (iso-latitude grids: Gauss-Legendre nodes at the roots of
P_nlat; equiangular Clenshaw-Curtis with pole rows) and App. C.2 (area weights
a with sum 4*pi so that the integral of f over S^2 is a^T f).

Conventions: row 0 is the northernmost latitude (colatitude closest to 0), so
the nodes x_j = cos(theta_j) are in descending order; column k sits at
longitude phi_k = 2*pi*k/nlon.  The area weight of point (j, k) is
w_j * 2*pi / nlon, with sum_j w_j = 2.
"""

from dataclasses import dataclass

import numpy as np


def _legendre_p_and_dp(n, x):
    """P_n(x) and P_n'(x) by the Bonnet recurrence (plain Legendre polynomials)."""
    p_prev = np.ones_like(x)
    p = x.copy()
    if n == 0:
        return p_prev, np.zeros_like(x)
    for k in range(1, n):
        p_prev, p = p, ((2 * k + 1) * x * p - k * p_prev) / (k + 1)
    dp = n * (x * p - p_prev) / (x * x - 1.0)
    return p, dp


def gauss_legendre(n):
    """Gauss-Legendre nodes (descending) and weights, by Newton's method on P_n."""
    i = np.arange(n, dtype=np.float64)
    x = np.cos(np.pi * (i + 0.75) / (n + 0.5))  # Tricomi-style initial guess
    for _ in range(100):
        p, dp = _legendre_p_and_dp(n, x)
        dx = p / dp
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    p, dp = _legendre_p_and_dp(n, x)
    w = 2.0 / ((1.0 - x * x) * dp * dp)
    return x, w


def clenshaw_curtis(n):
    """Clenshaw-Curtis nodes (theta_j = j*pi/(n-1), poles included) and weights.

    Explicit cosine-sum form of the Clenshaw-Curtis rule: with N = n - 1,
    w_j = (c_j/N) * (1 - sum_{k=1}^{floor(N/2)} b_k/(4k^2-1) * cos(2k theta_j)),
    c_j = 1 at the two poles and 2 elsewhere, b_k = 1 when k = N/2 and 2 otherwise.
    """
    N = n - 1
    theta = np.pi * np.arange(n, dtype=np.float64) / N
    w = np.empty(n)
    for j in range(n):
        s = 0.0
        for k in range(1, N // 2 + 1):
            b = 1.0 if 2 * k == N else 2.0
            s += b / (4.0 * k * k - 1.0) * np.cos(2.0 * k * theta[j])
        c = 1.0 if j in (0, N) else 2.0
        w[j] = c / N * (1.0 - s)
    return np.cos(theta), w


def gauss_lobatto(n):
    """Gauss-Lobatto nodes (descending: x = 1 first) and weights (sum 2), n >= 2.

    App. C.1's Lobatto grid: rows at the poles and at the zeros of P'_{n-1},
    i.e. the zeros of (1 - x^2) P'_{n-1}(x); the weights of this rule are
    w_j = 2 / (n (n-1) P_{n-1}(x_j)^2), and it integrates polynomials of degree
    up to 2n - 3 exactly.  Interior nodes by Newton's method on P'_{n-1},
    whose derivative follows from Legendre's equation:
    (1 - x^2) P''_{n-1} = 2 x P'_{n-1} - n (n-1) P_{n-1}.
    """
    if n < 2:
        raise ValueError("a Lobatto rule needs at least the two poles")
    N = n - 1
    x = np.cos(np.pi * np.arange(n, dtype=np.float64) / N)   # Chebyshev-Lobatto start
    xi = x[1:-1].copy()
    for _ in range(100):
        p, dp = _legendre_p_and_dp(N, xi)
        d2p = (2.0 * xi * dp - N * (N + 1) * p) / (1.0 - xi * xi)
        dx = dp / d2p
        xi = xi - dx
        if xi.size == 0 or np.max(np.abs(dx)) < 1e-16:
            break
    x[1:-1] = xi
    x[0], x[-1] = 1.0, -1.0
    pN = np.array([_legendre_p_and_dp(N, np.array([v]))[0][0] if abs(v) < 1 else (v ** N) for v in x])
    w = 2.0 / (n * N * pN * pN)
    return x, w


@dataclass
class Grid:
    kind: str          # "gl" (Gauss-Legendre), "cc" (Clenshaw-Curtis, equiangular with poles) or "lob" (Gauss-Lobatto)
    nlat: int
    nlon: int
    L: int             # band limit: degrees and orders l, m < L
    x: np.ndarray      # cos(colatitude), descending, shape (nlat,)
    w: np.ndarray      # latitude weights, sum 2, shape (nlat,)

    @property
    def n(self):
        return self.nlat * self.nlon

    @property
    def field_shape(self):
        return (self.nlat, self.nlon)

    @property
    def theta(self):
        return np.arccos(np.clip(self.x, -1.0, 1.0))

    @property
    def phi(self):
        return 2.0 * np.pi * np.arange(self.nlon) / self.nlon

    @property
    def area(self):
        """Area weights a_{jk} = w_j * 2 pi / nlon, shape (nlat, nlon), sum 4 pi."""
        return np.repeat((self.w * 2.0 * np.pi / self.nlon)[:, None], self.nlon, axis=1)

    def points(self):
        """Cartesian unit vectors (cos phi sin theta, sin phi sin theta, cos theta), shape (nlat, nlon, 3)."""
        th = self.theta[:, None]
        ph = self.phi[None, :]
        return np.stack(np.broadcast_arrays(np.cos(ph) * np.sin(th), np.sin(ph) * np.sin(th),
                                            np.cos(th) + 0 * ph), axis=-1)


def make_grid(kind, nlat, nlon, L):
    if 2 * L - 1 > nlon:
        raise ValueError("nlon must be at least 2L-1")
    if kind == "gl":
        x, w = gauss_legendre(nlat)
    elif kind == "cc":
        x, w = clenshaw_curtis(nlat)
    elif kind == "lob":
        x, w = gauss_lobatto(nlat)
    else:
        raise ValueError(kind)
    return Grid(kind, nlat, nlon, L, x, w)
