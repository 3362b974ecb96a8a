"""Orthonormal associated Legendre functions (oracle; test infrastructure only).

App. B defines Y_lm(theta, phi) = N_lm P_l^m(cos theta) e^{i m phi} with
N_lm = sqrt((2l+1)/(4 pi) * (l-m)!/(l+m)!).  Here P̄_l^m(x) = N_lm P_l^m(x) for
0 <= m <= l, without the Condon-Shortley phase (the phase cancels between
analysis and synthesis, so the heat operator does not depend on it).

P̄ is computed in float64 by the standard three-term recurrence in l:
  P̄_0^0 = 1/sqrt(4 pi)
  P̄_m^m = sqrt((2m+1)/(2m)) * sin(theta) * P̄_{m-1}^{m-1}
  P̄_{m+1}^m = sqrt(2m+3) * x * P̄_m^m
  P̄_l^m = A_lm * (x P̄_{l-1}^m - B_lm P̄_{l-2}^m),
     A_lm = sqrt((4l^2-1)/(l^2-m^2)),  B_lm = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)).
Values below the float64 range underflow to zero; they are negligible for the
band limits used here.
"""

import numpy as np


def normalised_legendre_column(L, m, x):
    """P̄_l^m(x) for l = m..L-1, shape (L-m, len(x)), float64."""
    x = np.asarray(x, dtype=np.float64)
    s = np.sqrt(np.maximum(0.0, 1.0 - x * x))
    pmm = np.full_like(x, 1.0 / np.sqrt(4.0 * np.pi))
    for k in range(1, m + 1):
        pmm = np.sqrt((2.0 * k + 1.0) / (2.0 * k)) * s * pmm
    out = np.zeros((L - m, x.size))
    out[0] = pmm
    if L - m > 1:
        out[1] = np.sqrt(2.0 * m + 3.0) * x * pmm
    for l in range(m + 2, L):
        A = np.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
        B = np.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
        out[l - m] = A * (x * out[l - m - 1] - B * out[l - m - 2])
    return out


def legendre_table(L, x):
    """List over m = 0..L-1 of arrays P̄_l^m(x_j), shape (L-m, nlat)."""
    return [normalised_legendre_column(L, m, x) for m in range(L)]
