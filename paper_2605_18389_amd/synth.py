"""Seeded synthetic measures on iso-latitude grids.

Input generation only: nothing here evaluates the heat operator, the SHT or
Sinkhorn.  The caller passes the grid's nodes x_j = cos(colatitude) and its
latitude weights w_j (sum 2); normalisation uses the area weights
a_{jk} = w_j * 2 pi / nlon so that sum_jk a_{jk} p_{jk} equals the requested mass.
Points follow App. B's parametrisation x = (cos phi sin theta, sin phi sin theta,
cos theta), phi_k = 2 pi k / nlon.

Generators (all draws from numpy's PCG64 ``default_rng(seed)`` in a fixed order):

* ``vmf_mixture``   -- equal-weight mixture of von Mises-Fisher densities
                       kappa/(2 pi (1 - e^{-2 kappa})) e^{kappa (mu.x - 1)} plus a floor.
                       Per measure: K centres (3 normals each, normalised), then
                       K concentrations kappa ~ U[5, 50].
* ``temperature_like`` -- zonal cos^2(latitude) background times
                       (1 + sum_k amp_k e^{kappa_k (mu_k.x - 1)}), clipped at 0, plus
                       a 1e-6 floor.  Per measure: K centres, K kappa ~ U[5, 50],
                       K amplitudes ~ U[-0.2, 0.2].
* ``uniform_field`` -- i.i.d. U[0, 1] per point, normalised.
* ``vmf_at``        -- one von Mises-Fisher density (the convolution study's input):
                       one centre (3 normals, normalised), fixed kappa, unit mass on
                       the sphere (not renormalised on the grid).

The ``*_at`` variants take any point set instead of a latitude-longitude grid
(e.g. HEALPix pixel centres): per point z = cos(colatitude), longitude phi
and area weight, same draws in the same order.
"""

import math

import numpy as np


def _points(x, nlon):
    x = np.asarray(x, dtype=np.float64)
    st = np.sqrt(np.maximum(0.0, 1.0 - x * x))[:, None]
    ph = 2.0 * np.pi * np.arange(nlon)[None, :] / nlon
    return np.stack(np.broadcast_arrays(np.cos(ph) * st, np.sin(ph) * st, x[:, None] + 0 * ph), -1)


def _centres(rng, K):
    c = rng.standard_normal((K, 3))
    return c / np.linalg.norm(c, axis=1, keepdims=True)


def _normalise(f, w, nlon, total):
    a = (np.asarray(w, dtype=np.float64) * 2.0 * np.pi / nlon)[:, None]
    return f * (total / float((a * f).sum()))


def vmf_mixture(rng, x, w, nlon, K=4, floor=1e-6, total=1.0):
    X = _points(x, nlon)
    mu = _centres(rng, K)
    kap = rng.uniform(5.0, 50.0, K)
    f = np.zeros(X.shape[:2])
    for k in range(K):
        dens = kap[k] / (2.0 * np.pi * (1.0 - math.exp(-2.0 * kap[k])))
        f += dens * np.exp(kap[k] * (X @ mu[k] - 1.0)) / K
    return _normalise(f + floor, w, nlon, total)


def temperature_like(rng, x, w, nlon, K=8, floor=1e-6, total=1.0):
    X = _points(x, nlon)
    mu = _centres(rng, K)
    kap = rng.uniform(5.0, 50.0, K)
    amp = rng.uniform(-0.2, 0.2, K)
    anom = np.ones(X.shape[:2])
    for k in range(K):
        anom += amp[k] * np.exp(kap[k] * (X @ mu[k] - 1.0))
    cos2lat = (1.0 - np.asarray(x, dtype=np.float64) ** 2)[:, None]
    f = np.maximum(cos2lat * anom, 0.0) + floor
    return _normalise(f, w, nlon, total)


def uniform_field(rng, x, w, nlon, total=1.0):
    f = rng.uniform(0.0, 1.0, (len(x), nlon))
    return _normalise(f, w, nlon, total)


def pair_seed(workload_id, pair_index):
    """Seed of pair i of the workload numbered w: 1000 w + i (each workload draws its
    pairs from its own block of seeds)."""
    return 1000 * workload_id + pair_index


def vmf_pair(seed, x, w, nlon, K=4):
    """Two probability measures of ``vmf_mixture``, q drawn after p from one stream."""
    rng = np.random.default_rng(seed)
    p = vmf_mixture(rng, x, w, nlon, K)
    q = vmf_mixture(rng, x, w, nlon, K)
    return p, q


def temperature_pair(seed, x, w, nlon, K=8, q_mass=1.0):
    """Two ``temperature_like`` measures; q is scaled to total mass ``q_mass``."""
    rng = np.random.default_rng(seed)
    p = temperature_like(rng, x, w, nlon, K)
    q = temperature_like(rng, x, w, nlon, K, total=q_mass)
    return p, q


def batch_pair_params(seed, npairs):
    """Per-pair (t, tau, q_mass) of the uneven batched workload.

    t = 10^U[-4,-2]; even pairs balanced (tau = inf, equal masses); odd pairs
    unbalanced with tau drawn from {0.1, 1, 10} and masses 1 vs 1.05.
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(npairs):
        t = 10.0 ** rng.uniform(-4.0, -2.0)
        if i % 2 == 0:
            out.append((t, math.inf, 1.0))
        else:
            tau = (0.1, 1.0, 10.0)[int(rng.integers(0, 3))]
            out.append((t, tau, 1.05))
    return out


def _points_at(z, phi):
    z = np.asarray(z, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    st = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([np.cos(phi) * st, np.sin(phi) * st, z], -1)


def _normalise_at(f, area, total):
    return f * (total / float((np.asarray(area, dtype=np.float64) * f).sum()))


def temperature_like_at(rng, z, phi, area, K=8, floor=1e-6, total=1.0):
    X = _points_at(z, phi)
    mu = _centres(rng, K)
    kap = rng.uniform(5.0, 50.0, K)
    amp = rng.uniform(-0.2, 0.2, K)
    anom = np.ones(X.shape[0])
    for k in range(K):
        anom += amp[k] * np.exp(kap[k] * (X @ mu[k] - 1.0))
    f = np.maximum((1.0 - np.asarray(z, dtype=np.float64) ** 2) * anom, 0.0) + floor
    return _normalise_at(f, area, total)


def uniform_at(rng, area, total=1.0):
    f = rng.uniform(0.0, 1.0, np.asarray(area).shape)
    return _normalise_at(f, area, total)


def temperature_pair_at(seed, z, phi, area, K=8, q_mass=1.0):
    """Two ``temperature_like_at`` measures on a point set; q has mass ``q_mass``."""
    rng = np.random.default_rng(seed)
    p = temperature_like_at(rng, z, phi, area, K)
    q = temperature_like_at(rng, z, phi, area, K, total=q_mass)
    return p, q


def uniform_pair_at(seed, area):
    """Two ``uniform_at`` probability measures (the paper's runtime workload)."""
    rng = np.random.default_rng(seed)
    return uniform_at(rng, area), uniform_at(rng, area)


def vmf_at(seed, z, phi, kappa=10.0):
    """One vMF density with a seeded random mean direction at points (z, phi); returns (f, mu)."""
    rng = np.random.default_rng(seed)
    mu = _centres(rng, 1)[0]
    X = _points_at(z, phi)
    c = kappa / (2.0 * np.pi * (1.0 - math.exp(-2.0 * kappa)))
    return c * np.exp(kappa * (X @ mu - 1.0)), mu


def mass_preserving_directions(seed, p, area, n):
    """n perturbation directions of a density p for finite differences:
    d = p (.) z - p <a, p (.) z> / <a, p> with z ~ N(0, 1) per point (numpy
    PCG64 ``default_rng(seed)``, one field of normals per direction), so that
    sum a d = 0 (the mass of p + h d stays that of p)."""
    rng = np.random.default_rng(seed)
    p = np.asarray(p, dtype=np.float64)
    a = np.asarray(area, dtype=np.float64)
    out = []
    for _ in range(n):
        d = p * rng.standard_normal(p.shape)
        out.append(d - p * float((a * d).sum()) / float((a * p).sum()))
    return np.array(out)


def sample_indices(seed, n, count):
    """`count` distinct flat point indices of an n-point field, sorted (PCG64
    ``default_rng(seed)``): where full-size results are compared point by point."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=min(count, n), replace=False))
