"""Spherical-harmonic Sinkhorn (Alg. 1), the divergence and its gradients (oracle; test infrastructure only).

What this module computes, in plain terms:

* ``sinkhorn`` runs the scaling iteration of Alg. 1 on a grid whose heat
  operator K is HeatConv (Sec. 3.2) at heat time t = eps/4.  The two scalings
  start at one and are refreshed alternately by dividing a marginal by K of the
  other scaling.  In the balanced branch (tau = inf) the pair is then
  re-gauged by the plain sum of u (a gauge only).  In the unbalanced branch
  each quotient is raised to the power tau/(tau+eps) and the pair is
  re-gauged by the translation of App. C.2, which balances the two
  area-weighted sums of p u^(-eps/tau) and q v^(-eps/tau).  Every C
  iterations the relative marginal error of App. C.3 is evaluated (and, with
  a threshold delta > 0, the loop stops early).  The potentials are eps times
  the logarithms of the final scalings; the returned cost is the area-weighted
  sum of App. C.2 (plain potentials for the balanced branch, the
  tau-saturated form for the unbalanced one).
* ``divergence`` combines three such runs with identical parameters into the
  debiased quantity of Def. 2.3, including its mass-difference term.
* ``envelope_gradient`` is the potential-based gradient of Sec. 4.2.2;
  ``fd_directional`` differentiates the whole fixed-T computation numerically.

Arrays may carry leading batch dimensions (..., nlat, nlon); every sum is over
the last two axes.  The positivity breakdown of App. C.4 (a truncated kernel
that goes non-positive) is recorded as the first iteration k at which K v or
K u has an entry <= 0 or non-finite; the iteration then simply continues.

Parity unpinned: the coefficient eps/2 of the mass-difference term of
Def. 2.3.  On constant densities every other part of the unbalanced branch
has a closed-form fixed point that the tests check, but positivity (Prop. 3.2)
does not constrain that coefficient there, so the tests can only restate it.
"""

import math

import numpy as np

from .sht import heat_apply


def _sum2(x):
    return x.sum(axis=(-2, -1))


def _bcast(s):
    return np.asarray(s)[..., None, None]


def sinkhorn(p, q, grid, eps, tau=math.inf, T=100, delta=0.0, C=10, K=None,
             normalize=True):
    """Run Alg. 1.  ``K`` overrides the heat operator (used with the dense pin).

    ``normalize=False`` skips the balanced s-rescaling (a gauge; used by a test).
    Returns a dict with u, v, phi, psi, cost, iters, e_hist [(k, e)], err (e_marg
    of the returned u, v), breakdown (first bad iteration per item, 0 if none),
    kratio (min over the run of min(K.)/max(K.) per item; -inf once non-finite)
    and kratio_hist (that minimum per iteration).
    """
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    if K is None:
        t = eps / 4.0
        K = lambda x: heat_apply(x, grid, t)
    a = grid.area
    balanced = math.isinf(tau)
    lead = np.broadcast_shapes(p.shape, q.shape)[:-2]
    u = np.ones(lead + grid.field_shape)
    v = np.ones(lead + grid.field_shape)
    breakdown = np.zeros(lead, dtype=np.int64)
    kratio = np.full(lead, np.inf)
    if delta > 0 and len(lead) > 0:
        raise ValueError("early exit is only defined for a single item")

    kratio_hist = []   # per iteration: min over its two heat applies of min(K.)/max(K.)

    def watch(Kx, k):
        nonlocal kratio
        mn = Kx.min(axis=(-2, -1))
        mx = Kx.max(axis=(-2, -1))
        bad = ~(np.isfinite(Kx).all(axis=(-2, -1))) | (mn <= 0)
        new = bad & (breakdown == 0)
        breakdown[new] = k
        with np.errstate(invalid="ignore", divide="ignore"):
            ratio = np.where(np.isfinite(mn / mx), mn / mx, -np.inf)
            kratio = np.fmin(kratio, ratio)
        if len(kratio_hist) < k:
            kratio_hist.append(ratio)
        else:
            kratio_hist[k - 1] = np.fmin(kratio_hist[k - 1], ratio)

    e_hist = []
    k = 0
    with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
        for k in range(1, T + 1):
            if balanced:
                Kv = K(v)
                watch(Kv, k)
                u = p / Kv
                Ku = K(u)
                watch(Ku, k)
                v = q / Ku
                if normalize:
                    s = _sum2(u)
                    u = u / _bcast(s)
                    v = _bcast(s) * v
            else:
                lam = tau / (tau + eps)
                Kv = K(v)
                watch(Kv, k)
                u = (p / Kv) ** lam
                Ku = K(u)
                watch(Ku, k)
                v = (q / Ku) ** lam
                c = tau / 2.0 * (np.log(_sum2(a * p * u ** (-eps / tau)))
                                 - np.log(_sum2(a * q * v ** (-eps / tau))))
                u = np.exp(_bcast(c) / eps) * u
                v = np.exp(-_bcast(c) / eps) * v
            if k % C == 0:
                e = np.sqrt(_sum2((u * K(v) - p) ** 2)) / np.sqrt(_sum2(p * p))
                e_hist.append((k, e))
                if delta > 0 and e < delta:
                    break
        err = np.sqrt(_sum2((u * K(v) - p) ** 2)) / np.sqrt(_sum2(p * p))
        phi = eps * np.log(u)
        psi = eps * np.log(v)
        if balanced:
            cost = _sum2(a * (phi * p + psi * q))
        else:
            cost = _sum2(a * (tau * (1.0 - np.exp(-phi / tau)) * p
                              + tau * (1.0 - np.exp(-psi / tau)) * q))
    return dict(u=u, v=v, phi=phi, psi=psi, cost=cost, iters=k, e_hist=e_hist,
                err=err, breakdown=breakdown, kratio=kratio, kratio_hist=kratio_hist)


def mass(p, grid):
    return _sum2(grid.area * np.asarray(p, dtype=np.float64))


def divergence(p, q, grid, eps, tau=math.inf, T=100, K=None, return_solves=False, r_qq=None):
    """Sinkhorn divergence of Def. 2.3 from three Alg. 1 runs with identical parameters.

    ``r_qq``: an already computed (q, q) solve with these parameters, reused."""
    r_pq = sinkhorn(p, q, grid, eps, tau, T, K=K)
    r_pp = sinkhorn(p, p, grid, eps, tau, T, K=K)
    if r_qq is None:
        r_qq = sinkhorn(q, q, grid, eps, tau, T, K=K)
    S = (r_pq["cost"] - 0.5 * (r_pp["cost"] + r_qq["cost"])
         + 0.5 * eps * (mass(p, grid) - mass(q, grid)) ** 2)
    if return_solves:
        return S, (r_pq, r_pp, r_qq)
    return S


def envelope_gradient(r_pq, r_pp, grid, eps, mp, mq):
    """dS/dp from the Kantorovich potentials (balanced), as a density-array gradient.

    d OT(p,q)/dp = a phi_pq and, for the symmetric term, d OT(p,p)/dp =
    a (phi_pp + psi_pp); the mass term contributes eps (m(p)-m(q)) a.  The
    potentials are defined up to a constant, so this is meaningful up to a
    multiple of a (compare along directions with sum a delta = 0, or centre).
    """
    a = grid.area
    return a * (r_pq["phi"] - 0.5 * (r_pp["phi"] + r_pp["psi"])) + eps * (mp - mq) * a


def fd_directional(p, q, deltas, grid, eps, T, h=1e-4, tau=math.inf):
    """Central finite differences of S(p, q) along each direction (fixed T)."""
    deltas = np.asarray(deltas, dtype=np.float64)
    r_qq = sinkhorn(q, q, grid, eps, tau, T)      # does not depend on p
    Sp = divergence(p[None] + h * deltas, q[None], grid, eps, tau, T, r_qq=r_qq)
    Sm = divergence(p[None] - h * deltas, q[None], grid, eps, tau, T, r_qq=r_qq)
    return (Sp - Sm) / (2.0 * h)
