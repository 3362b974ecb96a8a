"""Algorithm 1 (spherical-harmonic Sinkhorn), divergence and gradients (oracle; test infrastructure only).

Steps are taken literally from Alg. 1 ("Spherical Harmonic Sinkhorn", App. C):
  t = eps/4, h_l = exp(-t l(l+1)), u = v = 1, then for k = 1..T
  balanced (tau = inf):  u = p / K v ; v = q / K u ; s = sum_i u_i ; u = u/s ; v = s v
  unbalanced:            u = (p / K v)^(tau/(tau+eps)) ; v = (q / K u)^(tau/(tau+eps))
                         c = tau/2 (log sum_i a_i p_i u_i^(-eps/tau) - log sum_i a_i q_i v_i^(-eps/tau))
                         u = e^(c/eps) u ; v = e^(-c/eps) v
  every C iterations:    e_marg = ||u (.) K v - p||_2 / ||p||_2  (App. C.3), stop if < delta
  then phi = eps log u, psi = eps log v and the returned cost is
  balanced   sum_i a_i (phi_i p_i + psi_i q_i)
  unbalanced sum_i a_i (tau (1 - e^(-phi_i/tau)) p_i + tau (1 - e^(-psi_i/tau)) q_i)   (App. C.2).
K is HeatConv (Sec. 3.2).  The divergence is Def. 2.3 (eq. sinkhorn-divergence):
  S = OT(p,q) - (OT(p,p) + OT(q,q))/2 + eps/2 (m(p) - m(q))^2,  m(p) = sum_i a_i p_i.
The envelope gradient follows Sec. 4.2.2 (gradient from the Kantorovich potentials).

Arrays may carry leading batch dimensions (..., nlat, nlon); every sum is over
the last two axes.  The positivity breakdown of App. C.4 (a truncated kernel
that goes non-positive) is recorded as the first iteration k at which K v or
K u has an entry <= 0 or non-finite; the iteration then simply continues.
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


def divergence(p, q, grid, eps, tau=math.inf, T=100, K=None, return_solves=False):
    """Sinkhorn divergence of Def. 2.3 from three Alg. 1 runs with identical parameters."""
    r_pq = sinkhorn(p, q, grid, eps, tau, T, K=K)
    r_pp = sinkhorn(p, p, grid, eps, tau, T, K=K)
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
    Sp = divergence(p[None] + h * deltas, q[None], grid, eps, tau, T)
    Sm = divergence(p[None] - h * deltas, q[None], grid, eps, tau, T)
    return (Sp - Sm) / (2.0 * h)
