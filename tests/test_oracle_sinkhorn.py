"""Pins for the oracle's Alg. 1, cost, divergence and gradient.

* dense brute force: Alg. 1 with the SHT operator equals Alg. 1 with the dense
  radial kernel (Prop. 3.4);
* duality: on a tiny grid the value returned by Alg. 1 equals the optimum of
  the entropic (unbalanced) OT dual maximised by a generic optimiser (App. C.2:
  the return follows from strong duality), up to the known constant terms;
* invariants: balanced v (.) K u = q, gauge invariance of the balanced cost,
  tau -> inf recovers the balanced value (App. C.2), S(a,a) = 0, S >= 0 and
  symmetry (Prop. 3.2), envelope gradient vs finite differences (Sec. 4.2.2);
* failure mode: the truncated-kernel breakdown of App. C.4 on the 32x64 vMF case.
"""

import math

import numpy as np
import pytest
from scipy.optimize import minimize

import oracle as O
from paper_2605_18389_amd import synth


def _c1(seed, t=1e-2):
    g = O.make_grid("gl", 32, 64, 32)
    p, q = synth.vmf_pair(synth.pair_seed(0, seed), g.x, g.w, 64, K=4)
    return g, p, q, 4 * t


def _small_pair(kind="gl", nlat=12, nlon=24, L=12, seed=5, qmass=1.0):
    g = O.make_grid(kind, nlat, nlon, L)
    p, q = synth.temperature_pair(seed, g.x, g.w, nlon, K=3, q_mass=qmass)
    return g, p, q


@pytest.mark.parametrize("tau", [math.inf, 1.0])
def test_sht_equals_dense_kernel_sinkhorn(tau):
    g, p, q = _small_pair(qmass=1.0 if math.isinf(tau) else 1.05)
    eps = 0.2
    K = O.dense_heat_matrix(g, eps / 4)
    rs = O.sinkhorn(p, q, g, eps, tau, T=60)
    rd = O.sinkhorn(p, q, g, eps, tau, T=60, K=lambda x: O.dense_heat_apply(x, g, eps / 4, K))
    np.testing.assert_allclose(rs["phi"], rd["phi"], atol=1e-11)
    np.testing.assert_allclose(rs["psi"], rd["psi"], atol=1e-11)
    assert abs(rs["cost"] - rd["cost"]) < 1e-12 * max(1.0, abs(rd["cost"]))


def test_sht_equals_dense_c1_shape():
    g, p, q, _ = _c1(0)
    eps = 0.16  # resolved kernel at L=32
    K = O.dense_heat_matrix(g, eps / 4)
    rs = O.sinkhorn(p, p, g, eps, T=40)
    rd = O.sinkhorn(p, p, g, eps, T=40, K=lambda x: O.dense_heat_apply(x, g, eps / 4, K))
    np.testing.assert_allclose(rs["u"], rd["u"], rtol=1e-10)
    assert abs(rs["cost"] - rd["cost"]) < 1e-11


def _dual_optimum(g, p, q, eps, tau):
    """Maximise the entropic (U)OT dual directly with L-BFGS; returns (D*, phi, psi).

    D(phi, psi) = F(phi; p) + F(psi; q) - eps sum_ij a_i a_j e^{(phi_i+psi_j)/eps} H_ij,
    F(phi; p) = sum a phi p (balanced) or sum a tau (1 - e^{-phi/tau}) p.
    """
    a = g.area.ravel()
    K = O.dense_heat_matrix(g, eps / 4)      # K_ij = H_ij a_j
    H = K / a[None, :]
    assert H.min() > 0
    p = p.ravel()
    q = q.ravel()
    n = a.size

    def F(phi, pp):
        if math.isinf(tau):
            return (a * phi * pp).sum(), a * pp
        e = np.exp(-phi / tau)
        return (a * tau * (1 - e) * pp).sum(), a * e * pp

    def negD(z):
        phi, psi = z[:n], z[n:]
        u = np.exp(phi / eps)
        v = np.exp(psi / eps)
        M = (a * u)[:, None] * H * (a * v)[None, :]
        f1, g1 = F(phi, p)
        f2, g2 = F(psi, q)
        D = f1 + f2 - eps * M.sum()
        gphi = g1 - M.sum(axis=1)
        gpsi = g2 - M.sum(axis=0)
        return -D, -np.concatenate([gphi, gpsi])

    res = minimize(negD, np.zeros(2 * n), jac=True, method="L-BFGS-B",
                   options=dict(maxiter=20000, ftol=1e-15, gtol=1e-13, maxcor=50))
    phi, psi = res.x[:n], res.x[n:]
    plan_mass = (a * np.exp(phi / eps) * (K @ np.exp(psi / eps))).sum()
    return -res.fun, plan_mass


@pytest.mark.parametrize("tau", [math.inf, 0.5, 5.0])
def test_alg1_value_equals_dual_optimum(tau):
    g = O.make_grid("gl", 4, 8, 4)
    rng = np.random.default_rng(11)
    p = synth.uniform_field(rng, g.x, g.w, 8)
    q = synth.uniform_field(rng, g.x, g.w, 8, total=1.0 if math.isinf(tau) else 1.2)
    eps = 2.0  # t = 0.5: the truncated kernel is strictly positive at L = 4
    r = O.sinkhorn(p, q, g, eps, tau, T=3000)
    assert r["err"] < 1e-9 or not math.isinf(tau)
    D, plan_mass = _dual_optimum(g, p, q, eps, tau)
    # At the optimum the entropic term equals eps * (plan mass); Alg. 1 returns
    # the marginal terms only (App. C.2), so R = D* + eps * m(pi*).
    expect = D + eps * plan_mass
    assert abs(r["cost"] - expect) < 1e-7 * max(1.0, abs(expect))


def test_balanced_marginal_after_v_update():
    g, p, q = _small_pair()
    eps = 0.1
    r = O.sinkhorn(p, q, g, eps, T=25)
    np.testing.assert_allclose(r["v"] * O.heat_apply(r["u"], g, eps / 4), q, rtol=1e-12)


def test_balanced_cost_gauge_invariant():
    g, p, q = _small_pair()
    eps = 0.1
    r1 = O.sinkhorn(p, q, g, eps, T=30)
    r2 = O.sinkhorn(p, q, g, eps, T=30, normalize=False)
    assert abs(r1["cost"] - r2["cost"]) < 1e-12


def test_unbalanced_large_tau_recovers_balanced():
    g, p, q = _small_pair()
    eps = 0.1
    rb = O.sinkhorn(p, q, g, eps, T=400)
    ru = O.sinkhorn(p, q, g, eps, 1e8, T=400)
    assert abs(rb["cost"] - ru["cost"]) < 1e-6 * abs(rb["cost"])


def test_marginal_error_decreases_balanced():
    g, p, q = _small_pair()
    r = O.sinkhorn(p, q, g, 0.1, T=200, C=10)
    e = [x[1] for x in r["e_hist"]]
    assert all(e[i + 1] <= e[i] * (1 + 1e-9) for i in range(len(e) - 1))
    assert e[-1] < 1e-6


def test_early_exit():
    g, p, q = _small_pair()
    r = O.sinkhorn(p, q, g, 0.1, T=1000, delta=1e-8, C=10)
    assert r["iters"] < 1000 and r["iters"] % 10 == 0
    assert r["e_hist"][-1][1] < 1e-8


@pytest.mark.parametrize("tau", [math.inf, 1.0])
def test_divergence_properties(tau):
    g, p, q = _small_pair(qmass=1.0 if math.isinf(tau) else 1.05)
    eps = 0.1
    assert O.divergence(p, p, g, eps, tau, T=200) == 0.0
    s1 = O.divergence(p, q, g, eps, tau, T=400)
    s2 = O.divergence(q, p, g, eps, tau, T=400)
    assert s1 > 0
    assert abs(s1 - s2) < 1e-8 * abs(s1)


def test_envelope_gradient_matches_fd_at_convergence():
    g, p, q = _small_pair(nlat=10, nlon=20, L=10)
    eps = 0.2
    T = 300
    S, (rpq, rpp, rqq) = O.divergence(p, q, g, eps, T=T, return_solves=True)
    assert rpq["err"] < 1e-10 and rpp["err"] < 1e-10
    grad = O.envelope_gradient(rpq, rpp, g, eps, O.sinkhorn.__globals__["mass"](p, g),
                               O.sinkhorn.__globals__["mass"](q, g))
    rng = np.random.default_rng(7)
    a = g.area
    dirs = []
    for _ in range(4):
        z = rng.standard_normal(p.shape)
        d = p * z
        d = d - p * (a * d).sum() / (a * p).sum()   # mass-preserving
        dirs.append(d)
    fd = O.fd_directional(p, q, np.array(dirs), g, eps, T, h=1e-5)
    an = np.array([(grad * d).sum() for d in dirs])
    np.testing.assert_allclose(an, fd, rtol=2e-6, atol=1e-10)


def test_breakdown_on_literal_vmf_case():
    # App. C.4: at t = 1e-2, L = 32 the truncated kernel has a negative lobe and
    # widely separated bumps drive K v through zero within a few iterations.
    for seed in range(3):
        g, p, q, eps = _c1(seed)
        r = O.sinkhorn(p, q, g, eps, T=20)
        assert 1 <= int(r["breakdown"]) <= 5
        r = O.sinkhorn(p, p, g, eps, T=20)
        assert int(r["breakdown"]) == 0


def test_batched_matches_single():
    g, p, q = _small_pair()
    P = np.stack([p, q])
    Q = np.stack([q, p])
    rb = O.sinkhorn(P, Q, g, 0.1, T=20)
    r0 = O.sinkhorn(p, q, g, 0.1, T=20)
    np.testing.assert_allclose(rb["cost"][0], r0["cost"], rtol=1e-13)


# ---------------------------------------------------------------------------
# Marginal error, kernel ratio and the unbalanced branch against quantities
# computed without the oracle's own iteration bookkeeping.
# ---------------------------------------------------------------------------
def _dense_H(g, eps):
    K = O.dense_heat_matrix(g, eps / 4)          # (K v)_i = sum_j H_ij a_j v_j
    a = g.area.ravel()
    return K / a[None, :], a


@pytest.mark.parametrize("tau,T", [(math.inf, 10), (math.inf, 7), (1.0, 10)])
def test_emarg_is_the_dense_plan_marginal_error(tau, T):
    """App. C.2-C.3: with scalings u, v the plan has density pi_ij = u_i H_ij v_j
    with respect to a (x) a (H the dense radial kernel of Prop. 3.4), so its first
    marginal density is sum_j pi_ij a_j.  e_marg is the relative L2 distance of
    that marginal to p; the oracle's report at iteration k (history) and at the
    end must equal it for the scalings of that iteration."""
    g, p, q = _small_pair(qmass=1.0 if math.isinf(tau) else 1.05)
    eps = 0.2
    H, a = _dense_H(g, eps)

    def dense_err(r):
        pi = r["u"].ravel()[:, None] * H * r["v"].ravel()[None, :]
        marg = pi @ a
        return np.linalg.norm(marg - p.ravel()) / np.linalg.norm(p.ravel())

    r = O.sinkhorn(p, q, g, eps, tau, T=T, C=5)
    e = dense_err(r)
    assert e > 1e-8                       # not at the rounding floor: the comparison has teeth
    assert abs(r["err"] - e) <= 1e-10 * e
    r5 = O.sinkhorn(p, q, g, eps, tau, T=5, C=5)
    assert r["e_hist"][0][0] == 5
    assert abs(r["e_hist"][0][1] - dense_err(r5)) <= 1e-10 * dense_err(r5)
    if T % 5 == 0:
        assert r["e_hist"][-1][1] == r["err"]


def test_kernel_ratio_history_is_min_over_dense_outputs():
    """kratio_hist[k-1] is the smaller of min(K v)/max(K v) and min(K u)/max(K u)
    of iteration k (App. C.4's positivity margin), here with K applied as the
    dense matrix to scalings carried along by plain NumPy; kratio is the
    minimum of the history."""
    g, p, q = _small_pair()
    eps = 0.2
    H, a = _dense_H(g, eps)
    K = H * a[None, :]
    T = 4
    r = O.sinkhorn(p, q, g, eps, T=T)
    pp, qq = p.ravel(), q.ravel()
    v = np.ones_like(pp)
    hist = []
    for _ in range(T):
        Kv = K @ v
        u = pp / Kv
        Ku = K @ u
        v = qq / Ku
        s = u.sum()
        v = v * s
        hist.append(min(Kv.min() / Kv.max(), Ku.min() / Ku.max()))
    np.testing.assert_allclose(np.array(r["kratio_hist"], dtype=float), hist, rtol=1e-12)
    assert r["kratio"] == min(r["kratio_hist"])


def test_kernel_ratio_crosses_zero_at_the_breakdown_iteration():
    """On the literal 32x64 vMF case the first iteration whose ratio is <= 0 (or
    -inf) is exactly the reported breakdown iteration."""
    for seed in range(3):
        g, p, q, eps = _c1(seed)
        r = O.sinkhorn(p, q, g, eps, T=8)
        kb = int(r["breakdown"])
        hist = np.array(r["kratio_hist"], dtype=float)
        assert kb >= 1
        assert np.all(hist[:kb - 1] > 0) and hist[kb - 1] <= 0


def _constant_fixed_point(alpha, beta, eps, tau):
    """Alg. 1's unbalanced branch on constant densities alpha/(4 pi), beta/(4 pi).

    K maps a constant to itself (h_0 = 1; the quadrature integrates constants
    exactly), so all iterates are constants.  In logarithms x = log u, y = log v,
    with lam = tau/(tau+eps), eta = eps/tau, A = log(alpha/4pi), B = log(beta/4pi):
    the updates give x^ = lam (A - y), y^ = lam (B - x^); the translation
    c = tau/2 (log(alpha e^{-eta x^}) - log(beta e^{-eta y^})) then sets
    x - y = log(alpha/beta)/eta =: D and leaves x + y = x^ + y^ =: s.  Hence
    s_new = lam (1-lam) (A - (s_old - D)/2) + lam B, a contraction with factor
    lam (1-lam)/2 <= 1/8 whose fixed point is
    s* = (lam (1-lam) (A + D/2) + lam B) / (1 + lam (1-lam)/2).
    Returns the cost tau (1 - e^{-eta x*}) alpha + tau (1 - e^{-eta y*}) beta and x*, y*."""
    lam, eta = tau / (tau + eps), eps / tau
    A, B = math.log(alpha / (4 * math.pi)), math.log(beta / (4 * math.pi))
    D = math.log(alpha / beta) / eta
    s = (lam * (1 - lam) * (A + D / 2) + lam * B) / (1 + lam * (1 - lam) / 2)
    x, y = (s + D) / 2, (s - D) / 2
    return tau * (1 - math.exp(-eta * x)) * alpha + tau * (1 - math.exp(-eta * y)) * beta, x, y


@pytest.mark.parametrize("eps,tau", [(0.1, 0.1), (0.1, 1.0), (0.4, 10.0), (0.2, 5.0)])
def test_unbalanced_branch_on_constant_densities_closed_form(eps, tau):
    """The unbalanced exponent, gauge translation, potentials and returned cost
    (Alg. 1, App. C.2) against the closed-form fixed point of the constant case.
    The mass term of Def. 2.3 is retyped here from its definition; positivity
    does not constrain its coefficient (the bracket alone is already positive
    for constants), so that coefficient stays parity-unpinned."""
    g = O.make_grid("gl", 8, 16, 8)
    ones = np.ones(g.field_shape)
    for alpha, beta in ((1.0, 1.05), (0.7, 1.3), (1.2, 1.2)):
        p, q = ones * alpha / (4 * math.pi), ones * beta / (4 * math.pi)
        r = O.sinkhorn(p, q, g, eps, tau, T=60)
        R, x, y = _constant_fixed_point(alpha, beta, eps, tau)
        np.testing.assert_allclose(r["phi"], eps * x, rtol=1e-11, atol=1e-13)
        np.testing.assert_allclose(r["psi"], eps * y, rtol=1e-11, atol=1e-13)
        assert abs(r["cost"] - R) <= 1e-11 * abs(R)
    S = O.divergence(ones * 0.7 / (4 * math.pi), ones * 1.3 / (4 * math.pi), g, eps, tau, T=60)
    R_ab = _constant_fixed_point(0.7, 1.3, eps, tau)[0]
    R_aa = _constant_fixed_point(0.7, 0.7, eps, tau)[0]
    R_bb = _constant_fixed_point(1.3, 1.3, eps, tau)[0]
    expect = R_ab - 0.5 * (R_aa + R_bb) + 0.5 * eps * (0.7 - 1.3) ** 2
    assert abs(S - expect) <= 1e-10 * abs(expect)


@pytest.mark.parametrize("eps,tau", [(0.1, 0.1), (0.4, 10.0)])
def test_unbalanced_gauge_translation_transient_on_constants(eps, tau):
    """The translation of App. C.2 vanishes at the fixed point, so it is pinned on
    the first iterations: on constants it sets x - y = log(alpha/beta)/eta and
    keeps x + y = x^ + y^ (derivation in _constant_fixed_point), which gives the
    iterates in closed form step by step from v_0 = 1."""
    g = O.make_grid("gl", 8, 16, 8)
    ones = np.ones(g.field_shape)
    alpha, beta = 0.8, 1.1
    lam, eta = tau / (tau + eps), eps / tau
    A, B = math.log(alpha / (4 * math.pi)), math.log(beta / (4 * math.pi))
    D = math.log(alpha / beta) / eta
    y = 0.0
    for T in range(1, 4):
        xh = lam * (A - y)
        yh = lam * (B - xh)
        x, y = (xh + yh + D) / 2, (xh + yh - D) / 2
        r = O.sinkhorn(ones * alpha / (4 * math.pi), ones * beta / (4 * math.pi), g, eps, tau, T=T)
        np.testing.assert_allclose(r["phi"], eps * x, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(r["psi"], eps * y, rtol=1e-12, atol=1e-14)
