"""Full-size parity against stored oracle references.

The references in tests/golden/oracle_*.json were written by
tests/golden/make_oracle_refs.py, which runs only the float64 oracle on the
seeded inputs that these tests regenerate (the oracle needs minutes to hours
for these sizes).  Each test runs the HIP path in the launch configuration the
benchmark times and grades it with tests/parity.py: status against the
oracle's on every solve, values on solves outside the kernel-ratio margin.
Divergences are graded at the stated bounds (1e-4 relative in float32, 1e-10 in
float64) when every solve of the pair is graded; every test prints the achieved
errors next to the bounds.
"""

import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2605_18389_amd import synth

from helpers import announce, ensure_built, to_dev, to_np
from parity import BASE, check_status, report, s_bound, tolerance, well_conditioned

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module", autouse=True)
def _built():
    ensure_built()


def _ref(case):
    with open(os.path.join(GOLDEN, f"oracle_{case}.json")) as f:
        return json.load(f)


def _plan(grids, precision, legendre="recurrence"):
    from paper_2605_18389_amd import Plan
    return Plan(grids, precision=precision, legendre=legendre)


def grade_pair(name, S, info, pr, prec, S_bound=None):
    """Status of the three solves, their costs, and S.  Returns (graded, achieved S error)."""
    graded = [check_status(inf, r, prec) for inf, r in zip(info, pr["solves"])]
    for tag, inf, r, gr in zip(("pq", "pp", "qq"), info, pr["solves"], graded):
        err = abs(inf["cost"] - r["cost"]) / abs(r["cost"])
        tol = tolerance(r, prec)
        print(f"  {name} {tag}: graded={gr} kratio={r['kratio']:.3e} breakdown gpu/oracle="
              f"{inf['breakdown_iter']}/{r['breakdown']} cost err {err:.2e} (bound {tol:.1e})", flush=True)
        if gr:
            assert err <= tol, (tag, err, tol)
    Serr = None
    if all(graded):
        bound = s_bound(pr["solves"], pr["S"], prec) if S_bound is None else S_bound
        Serr = abs(S - pr["S"]) / abs(pr["S"])
        print(f"  {name} S={S:.12e} oracle={pr['S']:.12e} rel err {Serr:.2e} (bound {bound:.0e})", flush=True)
        report(name, S=S, S_ref=pr["S"], S_err=Serr, bound=bound)
        assert Serr <= bound
    return graded, Serr


def grade_potentials(name, phi, psi, r, idx, eps, prec):
    """Potentials at the sample points: |phi - phi_ref| / eps is the relative error of u."""
    tol = tolerance(r, prec)
    for tag, got, ref in (("phi", phi, r["phi_sample"]), ("psi", psi, r["psi_sample"])):
        d = np.abs(to_np(got).ravel()[idx] - np.asarray(ref)) / eps
        print(f"  {name} {tag}: max |d|/eps {d.max():.2e} (bound {tol:.1e})", flush=True)
        assert d.max() <= tol


GL180_FORMS = [("fp32", "recurrence"), ("fp32", "table"), ("fp64", "recurrence")]


@pytest.mark.parametrize("prec,legendre", GL180_FORMS)
@pytest.mark.parametrize("k", [0, 1], ids=["balanced", "unbalanced"])
def test_gl180_resolved_divergence(k, prec, legendre):
    """180x360 temperature-like pair at t = 1e-2, T = 500: balanced, and unbalanced
    with tau = 1 and masses 1 vs 1.05.  All three solves stay clear of the
    breakdown, so S is graded at the stated bound; the potentials of the cross
    solve are compared at the sample points."""
    ref = _ref("gl180_temperature_t1e-2")
    pr = ref["pairs"][k]
    tau = math.inf if pr["tau"] is None else pr["tau"]
    announce(f"gl180 t=1e-2 tau={tau} {prec} {legendre}")
    grid = tuple(ref["grid"])
    g = O.make_grid(*grid)
    p, q = synth.temperature_pair(pr["seed"], g.x, g.w, g.nlon, K=8, q_mass=pr["q_mass"])
    P = _plan([grid], prec, legendre)
    pd, qd = to_dev(p, P.dtype), to_dev(q, P.dtype)
    S, info = P.divergence(pd, qd, ref["eps"], tau, T=ref["T"])
    graded, _ = grade_pair(f"gl180 {prec} {legendre} tau={tau}", S[0], info, pr, prec)
    assert all(graded)
    phi, psi, inf = P.sinkhorn(pd, qd, ref["eps"], tau, T=ref["T"])
    grade_potentials("gl180 pq", phi, psi, pr["solves"][0], np.asarray(ref["sample_idx"]), ref["eps"], prec)


CC721 = ("cc", 721, 1440, 720)


@pytest.mark.parametrize("prec,legendre", [("fp32", "recurrence"), ("fp64", "recurrence"),
                                           ("bf16x3", "recurrence")])
def test_cc721_resolved_divergence(prec, legendre):
    """0.25-degree grid (721 x 1440, L = 720), the 32-anomaly pair at t = 1e-2, T = 100:
    a heat time at which all three solves stay clear of the breakdown (kernel ratios
    5e-3 and above).  The three solves advance together, as the benchmark runs them."""
    ref = _ref("cc721_temperature_t1e-2")
    pr = ref["pairs"][0]
    announce(f"CC721 t=1e-2 {prec} {legendre}")
    g = O.make_grid(*CC721)
    p, q = synth.temperature_pair(pr["seed"], g.x, g.w, g.nlon, K=32)
    P = _plan([CC721], prec, legendre)
    pd, qd = to_dev(p, P.dtype), to_dev(q, P.dtype)
    S, info = P.divergence(pd, qd, ref["eps"], T=ref["T"])
    graded, _ = grade_pair(f"CC721 {prec}", S[0], info, pr, prec)
    assert all(graded)
    phi, psi, _ = P.sinkhorn(pd, qd, ref["eps"], T=ref["T"])
    grade_potentials("CC721 pq", phi, psi, pr["solves"][0], np.asarray(ref["sample_idx"]), ref["eps"], prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_cc721_runtime_workload_divergence(prec):
    """The paper's runtime workload on the 0.25-degree grid: two i.i.d. uniform fields
    normalised by the area weights, eps = 0.1, balanced, T = 100.  S (4.8e-6) is about
    45 000 times smaller than each cost, so float32 fields cannot carry it to 1e-4
    relative (that needs 2e-9 per cost); float32 is held to the rounding of the costs
    instead, |dS| <= 10 u (|R_pq| + (|R_pp| + |R_qq|)/2), and float64 to 1e-10."""
    ref = _ref("cc721_uniform_eps0.1")
    pr = ref["pairs"][0]
    announce(f"CC721 uniform eps=0.1 {prec}")
    g = O.make_grid(*CC721)
    p, q = synth.uniform_pair_at(pr["seed"], g.area)
    P = _plan([CC721], prec, "recurrence")
    S, info = P.divergence(to_dev(p, P.dtype), to_dev(q, P.dtype), ref["eps"], T=ref["T"])
    bound = None
    if prec == "fp32":
        from parity import U
        R = [abs(s["cost"]) for s in pr["solves"]]
        bound = 10 * U["fp32"] * (R[0] + 0.5 * (R[1] + R[2])) / abs(pr["S"])
    graded, err = grade_pair(f"CC721 uniform {prec}", S[0], info, pr, prec, S_bound=bound)
    assert all(graded) and err is not None


UNEVEN_GRIDS = [("gl", 90, 180, 90), ("gl", 180, 360, 180), ("gl", 360, 720, 360)]
UNEVEN_COUNTS = [96, 96, 64]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_uneven256_batch_subset(prec):
    """The whole uneven batch (256 pairs on three grids, 768 solves advanced together,
    one divergence call, Legendre shapes from the autotuner, T = 300) in the launch
    configuration the benchmark times; 23 of its pairs -- per grid and per kind
    (balanced, tau = 0.1, 1, 10) the first pair drawn and the best resolved -- are
    compared with the oracle: status of every solve, costs and S of pairs outside the
    margin (tests/parity.py s_bound: for float32 the stated bound when every solve
    is at least 10x above the margin, else the summed cost tolerances)."""
    ref = _ref("uneven256_subset")
    announce(f"uneven256 uneven batch {prec}")
    P = _plan(UNEVEN_GRIDS, prec, "recurrence")
    goi = sum(([k] * c for k, c in enumerate(UNEVEN_COUNTS)), [])
    for k, c in enumerate(UNEVEN_COUNTS):
        P.autotune(k, 3 * c)
    prm = synth.batch_pair_params(synth.pair_seed(3, 0), len(goi))
    gs = [O.make_grid(*gr) for gr in UNEVEN_GRIDS]
    ps, qs = [], []
    for i, k in enumerate(goi):
        p, q = synth.temperature_pair(synth.pair_seed(3, i), gs[k].x, gs[k].w, gs[k].nlon, K=8, q_mass=prm[i][2])
        ps.append(p.ravel())
        qs.append(q.ravel())
    pd = to_dev(np.concatenate(ps), P.dtype)
    qd = to_dev(np.concatenate(qs), P.dtype)
    S, info = P.divergence(pd, qd, [4 * t for t, _, _ in prm], [tt for _, tt, _ in prm], T=ref["T"],
                           grid_of_pair=goi)
    n_graded = n_stated = 0
    for pr in ref["pairs"]:
        i = pr["index"]
        assert goi[i] == pr["grid"] and abs(prm[i][0] - pr["t"]) < 1e-15
        inf = info[3 * i:3 * i + 3]
        graded, err = grade_pair(f"uneven256 pair {i} grid {pr['grid']} t={pr['t']:.2e} tau={pr['tau']}", S[i], inf, pr,
                                 prec)
        if all(graded):
            n_graded += 1
            n_stated += well_conditioned(pr["solves"], prec)
    print(f"  uneven256 {prec}: {n_graded} of {len(ref['pairs'])} pairs value-graded, {n_stated} at the stated S bound",
          flush=True)
    assert n_graded >= 10


@pytest.mark.parametrize("prec", ["bf16x3", "bf16"])
def test_gl180_matrix_core_forms(prec):
    """The 180x360 pair at t = 1e-2 on the bfloat16 forms of the recurrence path: status
    against the oracle on every solve; values where the margin allows."""
    ref = _ref("gl180_temperature_t1e-2")
    for pr in ref["pairs"]:
        tau = math.inf if pr["tau"] is None else pr["tau"]
        announce(f"gl180 {prec} tau={tau}")
        grid = tuple(ref["grid"])
        g = O.make_grid(*grid)
        p, q = synth.temperature_pair(pr["seed"], g.x, g.w, g.nlon, K=8, q_mass=pr["q_mass"])
        P = _plan([grid], prec, "recurrence")
        S, info = P.divergence(to_dev(p, P.dtype), to_dev(q, P.dtype), ref["eps"], tau, T=ref["T"])
        grade_pair(f"gl180 {prec} tau={tau}", S[0], info, pr, prec)


GL360 = ("gl", 360, 720, 360)


def _gl360_pairs(P, idx):
    x, w = P.grid_nodes(0)
    ps, qs = [], []
    for i in idx:
        p, q = synth.temperature_pair(synth.pair_seed(4, i), x, w, GL360[2], K=8)
        ps.append(p)
        qs.append(q)
    return np.stack(ps), np.stack(qs)


def _grade_gradient(name, G, p, fdref, a, idx_sample, tol):
    """Directional derivatives of the adjoint along the stored mass-preserving
    directions against the oracle's central differences, relative to the largest."""
    D = synth.mass_preserving_directions(fdref["direction_seed"], p, a, fdref["ndir"])
    an = np.array([(G * d).sum() for d in D])
    fd = np.asarray(fdref["fd"])
    err = np.abs(an - fd).max() / np.abs(fd).max()
    print(f"  {name}: directional derivatives {an} vs oracle FD {fd}: rel err {err:.2e} (bound {tol:.1e})",
          flush=True)
    assert err <= tol, (an, fd)
    return err


def _grade_envelope(name, Genv, a, fdref, idx_sample, tol):
    """Envelope gradient (Sec. 4.2.2) as the centred field dS/dp / a at the sampled points."""
    c = Genv / a
    c = c - (a * c).sum() / a.sum()
    ref = np.asarray(fdref["envelope_centred_sample"])
    err = np.abs(c.ravel()[idx_sample] - ref).max() / np.abs(ref).max()
    print(f"  {name}: envelope field at {len(ref)} points, rel err {err:.2e} (bound {tol:.1e})", flush=True)
    assert err <= tol
    return err


def test_gl360_batch16_fp32_status_and_values():
    """The 16-pair 360x720 divergence + gradient (t = 1e-3, T = 300) in float32 in the
    launch configuration the benchmark times: every solve's status against the
    oracle's, and values (costs, S where every solve is graded) outside the margin.
    At t = 1e-3 the cross solves sit far below the float32 margin (kernel ratios
    1e-7 to 1e-15), so the self solves carry the value grading; the test fails if
    fewer than 16 solves are value-graded."""
    ref = _ref("gl360_batch16_t1e-3")
    announce("gl360 batch16 fp32")
    P = _plan([GL360], "fp32")
    P.autotune(0, 48)
    p, q = _gl360_pairs(P, range(16))
    S, G, info = P.divergence_grad(to_dev(p, P.dtype), to_dev(q, P.dtype), ref["eps"], T=ref["T"])
    assert np.isfinite(to_np(G)).any()
    n_solves = 0
    for pr in ref["pairs"]:
        i = pr["index"]
        graded, _ = grade_pair(f"gl360 batch pair {i}", S[i], info[3 * i:3 * i + 3], pr, "fp32")
        n_solves += sum(graded)
    print(f"  gl360 batch16 fp32: {n_solves} of 48 solves value-graded", flush=True)
    assert n_solves >= 16


def test_gl360_batch16_fp64_gradient_against_oracle_fd():
    """Float64 adjoint (unrolled, whole history) and envelope gradient of the two
    best-conditioned pairs of the 16-pair batch against the oracle: central
    differences of the oracle's fixed-T computation along 4 mass-preserving
    directions (h = 1e-4) and the oracle's envelope field at sampled points.
    Bound: the value tolerance of the worst solve the gradient depends on, at
    least 1e-5 (the differences' truncation error, O(h^2))."""
    from parity import U
    ref = _ref("gl360_batch16_t1e-3")
    best = sorted(int(k) for k in ref["fd"])
    announce(f"gl360 batch16 fp64 gradient, pairs {best}")
    P = _plan([GL360], "fp64")
    p, q = _gl360_pairs(P, best)
    a = P.area(0)
    pd, qd = to_dev(p, P.dtype), to_dev(q, P.dtype)
    S, G, info = P.divergence_grad(pd, qd, ref["eps"], T=ref["T"])
    Se, Genv, _ = P.divergence_grad(pd, qd, ref["eps"], T=ref["T"], mode="envelope")
    G = to_np(G).reshape(p.shape)
    Genv = to_np(Genv).reshape(p.shape)
    idx = np.asarray(ref["sample_idx"])
    for k, i in enumerate(best):
        pr = next(x for x in ref["pairs"] if x["index"] == i)
        graded, _ = grade_pair(f"gl360 batch pair {i} fp64", S[k], info[3 * k:3 * k + 3], pr, "fp64")
        assert graded[0] and graded[1]
        kr = min(pr["solves"][0]["kratio"], pr["solves"][1]["kratio"])
        tol = max(1e-5, 10 * U["fp64"] / kr)
        _grade_gradient(f"pair {i} adjoint", G[k], p[k], ref["fd"][str(i)], a, idx, tol)
        _grade_envelope(f"pair {i} envelope", Genv[k], a, ref["fd"][str(i)], idx, max(1e-8, 100 * U["fp64"] / kr))


def test_gl360_pairs01_resolved_fp32_gradient():
    """Pairs 0 and 1 of the batch at t = 1e-2, where every solve stays clear of the
    breakdown at T = 300: float32 S at the stated bound, the float32 adjoint against
    the oracle's central differences (bound 2e-4: float32 rounding of the T-iteration
    computation and its reverse sweep) and the envelope field (1e-3)."""
    path = os.path.join(GOLDEN, "oracle_gl360_pairs01_t1e-2.json")
    if not os.path.exists(path):
        pytest.skip("stored oracle results for the 360x720 pairs at t = 1e-2 not written yet")
    ref = _ref("gl360_pairs01_t1e-2")
    announce("gl360 pairs 0, 1 at t = 1e-2, fp32")
    P = _plan([GL360], "fp32")
    P.autotune(0, 6)
    idx_pairs = [pr["index"] for pr in ref["pairs"]]
    p, q = _gl360_pairs(P, idx_pairs)
    a = P.area(0)
    pd, qd = to_dev(p, P.dtype), to_dev(q, P.dtype)
    S, G, info = P.divergence_grad(pd, qd, ref["eps"], T=ref["T"])
    _, Genv, _ = P.divergence_grad(pd, qd, ref["eps"], T=ref["T"], mode="envelope")
    G = to_np(G).reshape(p.shape).astype(np.float64)
    Genv = to_np(Genv).reshape(p.shape).astype(np.float64)
    sidx = np.asarray(ref["sample_idx"])
    for k, pr in enumerate(ref["pairs"]):
        i = pr["index"]
        graded, err = grade_pair(f"gl360 t=1e-2 pair {i} fp32", S[k], info[3 * k:3 * k + 3], pr, "fp32")
        assert all(graded) and err is not None
        _grade_gradient(f"pair {i} adjoint fp32", G[k], p[k], ref["fd"][str(i)], a, sidx, 2e-4)
        _grade_envelope(f"pair {i} envelope fp32", Genv[k], a, ref["fd"][str(i)], sidx, 1e-3)
