"""GPU parity on HEALPix grids (Sec. 3.3, App. C.1) against the FP64 oracle.

The library runs the same semi-naive path as on latitude-longitude grids, with
per-ring FFT lengths (4 i pixels on polar ring i, generic radix stages for
primes above 5), the rings' first-pixel longitudes, and orders m beyond a
ring's length folded modulo that length.  The oracle sums every ring
directly (no FFT, no folding), so agreement pins all three.

Tolerances as on the other grids: float64 1e-12 and float32 1e-5 relative L2
for the heat apply; Sinkhorn graded by the kernel-ratio rule of tests/parity.py.
"""

import numpy as np
import pytest

import oracle as O
from paper_2605_18389_amd import synth

from helpers import announce, ensure_built, rel_l2, to_dev, to_np
from parity import check_status, report, tolerance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _built():
    ensure_built()


def _plan(grids, precision, legendre="recurrence"):
    from paper_2605_18389_amd import Plan
    return Plan(grids, precision=precision, legendre=legendre)


# (nside, L): band limits below and above the polar rings' lengths (orders
# alias there), Nside = 7 puts ring lengths 28 = 4 x 7 through a radix-7 stage
CASES = [(1, 2), (2, 4), (2, 7), (4, 8), (4, 13), (7, 14), (8, 16), (8, 24), (16, 32)]


def _fields(g, n, seed):
    rng = np.random.default_rng(seed)
    return np.stack([synth.temperature_like_at(rng, g.pixel_z, g.pixel_phi, g.area[0], K=6)
                     for _ in range(n)])


@pytest.mark.parametrize("nside,L", CASES)
def test_ring_layout_matches_oracle(nside, L):
    announce(f"healpix layout nside={nside} L={L}")
    P = _plan([("hp", nside, L)], "fp64")
    g = O.HealpixGrid(nside, L)
    x, w = P.grid_nodes(0)
    npix, phi0 = P.ring_layout(0)
    np.testing.assert_allclose(x, g.x, rtol=0, atol=1e-15)
    assert np.array_equal(npix, g.ring_npix)
    np.testing.assert_allclose(phi0, g.ring_phi0, rtol=0, atol=1e-15)
    assert P.field_size(0) == g.npix
    np.testing.assert_allclose(w.sum(), 2.0, rtol=1e-14)


@pytest.mark.parametrize("prec,legendre,tol", [("fp64", "recurrence", 1e-12), ("fp64", "table", 1e-12),
                                               ("fp32", "recurrence", 1e-5), ("fp32", "table", 1e-5)])
@pytest.mark.parametrize("nside,L", CASES)
def test_heat_apply_matches_oracle(nside, L, prec, legendre, tol):
    announce(f"healpix heat nside={nside} L={L} {prec} {legendre}")
    P = _plan([("hp", nside, L)], prec, legendre)
    g = O.HealpixGrid(nside, L)
    v = _fields(g, 3, 10 + nside)
    t = np.array([1e-3, 1e-2, 4e-2])
    out = to_np(P.heat_apply(to_dev(v, P.dtype), t)).reshape(v.shape)
    ref = np.stack([O.heat_apply(v[i][None], g, t[i])[0] for i in range(3)])
    assert rel_l2(out, ref) < tol
    outT = to_np(P.heat_apply(to_dev(v, P.dtype), t, transpose=True)).reshape(v.shape)
    refT = np.stack([O.heat_apply(v[i][None], g, t[i], transpose=True)[0] for i in range(3)])
    assert rel_l2(outT, refT) < tol


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 1e-2)])
@pytest.mark.parametrize("nside,L", CASES)
def test_single_item_table_heat_apply_on_rings(nside, L, prec, tol):
    """One item on a ring-grid table plan: the single-item table kernel (each table row
    read once for analysis and synthesis) with ring latitudes, against the oracle."""
    announce(f"healpix single item table nside={nside} L={L} {prec}")
    P = _plan([("hp", nside, L)], prec, "table")
    g = O.HealpixGrid(nside, L)
    v = _fields(g, 1, 30 + nside)
    out = to_np(P.heat_apply(to_dev(v, P.dtype), [1e-2])).reshape(v.shape)
    ref = O.heat_apply(v[0][None], g, 1e-2)[0]
    err = rel_l2(out[0], ref)
    print(f"[healpix single item] nside={nside} L={L} {prec} rel L2 {err:.2e}", flush=True)
    assert err < tol


@pytest.mark.parametrize("nside,L", [(4, 8), (4, 13), (7, 14)])
def test_sht_coefficients_match_oracle(nside, L):
    """Packed (m, l) coefficients position by position, and the synthesis."""
    announce(f"healpix sht nside={nside} L={L}")
    P = _plan([("hp", nside, L)], "fp64")
    g = O.HealpixGrid(nside, L)
    v = _fields(g, 2, 77)
    cz = P.analysis(to_dev(v, P.dtype)).cpu().numpy().astype(np.complex128).reshape(2, -1)
    for i in range(2):
        ref = np.concatenate(O.analysis(v[i][None], g))
        np.testing.assert_allclose(cz[i], ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    rng = np.random.default_rng(5)
    coeffs = [rng.standard_normal((2, L - m)) + 1j * rng.standard_normal((2, L - m)) for m in range(L)]
    for cm in coeffs[:1]:
        cm.imag[:] = 0.0   # m = 0 coefficients of a real field are real
    packed = np.concatenate([np.stack([cm.real, cm.imag], -1) for cm in coeffs], axis=1)
    f = to_np(P.synthesis(to_dev(packed.reshape(-1), P.dtype))).reshape(2, -1)
    ref = O.synthesis(coeffs, g).reshape(2, -1)
    np.testing.assert_allclose(f, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def _grade_solves(case, info, solves, prec):
    graded = [check_status(inf, r, prec) for inf, r in zip(info, solves)]
    for name, inf, r, gr in zip(("pq", "pp", "qq"), info, solves, graded):
        report(f"{case} {name}", graded=gr, kratio=r["kratio"], oracle_breakdown=r["breakdown"],
               gpu_breakdown=inf["breakdown_iter"], cost=inf["cost"], cost_ref=r["cost"])
        if gr:
            tol = tolerance(r, prec)
            assert abs(inf["cost"] - r["cost"]) <= tol * abs(r["cost"]), (name, inf["cost"], r["cost"])
    return graded


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("tau", [np.inf, 1.0])
def test_divergence_matches_oracle(prec, tau):
    """Nside = 8, L = 16, the runtime benchmarks' eps = 0.1 (t = 0.025), 100 iterations."""
    nside, L, T, eps = 8, 16, 100, 0.1
    announce(f"healpix divergence nside={nside} {prec} tau={tau}")
    g = O.HealpixGrid(nside, L)
    p, q = synth.temperature_pair_at(synth.pair_seed(6, 0), g.pixel_z, g.pixel_phi, g.area[0], K=6,
                                     q_mass=1.0 if np.isinf(tau) else 1.05)
    P = _plan([("hp", nside, L)], prec)
    S, info = P.divergence(to_dev(p, P.dtype), to_dev(q, P.dtype), eps, tau, T=T)
    Sref, solves = O.divergence(p[None], q[None], g, eps, tau=tau, T=T, return_solves=True)
    graded = _grade_solves(f"healpix div {prec} tau={tau}", info, solves, prec)
    if all(graded):
        tol = max(tolerance(r, prec) for r in solves)
        # S is a small difference of costs: compare on the scale of the costs
        scale = max(abs(r["cost"]) for r in solves)
        assert abs(S[0] - Sref) <= tol * scale, (S[0], Sref)
        phi, psi, inf = P.sinkhorn(to_dev(p, P.dtype), to_dev(q, P.dtype), eps, tau, T=T)
        assert rel_l2(to_np(phi).reshape(-1), solves[0]["phi"].reshape(-1)) < 10 * tol


def test_divergence_gradient_fp64_matches_oracle_fd():
    nside, L, T, eps = 4, 8, 30, 0.1
    announce("healpix gradient fp64")
    g = O.HealpixGrid(nside, L)
    p, q = synth.temperature_pair_at(synth.pair_seed(6, 1), g.pixel_z, g.pixel_phi, g.area[0], K=4)
    P = _plan([("hp", nside, L)], "fp64")
    S, G, info = P.divergence_grad(to_dev(p, P.dtype), to_dev(q, P.dtype), eps, T=T)
    G = to_np(G).reshape(-1)
    a = g.area[0]
    rng = np.random.default_rng(9)
    D = []
    for _ in range(2):
        d = p * rng.standard_normal(p.shape)
        D.append(d - p * (a * d).sum() / (a * p).sum())
    D = np.stack(D)
    fd = O.fd_directional(p[None], q[None], D[:, None], g, eps, T, h=1e-4)
    an = D @ G
    np.testing.assert_allclose(an, fd, rtol=1e-7, atol=1e-7 * np.abs(fd).max())


def test_mixed_batch_healpix_and_gauss_legendre():
    """Items on a HEALPix and a Gauss-Legendre grid in one call, interleaved."""
    announce("healpix + gl batch")
    grids = [("hp", 4, 10), ("gl", 16, 32, 16)]
    P = _plan(grids, "fp64")
    gh = O.HealpixGrid(4, 10)
    gg = O.make_grid("gl", 16, 32, 16)
    goi = [0, 1, 1, 0, 0]
    rng = np.random.default_rng(21)
    items = []
    for k in goi:
        if k == 0:
            items.append(synth.temperature_like_at(rng, gh.pixel_z, gh.pixel_phi, gh.area[0], K=4))
        else:
            items.append(synth.temperature_like(rng, gg.x, gg.w, gg.nlon, K=4).ravel())
    v = np.concatenate(items)
    t = [1e-2, 2e-2, 3e-3, 5e-3, 4e-2]
    out = to_np(P.heat_apply(to_dev(v, P.dtype), t, grid_of_item=goi))
    off = 0
    for i, k in enumerate(goi):
        n = items[i].size
        if k == 0:
            ref = O.heat_apply(items[i][None], gh, t[i]).ravel()
        else:
            ref = O.heat_apply(items[i].reshape(16, 32), gg, t[i]).ravel()
        assert rel_l2(out[off:off + n], ref) < 1e-12, i
        off += n


def test_nside64_fp32():
    """The climate grid of the paper (Nside = 64, 49 152 pixels) at L = 128."""
    nside, L = 64, 128
    announce(f"healpix nside={nside} L={L} fp32")
    g = O.HealpixGrid(nside, L)
    P = _plan([("hp", nside, L)], "fp32")
    v = _fields(g, 2, 64)
    t = np.array([1e-4, 1e-3])
    out = to_np(P.heat_apply(to_dev(v, P.dtype), t)).reshape(v.shape)
    ref = np.stack([O.heat_apply(v[i][None], g, t[i])[0] for i in range(2)])
    assert rel_l2(out, ref) < 1e-5
    p, q = synth.temperature_pair_at(synth.pair_seed(6, 2), g.pixel_z, g.pixel_phi, g.area[0], K=8)
    eps, T = 4e-3, 50
    _, _, info = P.sinkhorn(to_dev(p, P.dtype), to_dev(q, P.dtype), eps, T=T)
    r = O.sinkhorn(p[None], q[None], g, eps, T=T)
    graded = check_status(info[0], r, "fp32")
    report("healpix nside64 sinkhorn", graded=graded, kratio=r["kratio"], cost=info[0]["cost"],
           cost_ref=r["cost"])
    if graded:
        assert abs(info[0]["cost"] - r["cost"]) <= tolerance(r, "fp32") * abs(r["cost"])


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_bluestein_rings_match_oracle(prec, tol):
    """Nside = 80, L = 160: the polar rings of 4p pixels with p = 67, 71, 73 and
    79 (prime factors above 64) take the Bluestein transform in both
    directions; heat apply and its transpose against the direct ring sums."""
    nside, L = 80, 160
    announce(f"healpix bluestein nside={nside} {prec}")
    P = _plan([("hp", nside, L)], prec)
    g = O.HealpixGrid(nside, L)
    v = _fields(g, 2, 80)
    t = np.array([2e-4, 3e-3])
    out = to_np(P.heat_apply(to_dev(v, P.dtype), t)).reshape(v.shape)
    ref = np.stack([O.heat_apply(v[i][None], g, t[i])[0] for i in range(2)])
    assert rel_l2(out, ref) < tol
    outT = to_np(P.heat_apply(to_dev(v, P.dtype), t, transpose=True)).reshape(v.shape)
    refT = np.stack([O.heat_apply(v[i][None], g, t[i], transpose=True)[0] for i in range(2)])
    assert rel_l2(outT, refT) < tol


_HP256 = {}


def _hp256_reference():
    """Oracle heat apply (direct ring sums) of the Nside 256 workload's first field, once."""
    if not _HP256:
        g = O.HealpixGrid(256, 512)
        p, _ = synth.uniform_pair_at(synth.pair_seed(7, 256), g.area[0])
        _HP256.update(g=g, p=p, ref=O.heat_apply(p[None], g, 0.025)[0])
    return _HP256["g"], _HP256["p"], _HP256["ref"]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_nside256_full_size_heat_apply(prec, tol):
    """The HEALPix workload of the throughput measurement at full size: Nside 256
    (786 432 pixels, 1023 rings, polar rings through the Bluestein transform), L = 512,
    t = eps / 4 = 0.025, one heat apply of its first field against the oracle."""
    announce(f"healpix nside=256 full size {prec}")
    g, p, ref = _hp256_reference()
    P = _plan([("hp", 256, 512)], prec)
    out = to_np(P.heat_apply(to_dev(p[None], P.dtype), [0.025])).reshape(ref.shape)
    assert rel_l2(out, ref) < tol, rel_l2(out, ref)
