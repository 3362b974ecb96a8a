"""Benchmark: Sinkhorn iterations/s on the 0.25-degree 721x1440 equiangular grid (L = 720).

One step = one full Alg. 1 solve (T = 1000 iterations, balanced, t = 1e-4) of a
seeded temperature-like pair (32 anomalies) already resident in HBM, through
the libshot C ABI.  Prints ONE JSON line (see --help) with, beside `value`:
* roofline: the dominant (Legendre) kernel, timed live with HIP events on its
  launch stream, with the calibrated HBM traffic of profiles/traffic.json;
* cpu_baseline: the FP64 oracle on the host cores (and on one thread), on a
  bounded sample of the same workload;
* secondary: the other Legendre forms (fp32 table, bfloat16 table, fp64,
  split bfloat16) at the same shape, the headline divergence, HEALPix and the
  climate attribution;
* companions: full-size workloads whose runs stay finite, each with its S and
  cost errors against stored oracle results (tests/golden/);
* batched: the 16-pair 360x720 divergence + gradient and the 256-pair uneven
  batch per form, with status agreement and S errors against the stored
  oracle pairs and the matrix-core kernel's roofline at the batch's shape.

Single GPU only: --gpus N with N > 1 exits with a message.
"""

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Sinkhorn iters/s at 721×1440 (FP32 vs BF16-MFMA); batched divergence+grad/s"
GRID = ("cc", 721, 1440, 720)
T_HEAT = 1e-4
ITERS = 1000
HBM_PEAK_GBS = 8000.0
VALU_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz, non-packed FP32 or FP64


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def legendre_work(grid, nitems, legendre, precision):
    """Algorithmic work of one Legendre launch (one heat apply's Legendre stage).

    Entries (l, m, j) of the folded transform: E = L(L+1)/2 * ceil(nlat/2).
    Contraction: 4 flop per entry per pass (complex x real), 2 passes (analysis,
    synthesis), per item.  Recurrence: 3 flop per entry per pass (one multiply,
    one fused multiply-add).  Table mode: the table read once per launch, the
    algorithmic minimum (the single-item kernel reads each row once for both
    passes; the batched matrix-core kernel streams it for each pass, the second
    mostly from the caches).
    """
    _, nlat, nlon, L = grid
    h = (nlat + 1) // 2
    E = L * (L + 1) // 2 * h
    flops = 2 * E * 4 * nitems
    if legendre == "recurrence":
        flops += 2 * E * 3
    tab_bytes = {"fp32": 4, "bf16": 2, "fp64": 8}[precision]
    field = 8 if precision == "fp64" else 4
    spec_bytes = nitems * 2 * L * h * 2 * field * 2      # folded spectrum in and out
    bytes_ = spec_bytes + (E * tab_bytes if legendre == "table" else 0)
    return flops, bytes_


def make_inputs(plan, torch):
    from paper_2605_18389_amd import synth
    x, w = plan.grid_nodes(0)
    p, q = synth.temperature_pair(synth.pair_seed(2, 0), x, w, GRID[2], K=32)
    dev = torch.device("cuda")
    return (torch.as_tensor(p, dtype=plan.dtype, device=dev).contiguous(),
            torch.as_tensor(q, dtype=plan.dtype, device=dev).contiguous(), p, q)


def time_solves(plan, p, q, steps, warmup, torch, profile=False):
    """Wall time of `steps` full solves (HIP graph replay unless profiling).

    With profile=True every Legendre and row-FFT launch is bracketed by HIP
    events on its launch stream (eager launches) and their summed durations
    are returned with the launch counts."""
    eps = 4 * T_HEAT
    if profile:
        plan.profile(True)
    for _ in range(warmup):
        plan.sinkhorn(p, q, eps, T=ITERS, potentials=True)
    torch.cuda.synchronize()
    if profile:
        plan.profile(True)  # reset counts after the warm-up
    t0 = time.perf_counter()
    info = None
    for _ in range(steps):
        _, _, info = plan.sinkhorn(p, q, eps, T=ITERS, potentials=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    leg = plan.profile_read(0) if profile else (0, 0.0)
    rows = plan.profile_read(1) if profile else (0, 0.0)
    if profile:
        plan.profile(False)
    return dt, info[0], leg, rows


GOLDEN = os.path.join(ROOT, "tests", "golden")


def oracle_ref(case):
    """Stored oracle results of a workload (tests/golden/oracle_<case>.json, written by
    tests/golden/make_oracle_refs.py from the oracle alone), or None."""
    try:
        with open(os.path.join(GOLDEN, f"oracle_{case}.json")) as f:
            return json.load(f)
    except (OSError, ValueError):
        return None


def rel(a, b):
    return abs(a - b) / abs(b) if b not in (0, None) and math.isfinite(b) else None


MARGIN = {"fp64": 1e-13, "fp32": 1e-5, "bf16x3": 2e-3, "bf16": 0.5}   # kernel-ratio grading margins


def pair_errors(S, info, ref_pairs, prec, index_of=lambda k, pr: k, kr_min=1e-4):
    """S and status against stored oracle pairs.

    status_equal: pairs whose three solves break down (or not) as the oracle's do;
    status_consistent: pairs where every GPU breakdown happens at an iteration at which
    the oracle's kernel ratio min(K.)/max(K.) is below the form's margin (or, when the
    oracle breaks down too, within 100x of it or at or after the oracle's breakdown):
    an output below that ratio cannot be told from zero in the form's arithmetic
    (App. C.4).  S errors: over the pairs finite on both sides, and over those whose
    three oracle solves keep a kernel ratio above kr_min (ten times the float32 margin)."""
    margin = MARGIN[prec]
    equal, consistent, errs, errs_wc = 0, 0, [], []
    for k, pr in enumerate(ref_pairs):
        i = index_of(k, pr)
        ok = True
        for g, o in zip(info[3 * i:3 * i + 3], pr["solves"]):
            kg, kb = int(g["breakdown_iter"]), int(o["breakdown"])
            if kg:
                r = float(o["kratio_hist"][kg - 1]) if kg <= len(o["kratio_hist"]) else 0.0
                ok &= r < margin or (kb > 0 and (kg >= kb or r < 100.0 * margin))
        consistent += ok
        gpu_b = [int(x["breakdown_iter"] > 0) for x in info[3 * i:3 * i + 3]]
        orc_b = [int(x["breakdown"] > 0) for x in pr["solves"]]
        equal += gpu_b == orc_b
        if not any(orc_b) and not any(gpu_b) and math.isfinite(S[i]):
            errs.append(rel(S[i], pr["S"]))
            if min(x["kratio"] for x in pr["solves"]) > kr_min:
                errs_wc.append(rel(S[i], pr["S"]))
    return {"pairs_compared": len(ref_pairs), "status_equal": equal, "status_consistent": consistent,
            "margin": margin, "finite_both": len(errs), "max_S_rel_err": max(errs) if errs else None,
            "well_conditioned": len(errs_wc), "kratio_min": kr_min,
            "max_S_rel_err_well_conditioned": max(errs_wc) if errs_wc else None}


BATCH16_GRID = ("gl", 360, 720, 360)
UNEVEN_GRIDS = [("gl", 90, 180, 90), ("gl", 180, 360, 180), ("gl", 360, 720, 360)]
UNEVEN_COUNTS = [96, 96, 64]


MFMA_PEAK = {"fp32": 157.3, "bf16x3": 2500.0 / 3, "bf16": 2500.0}   # TFLOP/s of the contraction


def batched_roofline(torch, precision, grid, nitems, tuning):
    """Roofline of the matrix-core recurrence Legendre kernel at a batch's launch shape:
    one heat apply of `nitems` items with the batch's tuning, HIP events on the launch
    stream around each of 5 launches.  Work per launch: the contraction 2 E 4 flop per
    item (complex x real, analysis + synthesis; split bfloat16 takes three products,
    so its peak is a third of the bfloat16 one), the folded spectra in and out."""
    from paper_2605_18389_amd import Plan
    P = Plan([grid], precision=precision, legendre="recurrence")
    P.set_tuning(0, *tuning)
    _, nlat, nlon, L = grid
    v = torch.rand(nitems, nlat, nlon, dtype=torch.float32, device="cuda") + 0.5
    P.heat_apply(v, [1e-3] * nitems)
    P.profile(True)
    for _ in range(5):
        P.heat_apply(v, [1e-3] * nitems)
    n, ms = P.profile_read(0)
    P.profile(False)
    avg_ms = ms / max(n, 1)
    h = (nlat + 1) // 2
    E = L * (L + 1) // 2 * h
    flops = 2 * E * 4 * nitems
    bytes_ = nitems * 2 * L * h * 2 * 8
    achieved = flops / (avg_ms * 1e-3) / 1e12
    traffic = measured_traffic("legendre_rmma_kernel") if (precision, nitems) == ("fp32", 48) else None
    return {"bound": "mfma", "achieved": achieved, "peak": MFMA_PEAK[precision], "unit": "TFLOP/s",
            "frac": achieved / MFMA_PEAK[precision], "traffic": traffic,
            "kernel": "legendre_rmma_kernel (recurrence-fed matrix-core Legendre)",
            "launch": {"grid": list(grid), "items": nitems, "tuning": list(tuning)},
            "avg_launch_ms": avg_ms, "work_per_launch": {"flop": flops, "bytes": bytes_},
            "hbm_GBps": bytes_ / (avg_ms * 1e-3) / 1e9}


def bench_grad_batch(torch, precision, legendre, reps=1):
    """16 pairs on 360x720 Gauss-Legendre, t = 1e-3, balanced, T = 300: S and dS/dp per pair
    (forward, then the hand-written adjoint with checkpoint recompute)."""
    from paper_2605_18389_amd import Plan, synth
    plan = Plan([BATCH16_GRID], precision=precision, legendre=legendre)
    plan.autotune(0, 48)
    x, w = plan.grid_nodes(0)
    ps, qs = [], []
    for i in range(16):
        p, q = synth.temperature_pair(synth.pair_seed(4, i), x, w, BATCH16_GRID[2], K=8)
        ps.append(p)
        qs.append(q)
    p = torch.as_tensor(np.stack(ps), dtype=plan.dtype, device="cuda").contiguous()
    q = torch.as_tensor(np.stack(qs), dtype=plan.dtype, device="cuda").contiguous()
    plan.divergence_grad(p, q, 4e-3, T=300)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        S, g, info = plan.divergence_grad(p, q, 4e-3, T=300)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    bad = sum(1 for i in range(16) if any(x["status"] == 17 for x in info[3 * i:3 * i + 3]))
    out = {"divergence_grad_per_s": 16 / dt, "ms_per_batch": dt * 1e3, "pairs": 16,
           "pairs_with_breakdown": bad, "tuning": plan.get_tuning(0)}
    if legendre == "recurrence" and plan.get_tuning(0)[0] >= 8:
        out["roofline"] = batched_roofline(torch, precision, BATCH16_GRID, 48, plan.get_tuning(0))
    ref = oracle_ref("gl360_batch16_t1e-3")
    if ref and len(ref["pairs"]) == 16:
        out["vs_oracle"] = pair_errors(S, info, ref["pairs"], precision)
        out["oracle_pairs_with_breakdown"] = sum(1 for pr in ref["pairs"] if any(x["breakdown"] for x in pr["solves"]))
    return out


def bench_uneven_batch(torch, precision, legendre, reps=1):
    """256 pairs on three grids (96 at 90x180, 96 at 180x360, 64 at 360x720), per-pair t
    log-uniform in [1e-4, 1e-2], half balanced and half unbalanced (tau in {0.1, 1, 10},
    masses 1 vs 1.05), T = 300, one divergence call (768 solves advanced together)."""
    from paper_2605_18389_amd import Plan, synth
    plan = Plan(UNEVEN_GRIDS, precision=precision, legendre=legendre)
    goi = sum(([k] * c for k, c in enumerate(UNEVEN_COUNTS)), [])
    for k, c in enumerate(UNEVEN_COUNTS):
        plan.autotune(k, 3 * c)
    prm = synth.batch_pair_params(synth.pair_seed(3, 0), len(goi))
    ps, qs = [], []
    for i, k in enumerate(goi):
        x, w = plan.grid_nodes(k)
        p, q = synth.temperature_pair(synth.pair_seed(3, i), x, w, UNEVEN_GRIDS[k][2], K=8, q_mass=prm[i][2])
        ps.append(p.ravel())
        qs.append(q.ravel())
    p = torch.as_tensor(np.concatenate(ps), dtype=plan.dtype, device="cuda")
    q = torch.as_tensor(np.concatenate(qs), dtype=plan.dtype, device="cuda")
    eps = [4 * t for t, _, _ in prm]
    tau = [tt for _, tt, _ in prm]
    plan.divergence(p, q, eps, tau, T=300, grid_of_pair=goi)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        S, info = plan.divergence(p, q, eps, tau, T=300, grid_of_pair=goi)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    bad = sum(1 for i in range(len(goi)) if any(x["status"] == 17 for x in info[3 * i:3 * i + 3]))
    out = {"divergences_per_s": len(goi) / dt, "ms_per_batch": dt * 1e3, "pairs": len(goi),
           "pairs_with_breakdown": bad, "tuning": [plan.get_tuning(k) for k in range(3)]}
    if legendre == "recurrence" and plan.get_tuning(2)[0] >= 8:
        out["roofline"] = batched_roofline(torch, precision, UNEVEN_GRIDS[2], 3 * UNEVEN_COUNTS[2], plan.get_tuning(2))
    ref = oracle_ref("uneven256_subset")
    if ref:
        out["vs_oracle_subset"] = pair_errors(S, info, ref["pairs"], precision, lambda k, pr: pr["index"])
    return out


def bench_companion(torch, case, precision, steps=3):
    """A stored oracle workload at full size: divergence (three solves advanced together)
    per second, S against the oracle, statuses; unbalanced pairs also report the fixed-point
    residual max |phi_T - phi_(T-C)| (C = 10) of the cross solve."""
    from paper_2605_18389_amd import Plan, synth
    ref = oracle_ref(case)
    if ref is None:
        return {"error": f"no stored oracle results for {case}"}
    grid = tuple(ref["grid"])
    plan = Plan([grid], precision=precision, legendre="recurrence")
    x, w = plan.grid_nodes(0)
    out = {}
    for k, pr in enumerate(ref["pairs"]):
        tau = math.inf if pr.get("tau") is None else pr["tau"]
        if case == "cc721_uniform_eps0.1":
            p, q = synth.uniform_pair_at(pr["seed"], plan.area(0))
        else:
            p, q = synth.temperature_pair(pr["seed"], x, w, grid[2], K=32 if grid[1] == 721 else 8,
                                          q_mass=pr.get("q_mass", 1.0))
        pd = torch.as_tensor(p, dtype=plan.dtype, device="cuda").contiguous()
        qd = torch.as_tensor(q, dtype=plan.dtype, device="cuda").contiguous()
        T = ref["T"]
        plan.divergence(pd, qd, ref["eps"], tau, T=T)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            S, info = plan.divergence(pd, qd, ref["eps"], tau, T=T)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        r = {"divergences_per_s": 1 / dt, "solve_iterations_per_s": 3 * T / dt, "T": T,
             "S": S[0], "S_oracle": pr["S"], "S_rel_err": rel(S[0], pr["S"]),
             "status": [x["status"] for x in info], "oracle_breakdown": [x["breakdown"] for x in pr["solves"]],
             "cost_rel_err": [rel(x["cost"], y["cost"]) for x, y in zip(info, pr["solves"])]}
        if not math.isinf(tau):
            C = 10
            phiT, _, _ = plan.sinkhorn(pd, qd, ref["eps"], tau, T=T, C=C)
            phiC, _, _ = plan.sinkhorn(pd, qd, ref["eps"], tau, T=T - C, C=C)
            r["fixed_point_residual"] = float((phiT - phiC).abs().max())
            r["fixed_point_residual_note"] = "max |phi_T - phi_(T-10)| = eps max |log(u_T / u_(T-10))|"
        out["balanced" if math.isinf(tau) else f"tau{tau:g}"] = r
    return out


def bench_healpix(torch, nside, precision, T=200):
    """The runtime workload on HEALPix: a pair of uniform random probability
    measures (normalised by the pixel areas), eps = 0.1, balanced, band limit
    L = 2 Nside; Sinkhorn iterations per second (graph replay)."""
    from paper_2605_18389_amd import Plan, synth
    L = 2 * nside
    plan = Plan([("hp", nside, L)], precision=precision, legendre="recurrence")
    p, q = synth.uniform_pair_at(synth.pair_seed(7, nside), plan.area(0))
    p = torch.as_tensor(p, dtype=plan.dtype, device="cuda")
    q = torch.as_tensor(q, dtype=plan.dtype, device="cuda")
    plan.sinkhorn(p, q, 0.1, T=T)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, info = plan.sinkhorn(p, q, 0.1, T=T)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"iterations_per_s": T / dt, "pixels": 12 * nside * nside, "L": L,
            "status": info[0]["status"], "kratio": info[0]["kratio"]}


def bench_climate_attribution(torch, precision, npairs=8, T=300):
    """The climate study's computation on synthetic fields: npairs pairs on HEALPix
    Nside 64 (L = 128), eps = 0.01, tau = 100 (unbalanced, masses 1 vs 1.05), T
    iterations; per pair the divergence, its exact gradient and the five regional
    RMS indices.  Pairs (with attribution) per second."""
    from paper_2605_18389_amd import Plan, synth
    nside, L = 64, 128
    plan = Plan([("hp", nside, L)], precision=precision, legendre="recurrence")
    z, phi = plan.pixel_coords(0)
    area = plan.area(0)
    ps, qs = [], []
    for i in range(npairs):
        p, q = synth.temperature_pair_at(synth.pair_seed(8, i), z, phi, area, K=8, q_mass=1.05)
        ps.append(p)
        qs.append(q)
    p = torch.as_tensor(np.concatenate(ps), dtype=plan.dtype, device="cuda")
    q = torch.as_tensor(np.concatenate(qs), dtype=plan.dtype, device="cuda")

    def once():
        S, g, info = plan.divergence_grad(p, q, 0.01, T=T, tau=100.0)
        return S, plan.regional_rms(g), info

    once()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S, rms, info = once()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"pairs_per_s": npairs / dt, "ms_per_batch": dt * 1e3, "pairs": npairs,
            "pairs_with_breakdown": sum(1 for i in range(npairs)
                                        if any(x["status"] == 17 for x in info[3 * i:3 * i + 3]))}


def cpu_baseline(budget_s, gpu_heat=None, one_thread_budget_s=0.0):
    """FP64 oracle on host cores: iterations/s of Alg. 1 on the same workload.

    With gpu_heat ({name: K p computed by a GPU plan}) also returns each
    plan's relative L2 error against the oracle's heat apply of the same p.
    With one_thread_budget_s > 0 the oracle is also timed with BLAS limited to
    one thread."""
    import oracle as O
    from paper_2605_18389_amd import synth
    try:
        from threadpoolctl import threadpool_info
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    g = O.make_grid(*GRID)
    p, q = synth.temperature_pair(synth.pair_seed(2, 0), g.x, g.w, GRID[2], K=32)
    Kp = O.heat_apply(p, g, T_HEAT)  # also builds the Legendre table (plan time, excluded)
    errors = {}
    for name, got in (gpu_heat or {}).items():
        got = np.asarray(got, dtype=np.float64).reshape(Kp.shape)
        errors[name] = float(np.linalg.norm(got - Kp) / np.linalg.norm(Kp))
    t0 = time.perf_counter()
    n = 1
    O.sinkhorn(p, q, g, 4 * T_HEAT, T=n)
    one = time.perf_counter() - t0
    n = max(2, int(budget_s / max(one, 1e-3)))
    t0 = time.perf_counter()
    O.sinkhorn(p, q, g, 4 * T_HEAT, T=n)
    dt = time.perf_counter() - t0
    res = {"value": n / dt, "unit": "iterations/s", "cores": int(threads), "kind": "oracle",
           "sample": f"{n} Alg. 1 iterations (2 heat applies each) of the 721x1440 pair, "
                     f"float64 NumPy, Legendre table built beforehand"}
    if one_thread_budget_s > 0:
        try:
            from threadpoolctl import threadpool_limits
            with threadpool_limits(limits=1):
                t0 = time.perf_counter()
                O.sinkhorn(p, q, g, 4 * T_HEAT, T=1)
                one = time.perf_counter() - t0
                n1 = max(1, int(one_thread_budget_s / max(one, 1e-3)))
                t0 = time.perf_counter()
                O.sinkhorn(p, q, g, 4 * T_HEAT, T=n1)
                d1 = time.perf_counter() - t0
            res["one_thread"] = {"value": n1 / d1, "unit": "iterations/s", "cores": 1,
                                 "sample": f"{n1} iterations, BLAS limited to one thread"}
        except Exception as e:
            res["one_thread"] = {"error": str(e)}
    return res, errors


KERNEL_SRC = os.path.join(ROOT, "paper_2605_18389_amd", "csrc", "kernels.hip")
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")
COPY_BYTES = 1 << 30          # calibration copy: 1 GiB read + 1 GiB written
LEG_KERNEL = "legendre_split_kernel"


def kernel_source_hash():
    import hashlib
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_probe():
    """Short program for the two `rocprofv3 --pmc` passes (FETCH_SIZE, then
    WRITE_SIZE): one device-to-device copy of COPY_BYTES (the calibration
    kernel of known traffic), then eager solves of the benchmark workload."""
    import torch
    from paper_2605_18389_amd import Plan, load_library
    load_library()
    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    plan = Plan([GRID], precision="fp32", legendre="recurrence")
    plan.set_graphs(False)
    p, q, _, _ = make_inputs(plan, torch)
    for _ in range(2):
        plan.sinkhorn(p, q, 4 * T_HEAT, T=10, potentials=True)
    torch.cuda.synchronize()
    # the matrix-core recurrence kernel at the 16-pair batch's forward shape
    bp = Plan([BATCH16_GRID], precision="fp32", legendre="recurrence")
    bp.set_tuning(0, 8, 0)
    v = torch.rand(48, BATCH16_GRID[1], BATCH16_GRID[2], dtype=torch.float32, device="cuda") + 0.5
    for _ in range(3):
        bp.heat_apply(v, [1e-3] * 48)
    torch.cuda.synchronize()
    del bp, v
    # one item on bfloat16 and float32 tables (the single-item table kernel)
    for prec in ("bf16", "fp32"):
        tp = Plan([GRID], precision=prec, legendre="table")
        tp.set_graphs(False)
        pt, _, _, _ = make_inputs(tp, torch)
        for _ in range(3):
            tp.heat_apply(pt[None], [T_HEAT])
        torch.cuda.synchronize()
        del tp
    print("traffic probe done", flush=True)


def pmc_summary(fetch_dir, write_dir, command):
    """Per-launch HBM bytes of every kernel from the two counter runs, scaled
    by the ratio of the copy kernel's known traffic to its counter reading."""
    import csv
    import glob

    def load(d, counter):
        per = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] != counter:
                    continue
                per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return per

    fetch = load(fetch_dir, "FETCH_SIZE")
    write = load(write_dir, "WRITE_SIZE")

    def copy_reading(per):
        vals = [max(v) for k, v in per.items() if "copyBuffer" in k]
        if not vals:
            raise SystemExit("no copy kernel in the counter output")
        return max(vals) * 1024.0   # KiB -> bytes (largest copy = the calibration copy)

    f_fac = COPY_BYTES / copy_reading(fetch)
    w_fac = COPY_BYTES / copy_reading(write)
    kernels = {}
    for name in sorted(set(fetch) | set(write)):
        if "copyBuffer" in name or "fillBuffer" in name:
            continue
        fv, wv = fetch.get(name, []), write.get(name, [])
        kernels[name] = {"dispatches": max(len(fv), len(wv)),
                         "fetch_bytes_per_launch": f_fac * 1024.0 * sum(fv) / max(len(fv), 1),
                         "write_bytes_per_launch": w_fac * 1024.0 * sum(wv) / max(len(wv), 1)}
    out = {"command": command, "kernels_hip_sha256_16": kernel_source_hash(),
           "copy_calibration": {"bytes": COPY_BYTES, "fetch_factor": f_fac, "write_factor": w_fac},
           "kernels": kernels}
    os.makedirs(os.path.dirname(TRAFFIC_JSON), exist_ok=True)
    with open(TRAFFIC_JSON, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({"written": TRAFFIC_JSON, "fetch_factor": f_fac, "write_factor": w_fac}))


def measured_traffic(kernel_substr):
    """HBM bytes per launch of the named kernel from profiles/traffic.json, or
    None when absent or taken from another revision of the kernels."""
    try:
        with open(TRAFFIC_JSON) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernels_hip_sha256_16") != kernel_source_hash():
        return None
    hits = [v for k, v in t["kernels"].items() if kernel_substr in k and "float" in k]
    if not hits:
        return None
    v = max(hits, key=lambda x: x["dispatches"])
    return v["fetch_bytes_per_launch"] + v["write_bytes_per_launch"]


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "bf16x3", "fp64"])
    ap.add_argument("--legendre", default="recurrence", choices=["recurrence", "table"])
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run the short program profiled by the FETCH_SIZE / WRITE_SIZE passes")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="reduce the two counter runs to profiles/traffic.json")
    ap.add_argument("--pmc-command", default="", help="command line recorded in profiles/traffic.json")
    ap.add_argument("--only", choices=["grad16", "uneven256"],
                    help="run one batched workload at --precision / --legendre and print its entry "
                         "(the command the batched kernel profiles are taken over)")
    args = ap.parse_args()
    if args.pmc_summary:
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.pmc_command)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; sharding the path "
                                   "over several GPUs is designed but not built", "n_gpus": args.gpus}))
        sys.exit(2)

    if args.traffic_probe:
        traffic_probe()
        return
    if args.only:
        import torch
        fn = bench_grad_batch if args.only == "grad16" else bench_uneven_batch
        print(json.dumps({args.only: fn(torch, args.precision, args.legendre)}), flush=True)
        return

    import torch
    from paper_2605_18389_amd import Plan, load_library
    load_library()
    log(f"[bench] plan {GRID} {args.precision} {args.legendre}")
    plan = Plan([GRID], precision=args.precision, legendre=args.legendre)
    p, q, _, _ = make_inputs(plan, torch)
    log("[bench] timing")
    dt, info, _, _ = time_solves(plan, p, q, args.steps, args.warmup, torch)
    ms_step = dt / args.steps * 1e3
    value = args.steps * ITERS / dt
    log("[bench] kernel timing (HIP events per launch)")
    dtp, _, leg, rows = time_solves(plan, p, q, args.steps, 0, torch, profile=True)
    launches, leg_ms = leg
    avg_leg_ms = leg_ms / max(launches, 1)
    flops, bytes_ = legendre_work(GRID, 1, args.legendre, args.precision)
    if args.legendre == "recurrence":
        achieved = flops / (avg_leg_ms * 1e-3) / 1e12
        traffic = measured_traffic(LEG_KERNEL) if args.precision == "fp32" else None
        roof = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / VALU_PEAK_TFLOPS, "traffic": traffic}
    else:
        achieved = bytes_ / (avg_leg_ms * 1e-3) / 1e9
        tt = "unsigned short," if args.precision == "bf16" else "float,"
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": measured_traffic(f"legendre_gemv_kernel<float, {tt}")
                if args.precision in ("bf16", "fp32") else None}
    roof.update({"kernel": "legendre (per-order analysis + h_l + synthesis)",
                 "avg_launch_ms": avg_leg_ms, "launches": launches,
                 "timing": f"HIP events around every launch on its stream during {args.steps} further "
                           f"timed solves launched eagerly ({dtp / args.steps * 1e3:.1f} ms/step); "
                           f"`value` is from HIP-graph replay",
                 "work_per_launch": {"flop": flops, "bytes": bytes_},
                 "row_fft_avg_launch_ms": rows[1] / max(rows[0], 1)})
    if args.legendre == "recurrence":
        # the other counting: 4 flop per entry and pass for the recurrence at the
        # float64 peak plus the contraction at the packed-float32 peak
        _, nlat_, _, L_ = GRID
        E = L_ * (L_ + 1) // 2 * ((nlat_ + 1) // 2)
        ideal_us = (2 * E * 4 / 78.6e12 + 2 * E * 4 / 157.3e12) * 1e6
        roof["alt_counting"] = {"recurrence_fp64_flop": 2 * E * 4, "contraction_fp32_flop": 2 * E * 4,
                                "ideal_us": ideal_us, "frac": ideal_us / (avg_leg_ms * 1e3),
                                "note": "the kernel contracts in float64 (same issue rate as unpacked float32)"}
    out = {
        "metric": METRIC, "value": value, "unit": "iterations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16", "bf16x3": "bf16x3", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "sinkhorn_cc721x1440_L720_t1e-4_balanced_T1000",
                   "grid": "Clenshaw-Curtis 721x1440", "L": 720, "iterations_per_step": ITERS,
                   "legendre": args.legendre, "precision": args.precision,
                   "fields": "temperature-like pair, 32 vMF anomalies, seed 2000"},
        "status": {"code": info["status"], "breakdown_iter": info["breakdown_iter"],
                   "note": "Alg. 1 in scaling form breaks down on this workload in float64 as well "
                           "(truncated-kernel positivity, App. C.4); timing covers all iterations"},
        "roofline": roof,
    }
    if not args.no_secondary:
        sec = {}
        other = "table" if args.legendre == "recurrence" else "recurrence"
        for prec, legm in ((args.precision, other), ("bf16", "table"), ("fp64", "recurrence"),
                           ("bf16x3", "recurrence")):
            if (prec, legm) == (args.precision, args.legendre):
                continue
            try:
                log(f"[bench] secondary {prec} {legm}")
                pl = Plan([GRID], precision=prec, legendre=legm)
                pp, qq, _, _ = make_inputs(pl, torch)
                d2, _, _, _ = time_solves(pl, pp, qq, 2, 1, torch)
                _, _, lg, _ = time_solves(pl, pp, qq, 1, 0, torch, profile=True)
                _, _, inf2 = pl.sinkhorn(pp, qq, 4 * T_HEAT, T=ITERS, potentials=False)
                sec[f"{prec}_{legm}"] = {"iterations_per_s": 2 * ITERS / d2,
                                         "legendre_avg_launch_ms": lg[1] / max(lg[0], 1),
                                         "status": inf2[0]["status"], "breakdown_iter": inf2[0]["breakdown_iter"]}
                del pl
            except Exception as e:  # report, do not hide
                sec[f"{prec}_{legm}"] = {"error": str(e)}
        try:
            log("[bench] divergence 721x1440 (3 solves advanced together)")
            eps = 4 * T_HEAT
            plan.divergence(p, q, eps, T=ITERS)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.divergence(p, q, eps, T=ITERS)
            torch.cuda.synchronize()
            d3 = time.perf_counter() - t0
            sec["divergence_fp32_recurrence"] = {"divergences_per_s": 1 / d3,
                                                 "solve_iterations_per_s": 3 * ITERS / d3,
                                                 "ms_per_divergence": d3 * 1e3}
        except Exception as e:
            sec["divergence_fp32_recurrence"] = {"error": str(e)}
        comp = {}
        for case, precs in (("cc721_uniform_eps0.1", ("fp32", "fp64")), ("cc721_temperature_t1e-2", ("fp32", "fp64", "bf16x3")),
                            ("gl180_temperature_t1e-2", ("fp32", "fp64", "bf16x3"))):
            for prec in precs:
                try:
                    log(f"[bench] companion {case} {prec}")
                    comp[f"{case}_{prec}"] = bench_companion(torch, case, prec)
                except Exception as e:
                    comp[f"{case}_{prec}"] = {"error": str(e)}
                torch.cuda.empty_cache()
        out["companions"] = comp
        for prec in ("fp32", "fp64"):
            try:
                log(f"[bench] climate attribution {prec}")
                sec[f"climate_attribution_hp64_{prec}"] = bench_climate_attribution(torch, prec)
            except Exception as e:
                sec[f"climate_attribution_hp64_{prec}"] = {"error": str(e)}
            torch.cuda.empty_cache()
        for nside in (64, 256):
            for prec in ("fp32", "fp64"):
                try:
                    log(f"[bench] healpix nside={nside} {prec}")
                    sec[f"healpix_nside{nside}_{prec}"] = bench_healpix(torch, nside, prec)
                except Exception as e:
                    sec[f"healpix_nside{nside}_{prec}"] = {"error": str(e)}
                torch.cuda.empty_cache()
        out["secondary"] = sec
        bat = {}
        for prec, legm in (("fp32", "recurrence"), ("bf16x3", "recurrence"), ("bf16", "recurrence"),
                           ("bf16", "table")):
            key = f"{prec}_{'table_mfma' if legm == 'table' else 'recurrence'}"
            try:
                log(f"[bench] batched gradient {key}")
                bat[f"grad_16x360x720_{key}"] = bench_grad_batch(torch, prec, legm)
                log(f"[bench] uneven batch {key}")
                bat[f"uneven_256_{key}"] = bench_uneven_batch(torch, prec, legm)
            except Exception as e:
                bat[key] = {"error": str(e)}
            torch.cuda.empty_cache()
        out["batched"] = bat
    if not args.no_cpu_baseline:
        log("[bench] heat applies for the error report")
        gpu_heat = {}
        _, _, p_np, _ = make_inputs(plan, torch)
        for prec, legm in (("fp32", "recurrence"), ("bf16", "table"), ("fp64", "recurrence"),
                           ("bf16x3", "recurrence"), ("bf16", "recurrence")):
            try:
                pl = plan if (prec, legm) == (args.precision, args.legendre) else \
                    Plan([GRID], precision=prec, legendre=legm)
                v = torch.as_tensor(p_np, dtype=pl.dtype, device="cuda").contiguous()
                gpu_heat[f"{prec}_{legm}"] = pl.heat_apply(v, [T_HEAT]).double().cpu().numpy()
                del pl
            except Exception as e:
                log(f"[bench] heat apply {prec} {legm} failed: {e}")
            torch.cuda.empty_cache()
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"], errs = cpu_baseline(args.cpu_budget, gpu_heat, one_thread_budget_s=8.0)
        out["heat_apply_rel_l2_vs_oracle"] = errs
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
