"""YAND-MVSK throughput on one MI355X.

A step is one complete outer YAND iteration (Algorithm 1) on the full-scale
workload n = 5440 assets x T = 12000 bars: the exact sample-oracle pass, the
affine-normal direction with the exact log-det trace (SYRK of the tangent
Hessian, Cholesky and triangular inverse, trace GEMM, third-order pass), the
line-search pass with its FP64 power sums, the exact quartic step and the
update.  Inputs are resident in HBM before the timed region.

Prints one JSON line (see the metric fields below).  The FP64 CPU oracle is
timed on a bounded sample of the same workload (one outer iteration) as the
CPU baseline.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}
DTYPE_NAME = {"fp64": "f64",
              "fp32": "f32 products (A stored f32, FP32-accumulated MFMA), "
                      "f64 reductions and factor",
              "bf16": "bf16 products (A stored bf16, FP32-accumulated MFMA), "
                      "f64 reductions and factor"}
ESIZE = {"fp64": 8, "fp32": 4, "bf16": 2}


def kernel_model(name, T, n, esize):
    """Algorithmic work per launch: ('hbm', bytes) or ('mfma', flops)."""
    if name in ("oracle_pass", "hvp_pass", "line_pass", "dot_pass",
                "third_pass"):
        return "hbm", T * n * esize + 2 * 8 * (T + n)
    if name in ("syrk", "trace_gemm"):
        return "mfma", float(T) * n * (n + 1)
    if name == "potrf_trtri":
        return "mfma", 2.0 * n**3 / 3.0
    return None, None


def cpu_baseline(R, c):
    """One outer iteration of the FP64 oracle (bounded sample)."""
    import oracle as O
    try:
        from threadpoolctl import threadpool_info
        threads = max((p.get("num_threads", 1) for p in threadpool_info()),
                      default=1)
    except Exception:
        threads = os.cpu_count() or 1
    mu, A = O.center(R)
    Cm, b = O.constraints(mu)
    U = O.tangent_basis(Cm)
    x = O.feasible_start(Cm, b)
    t0 = time.perf_counter()
    dr = O.affine_normal(A, mu, c, x, U)
    coef = O.linesearch_coeffs(A, mu, c, x, dr.d)
    alpha = O.select_step(coef)
    _ = x + alpha * dr.d
    el = time.perf_counter() - t0
    return {"value": 1.0 / el, "unit": "iters/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"1 outer iteration (oracle pass, exact-trace direction, "
                      f"line search, step) at n={R.shape[1]}, T={R.shape[0]}; "
                      f"{el:.1f} s"}


def log(msg):
    """Progress line on stderr (stdout carries only the JSON result)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _conv(infos):
    return sum(1 for i in infos if i.status == 0 and i.gnorm <= 1e-8)


def frontier_bench(workload, n_targets, n_plain, precision="fp64",
                   autotune=True, pcg=False):
    """Frontier solves/s: batched (one call, lanes advancing together with
    graph-replayed iterations) vs plain single-instance solves of the same
    instances, at ||reduced gradient|| <= 1e-8; pcg: the PCG configuration
    (batched tangent solves: one pair of block products per CG step for all
    lanes)."""
    import torch

    import synth
    from paper_2604_25378_amd import binding as yb

    log(f"frontier {workload}")
    R = synth.workload_returns(workload)
    T, n = R.shape
    targets = synth.frontier_targets(R, n_targets)
    C4 = np.array([synth.crra_coefficients(g) for g in (2.0, 4.0, 6.0, 10.0)
                   for _ in targets])
    tg = np.tile(targets, 4)
    ctx = yb.Context(torch.from_numpy(R).cuda(), precision)
    if autotune:
        ctx.autotune()
    opts = yb.default_opts(large=True) if pcg else None
    ctx.frontier(C4[:2], tg[:2], opts=opts)  # warm-up (graph, allocations)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    W, infos = ctx.frontier(C4, tg, opts=opts)
    torch.cuda.synchronize()
    el_b = time.perf_counter() - t0
    its = [i.iterations for i in infos]
    t0 = time.perf_counter()
    plain_its = []
    for b in range(n_plain):
        _, inf = ctx.solve(C4[b], target=tg[b], opts=opts)
        plain_its.append(inf.iterations)
    torch.cuda.synchronize()
    el_p = time.perf_counter() - t0
    ctx.close()
    return {"workload": f"{workload}: n={n} T={T}, {len(tg)} instances "
                        f"({n_targets} targets x 4 CRRA gamma), "
                        f"{'PCG' if pcg else 'direct'} configuration",
            "batched_solves_per_s": len(tg) / el_b,
            "plain_solves_per_s": n_plain / el_p,
            "speedup": (len(tg) / el_b) / (n_plain / el_p),
            "converged": f"{_conv(infos)}/{len(tg)}",
            "iterations_mean": float(np.mean(its)),
            "plain_sample": n_plain,
            "plain_iterations_mean": float(np.mean(plain_its))}


def ragged_bench(count=32, T=6000, precision="fp64", autotune=True):
    """32 independent universes with n uniform in [100, 1500]: one batched
    call over all contexts vs plain single solves, budget set."""
    import torch

    import synth
    from paper_2604_25378_amd import binding as yb

    log(f"ragged universes: {count} contexts")
    sizes = synth.ragged_universe_sizes(count)
    ctxs = [yb.Context(torch.from_numpy(
        synth.factor_returns(int(m), T, 10, 0, 4.0, 0.0, 2000 + i)).cuda(),
        precision) for i, m in enumerate(sizes)]
    if autotune:
        for cx in ctxs:
            cx.autotune()
    C4 = np.tile(np.array([1.0, 5.0, 2.0, 10.0]), (count, 1))
    yb.batch_solve(ctxs[:2], C4[:2])        # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    W, infos = yb.batch_solve(ctxs, C4)
    torch.cuda.synchronize()
    el_b = time.perf_counter() - t0
    t0 = time.perf_counter()
    dev = 0.0
    for b in range(count):
        w, _ = ctxs[b].solve(C4[b])
        dev = max(dev, float((w - W[b]).abs().max()))
    torch.cuda.synchronize()
    el_p = time.perf_counter() - t0
    for cx in ctxs:
        cx.close()
    return {"workload": f"{count} universes, n in [{sizes.min()}, "
                        f"{sizes.max()}] (sum {int(sizes.sum())}), T={T}",
            "batched_solves_per_s": count / el_b,
            "plain_solves_per_s": count / el_p,
            "speedup": el_p / el_b,
            "converged": f"{_conv(infos)}/{count}",
            "iterations_mean": float(np.mean([i.iterations for i in infos])),
            "max_abs_w_diff_vs_plain": dev}


OUTCOME = {0: "converged", 1: "iteration budget", 2: "stalled"}


def probe_bench(workload="n5440_T12000", probes=64, seed=0):
    """PCG configuration (budget set, from equal weights) with the exact
    trace against the probe estimate (k sign vectors per direction, block
    PCG on the matrix cores): seconds per solve and per outer iteration,
    iterations, Krylov counts and the objective gap between the two
    minimisers."""
    import torch

    import synth
    from paper_2604_25378_amd import binding as yb

    log(f"probe trace: {workload}")
    R = synth.workload_returns(workload)
    T, n = R.shape
    c = np.array(synth.WORKLOADS[workload]["c"])
    ctx = yb.Context(torch.from_numpy(R).cuda(), "fp64")
    rows = {}
    res = {}
    for mode in ("exact", "probe"):
        opts = yb.default_opts(large=True, trace_mode=mode, probes=probes,
                               probe_seed=seed)
        ctx.solve(c, opts=yb.default_opts(large=True, trace_mode=mode,
                                          probes=probes, max_iter=1))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        w, info = ctx.solve(c, opts=opts)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        f, _, _ = ctx.eval(c, w, grad=False)
        res[mode] = f
        rows[mode] = {"solve_s": el, "iterations": info.iterations,
                      "ms_per_iteration": 1e3 * el / max(info.iterations, 1),
                      "cg_iters": info.cg_iters,
                      "probe_cg_iters": info.probe_cg_iters,
                      "outcome": OUTCOME.get(info.status, str(info.status)),
                      "gnorm": info.gnorm, "f": f}
    ctx.close()
    return {"workload": f"{workload}: n={n} T={T}, c={tuple(float(v) for v in c)}, budget set, "
                        f"PCG configuration, {probes} probes",
            **rows,
            "objective_rel_gap": abs(res["probe"] - res["exact"]) / abs(res["exact"]),
            "iteration_speedup": rows["exact"]["ms_per_iteration"]
                                 / rows["probe"]["ms_per_iteration"]}


def precision_bench(reps=3):
    """Single solves on the two single-solve workloads in each storage
    precision of A (FP32 and BF16 form the exact trace's products on the
    matrix cores with FP32 accumulation; every reduction stays FP64):
    n = 2000, T = 12000 with the PCG configuration and stall recovery
    (FP64, FP32, BF16), and n = 400, T = 4800 with the direct and the PCG
    configurations (FP64, FP32).  Per row: median seconds per solve,
    iterations, the distance of the weights to the FP64 solve's and the
    reduced gradient of the FP64 problem at the returned weights (the FP64
    context's own stationarity measure, max_iter = 0 from those weights)."""
    import torch

    import synth
    from paper_2604_25378_amd import binding as yb

    out = {}
    plan = [("n2000_T12000", "pcg", ("fp64", "fp32", "bf16")),
            ("n400_T4800", "direct", ("fp64", "fp32")),
            ("n400_T4800", "pcg", ("fp64", "fp32"))]
    for wl, solver, precs in plan:
        log(f"precision: {wl} {solver}")
        R = synth.workload_returns(wl)
        T, n = R.shape
        c = np.array(synth.WORKLOADS[wl]["c"])
        Rd = torch.from_numpy(R).cuda()
        ctx64 = yb.Context(Rd, "fp64")
        opts = yb.default_opts(large=solver == "pcg")
        rows, w64 = {}, None
        for prec in precs:
            ctx = ctx64 if prec == "fp64" else yb.Context(Rd, prec)
            ctx.solve(c, opts=opts)              # warm-up (allocations)
            torch.cuda.synchronize()
            times = []
            for _ in range(reps):
                t0 = time.perf_counter()
                w, info = ctx.solve(c, opts=opts)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
            if prec == "fp64":
                w64 = w.clone()
            _, i64 = ctx64.solve(c, w0=w, opts=yb.default_opts(max_iter=0))
            rows[prec] = {
                "median_s": float(np.median(times)),
                "iterations": info.iterations, "restarts": info.restarts,
                "cg_iters": info.cg_iters,
                "outcome": OUTCOME.get(info.status, str(info.status)),
                "gnorm_own": info.gnorm,
                "gnorm_fp64_problem": i64.gnorm,
                "max_abs_w_diff_vs_fp64": float((w - w64).abs().max()),
                "max_abs_w": float(w64.abs().max()),
            }
            if ctx is not ctx64:
                ctx.close()
        ctx64.close()
        del Rd
        out[f"{wl}_{solver}"] = {
            "workload": f"{wl}: n={n} T={T}, c={tuple(float(v) for v in c)}, budget set, "
                        f"{'PCG with stall recovery' if solver == 'pcg' else 'direct'}",
            **rows}
    return out


def simplex_bench(precision="fp64"):
    """Simplex set with the boundary block (face continuation, projected
    trial step, projected-KKT stop) on the paper's synthetic coefficient-
    stress generator: returns uniform on [-0.1, 0.4], T = 252, profiles
    [10,1,10,1], [1,10,1,10], [10,10,10,10]; the direct configuration at
    n = 100 and the PCG configuration with stall recovery at n = 1000 and
    5440 (n > T: the regularised stress regime).  Reports the rate, the
    iterations and the projected-KKT hits at the study's 1e-6 target."""
    import torch

    import synth
    from paper_2604_25378_amd import binding as yb

    profiles = ([10.0, 1.0, 10.0, 1.0], [1.0, 10.0, 1.0, 10.0],
                [10.0, 10.0, 10.0, 10.0])
    res = {}
    for n, large in ((100, False), (1000, True), (5440, True)):
        log(f"simplex boundary block: n={n} T=252 "
            f"({'PCG' if large else 'direct'})")
        R = synth.uniform_returns(n, 252, seed=n)
        ctx = yb.Context(torch.from_numpy(R).cuda(), precision)
        opts = yb.default_opts(large=large, feasible_set="simplex")
        ctx.solve(profiles[2], opts=yb.default_opts(large=large,
                                                    feasible_set="simplex",
                                                    max_iter=2))  # warm-up
        torch.cuda.synchronize()
        times, infos, outcome = [], [], []
        for c in profiles:
            t0 = time.perf_counter()
            try:
                _, info = ctx.solve(c, opts=opts)
                outcome.append(OUTCOME.get(info.status, str(info.status)))
            except yb.YandError as e:   # e.g. indefinite outside the certificate
                info = None
                outcome.append(yb.ERRORS.get(e.code, str(e.code)))
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            infos.append(info)
        ctx.close()
        ok = [i for i in infos if i is not None]
        res[f"n{n}_T252"] = {
            "config": "PCG (large), stall recovery" if large else "direct (small)",
            "profiles": [list(c) for c in profiles],
            "outcome": outcome,
            "solves_per_s": len(profiles) / sum(times),
            "median_s": float(np.median(times)),
            "iterations": [i.iterations if i else None for i in infos],
            "projected_steps": [i.projected_steps if i else None for i in infos],
            "restarts": [i.restarts if i else None for i in infos],
            "kkt": [i.kkt if i else None for i in infos],
            "kkt_hits_1e-6": f"{sum(i.kkt <= 1e-6 for i in ok)}/{len(infos)}",
            "traces_dense_thin": [[i.dense_traces - i.thin_traces,
                                   i.thin_traces] if i else None
                                  for i in infos]}
    return res


def conditioning_bench(precision="fp64"):
    """The controlled CRRA conditioning benchmark of the computational study
    and its n > T stress counterpart: CRRA gamma = 6, kappa_+(AU) in {1, 10,
    1e2, 1e3} prescribed by synth.conditioned_returns (A x0 = 0), simplex
    with the boundary block, PCG configuration with stall recovery; three
    instances (seeds) per level after one untimed warm-up solve, medians of
    time, iterations and projected-KKT residual."""
    import torch

    import synth
    from paper_2604_25378_amd import binding as yb

    c = synth.crra_coefficients(6.0)
    opts = yb.default_opts(large=True, feasible_set="simplex")
    res = {}
    for n, T in ((1000, 2000), (5000, 252)):
        rows = {}
        for kappa in (1.0, 10.0, 100.0, 1000.0):
            log(f"conditioning: n={n} T={T} kappa={kappa:g}")
            times, its, kkts, stat = [], [], [], []
            for seed in (0, 1, 2):
                R = synth.conditioned_returns(n, T, kappa, seed)
                ctx = yb.Context(torch.from_numpy(R).cuda(), precision)
                if seed == 0:
                    ctx.solve(c, opts=opts)     # untimed warm-up
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, info = ctx.solve(c, opts=opts)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
                its.append(info.iterations)
                kkts.append(info.kkt)
                stat.append(OUTCOME.get(info.status, str(info.status)))
                ctx.close()
            rows[f"kappa={kappa:g}"] = {
                "median_s": float(np.median(times)),
                "median_iterations": float(np.median(its)),
                "median_kkt": float(np.median(kkts)),
                "outcome": stat}
        res[f"n{n}_T{T}"] = rows
    return res


def return_floor_bench(precision="fp64"):
    """The return-floor protocol of the real-data comparison on a synthetic
    stand-in for the intraday panel: synth.priced_factor_returns(1000,
    12000, K=3, nu=5, seed 0) (riskier assets earn more, the market crashes
    now and then), simplex, PCG configuration with stall recovery.  The
    kurtosis-focused profile over the paper's floor sweep q in {0.4, 0.5,
    0.6}, and the balanced and skew-focused profiles at q = 0.5.  Each case
    is one yand_return_floor call: time, number of solves, calibrated c1,
    outcome of the returned solve and its distance to the floor."""
    import torch

    import synth
    from paper_2604_25378_amd import binding as yb

    n, T = 1000, 12000
    R = synth.priced_factor_returns(n, T, 3, 5.0, 0)
    mu = R.mean(axis=0)
    spread = float(mu.max() - mu.min())
    ctx = yb.Context(torch.from_numpy(R).cuda(), precision)
    opts = yb.default_opts(large=True, feasible_set="simplex")
    ctx.solve([0.0, 1.0, 1.0, 1.0], opts=opts)     # untimed warm-up
    cases = [("kurtosis", (1.0, 1.0, 10.0), q) for q in (0.4, 0.5, 0.6)]
    cases += [("balanced", (1.0, 1.0, 1.0), 0.5),
              ("skew", (1.0, 10.0, 1.0), 0.5)]
    rows = []
    for name, prof, q in cases:
        log(f"return floor: n={n} T={T} {name} q={q}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        row = {"profile": name, "p2_p3_p4": list(prof), "q": q}
        try:
            c, w, floor, ret, info, solves = ctx.return_floor(prof, q, opts=opts)
            el = time.perf_counter() - t0
            row.update({
                "seconds": el, "solves": solves, "ms_per_solve": 1e3 * el / solves,
                "c1": c[0], "outcome": OUTCOME.get(info.status, str(info.status)),
                "iterations": info.iterations, "kkt": info.kkt,
                "gap_to_floor_rel_spread": (ret - floor) / spread,
                "support": int((w > 1e-6).sum().item())})
        except yb.YandError as e:
            row.update({"seconds": time.perf_counter() - t0,
                        "outcome": yb.ERRORS.get(e.code, str(e.code))})
        rows.append(row)
    ctx.close()
    return {"workload": f"priced_factor n{n}_T{T}", "config": "PCG (large), simplex",
            "cases": rows}


REGIME_BLOCKS = (("n<=60", (20, 40, 60)), ("80<=n<=100", (80, 100)),
                 ("120<=n<=200", (120, 160, 200)),
                 ("250<=n<=500", (250, 350, 500)),
                 ("600<=n<=1000", (600, 800, 1000)))


def regime_bench(precision="fp64"):
    """The direct-versus-PCG regime comparison of the computational study on
    the T = 252 coefficient-stress generator (uniform returns on [-0.1, 0.4],
    profiles [10,1,10,1], [1,10,1,10], [10,10,10,10]), simplex with the
    boundary block, through n = 1000.  Per n-block: median time of each
    configuration, the median instance-wise ratio direct / PCG, projected-KKT
    hits at 1e-6, and objective ties (both within 1e-6 of the better value;
    a run that errors counts as neither)."""
    import torch

    import synth
    from paper_2604_25378_amd import binding as yb

    profiles = ([10.0, 1.0, 10.0, 1.0], [1.0, 10.0, 1.0, 10.0],
                [10.0, 10.0, 10.0, 10.0])
    res = {}
    for block, ns in REGIME_BLOCKS:
        log(f"regime: {block}")
        t_s, t_l, ratio, hit_s, hit_l, ties, runs = [], [], [], 0, 0, 0, 0
        for n in ns:
            ctx = yb.Context(torch.from_numpy(
                synth.uniform_returns(n, 252, seed=n)).cuda(), precision)
            for large in (False, True):    # untimed warm-up per configuration
                ctx.solve(profiles[2], opts=yb.default_opts(
                    large=large, feasible_set="simplex", max_iter=2))
            for c in profiles:
                runs += 1
                out = {}
                for large in (False, True):
                    opts = yb.default_opts(large=large, feasible_set="simplex")
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    try:
                        w, info = ctx.solve(c, opts=opts)
                        torch.cuda.synchronize()
                        f = ctx.eval(c, w, grad=False)[0]
                        out[large] = (time.perf_counter() - t0, info.kkt, f)
                    except yb.YandError:
                        out[large] = (time.perf_counter() - t0, math.inf,
                                      math.inf)
                (ts, ks, fs), (tl, kl, fl) = out[False], out[True]
                t_s.append(ts)
                t_l.append(tl)
                ratio.append(ts / tl)
                hit_s += ks <= 1e-6
                hit_l += kl <= 1e-6
                best = min(fs, fl)
                ties += (math.isfinite(best) and fs - best <= 1e-6
                         and fl - best <= 1e-6)
            ctx.close()
        res[block] = {"n": list(ns), "runs": runs,
                      "direct_median_s": float(np.median(t_s)),
                      "pcg_median_s": float(np.median(t_l)),
                      "median_ratio_direct_over_pcg": float(np.median(ratio)),
                      "kkt_hits_direct": f"{hit_s}/{runs}",
                      "kkt_hits_pcg": f"{hit_l}/{runs}",
                      "objective_ties": f"{ties}/{runs}"}
    return res


def line_search_bench(precision="fp64"):
    """The direct-configuration line-search diagnostic: Armijo backtracking
    against the exact quartic rule on the T = 252 coefficient-stress
    generator (three profiles), simplex with the boundary block; mean time,
    iterations and projected-KKT residual per n-block."""
    import torch

    import synth
    from paper_2604_25378_amd import binding as yb

    profiles = ([10.0, 1.0, 10.0, 1.0], [1.0, 10.0, 1.0, 10.0],
                [10.0, 10.0, 10.0, 10.0])
    res = {}
    for block in ((4, 8, 12), (20, 40, 60, 80, 100)):
        row = {}
        for rule in ("armijo", "exact"):
            opts = yb.default_opts(feasible_set="simplex", linesearch=rule)
            times, its, kkts, errors = [], [], [], 0
            for n in block:
                ctx = yb.Context(torch.from_numpy(
                    synth.uniform_returns(n, 252, seed=n)).cuda(), precision)
                ctx.solve(profiles[2], opts=opts)        # warm-up
                for c in profiles:
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    try:
                        _, info = ctx.solve(c, opts=opts)
                    except yb.YandError:
                        errors += 1
                        continue
                    torch.cuda.synchronize()
                    times.append(time.perf_counter() - t0)
                    its.append(info.iterations)
                    kkts.append(info.kkt)
                ctx.close()
            row[rule] = {"mean_s": float(np.mean(times)),
                         "median_s": float(np.median(times)),
                         "mean_iterations": float(np.mean(its)),
                         "mean_kkt": float(np.mean(kkts)),
                         "solves": len(times), "errors": errors}
        res["n in " + ",".join(map(str, block))] = row
    return res


def warmstart_hard_bench(precision="fp64"):
    """Warm start where plain solves take many iterations: the controlled
    conditioning generator (n = 1000, T = 2000), budget set, CRRA gamma in
    [1, 6]; the network (3 x 256, 4000 epochs, Adam step 3e-4) is trained on
    plain solutions at 24 gammas and evaluated on the 23 midpoints, batched
    both ways.  At the default step 1e-3 this training is bistable: targets
    perturbed at the 1e-12 level end at a loss of either 1.9e-3 or 0.12,
    the latter with every proposal rejected; at 3e-4 it lands at 2.2e-3
    every time.  At kappa_+(AU) = 1e3 the residual test rejects every
    proposal (the plain start is returned), which the second row shows."""
    import torch

    import synth
    from paper_2604_25378_amd import binding as yb

    res = {}
    for kappa in (1e2, 1e3):
        log(f"warm start, conditioned panel kappa={kappa:g}")
        R = synth.conditioned_returns(1000, 2000, kappa, 1)
        ctx = yb.Context(torch.from_numpy(R).cuda(), precision)
        gtr = np.linspace(1.0, 6.0, 24)
        Ctr = np.array([synth.crra_coefficients(g) for g in gtr])
        Cte = np.array([synth.crra_coefficients(g)
                        for g in 0.5 * (gtr[1:] + gtr[:-1])])
        Wtr, _ = ctx.frontier(Ctr)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        net, loss = yb.warmstart_train(
            ctx, Ctr, None, Wtr,
            yb.default_mlp_opts(hidden=256, epochs=4000, lr=3e-4))
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        ctx.frontier(Cte[:2])                    # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        W0, used, _ = yb.warmstart_predict(ctx, net, Cte, None)
        _, iw = ctx.frontier(Cte, W0=W0)
        torch.cuda.synchronize()
        t_w = time.perf_counter() - t0
        t0 = time.perf_counter()
        _, ip = ctx.frontier(Cte)
        torch.cuda.synchronize()
        t_p = time.perf_counter() - t0
        net.close()
        ctx.close()
        res[f"kappa_{kappa:g}"] = {
            "workload": f"conditioned panel n=1000 T=2000 kappa_+(AU)={kappa:g}, "
                        f"budget set, {len(Cte)} held-out CRRA gammas in [1, 6]",
            "plain_iterations_mean": float(np.mean([i.iterations for i in ip])),
            "warm_iterations_mean": float(np.mean([i.iterations for i in iw])),
            "proposals_used": float(np.mean(used)),
            "plain_solves_per_s": len(Cte) / t_p,
            "warm_solves_per_s": len(Cte) / t_w,
            "train_s": t_train, "train_loss": loss,
            "converged": f"{_conv(iw)}/{len(Cte)}"}
    return res


def warmstart_bench(workload, n_train_targets=16, n_points=256, n_plain=16,
                    precision="fp64", autotune=True):
    """Frontier sweep at full scale: batched + MLP-warm-started solves vs
    batched plain-start solves vs plain single-instance solves of the same
    n_points instances, all to ||reduced gradient|| <= 1e-8.

    The network is trained on plain solutions of a disjoint grid (16 targets
    x gamma in {2, 4, 6, 10}); the sweep uses gamma in {2.5, 3.5, 5, 8} and
    n_points / 4 targets from the minimum-variance mean to the largest mean.
    Warm-started timings include the prediction (features, forward pass,
    residual test against the plain start)."""
    import torch

    import synth
    from paper_2604_25378_amd import binding as yb

    R = synth.workload_returns(workload)
    T, n = R.shape
    ctx = yb.Context(torch.from_numpy(R).cuda(), precision)
    if autotune:
        ctx.autotune()

    def grid(gammas, k):
        tt = synth.frontier_targets(R, k)
        return (np.array([synth.crra_coefficients(g) for g in gammas for _ in tt]),
                np.tile(tt, len(gammas)))

    log(f"warm-start sweep {workload}: training solves")
    Ctr, ttr = grid((2.0, 4.0, 6.0, 10.0), n_train_targets)
    Cev, tev = grid((2.5, 3.5, 5.0, 8.0), n_points // 4)
    ctx.frontier(Ctr[:2], ttr[:2])          # warm-up (graph path, allocations)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Wtr, itr = ctx.frontier(Ctr, ttr)
    torch.cuda.synchronize()
    el_trsolve = time.perf_counter() - t0
    log(f"training set solved in {el_trsolve:.1f} s; training the network")
    t0 = time.perf_counter()
    net, loss = yb.warmstart_train(ctx, Ctr, ttr, Wtr)
    torch.cuda.synchronize()
    el_train = time.perf_counter() - t0
    t0 = time.perf_counter()
    W0, used, gns = yb.warmstart_predict(ctx, net, Cev, tev)
    torch.cuda.synchronize()
    el_pred = time.perf_counter() - t0
    Ww, iw = ctx.frontier(Cev, tev, W0=W0)
    torch.cuda.synchronize()
    el_warm = time.perf_counter() - t0
    log(f"trained in {el_train:.1f} s; warm sweep {el_warm:.1f} s; plain batched")
    t0 = time.perf_counter()
    Wp, ip = ctx.frontier(Cev, tev)
    torch.cuda.synchronize()
    el_batch = time.perf_counter() - t0
    log(f"plain batched sweep {el_batch:.1f} s; plain single solves")
    idx = np.linspace(0, len(tev) - 1, n_plain).astype(int)
    t0 = time.perf_counter()
    plain_its = []
    for b in idx:
        _, inf = ctx.solve(Cev[b], target=tev[b])
        plain_its.append(inf.iterations)
    torch.cuda.synchronize()
    el_plain = time.perf_counter() - t0
    dev = float((Ww - Wp).abs().max())
    net.close()
    ctx.close()
    P = len(tev)
    warm = P / el_warm
    return {"workload": f"{workload}: n={n} T={T}, {P}-point sweep "
                        f"({P // 4} targets x gamma 2.5/3.5/5/8)",
            "warm_batched_solves_per_s": warm,
            "batched_solves_per_s": P / el_batch,
            "plain_solves_per_s": n_plain / el_plain,
            "speedup_warm_vs_plain": warm / (n_plain / el_plain),
            "speedup_warm_vs_batched": warm / (P / el_batch),
            "converged_warm": f"{_conv(iw)}/{P}",
            "converged_batched": f"{_conv(ip)}/{P}",
            "iterations_mean_warm": float(np.mean([i.iterations for i in iw])),
            "iterations_mean_batched": float(np.mean([i.iterations for i in ip])),
            "plain_sample": n_plain,
            "plain_iterations_mean": float(np.mean(plain_its)),
            "mlp_used_frac": float(used.mean()),
            "gnorm_start_median": {"mlp": float(np.median(gns[:, 0])),
                                   "plain": float(np.median(gns[:, 1]))},
            "predict_s": el_pred,
            "max_abs_w_diff_warm_vs_batched": dev,
            "training": {"instances": len(ttr), "solve_s": el_trsolve,
                         "train_s": el_train, "final_loss": loss,
                         "network": f"{yb.WS_FEATURES}-512-512-512-{n - 1}, "
                                    "FP32, full-batch Adam, 2000 epochs"},
            "warm_solves_per_s_incl_training": P / (el_warm + el_trsolve + el_train)}


TRAFFIC_SOURCES = {   # kernel -> source file whose text the counters belong to
    "trace_gemm": "paper_2604_25378_amd/csrc/dense.hip",
    "syrk": "paper_2604_25378_amd/csrc/dense.hip",
    "oracle_pass": "paper_2604_25378_amd/csrc/pass.hip",
    "hvp_pass": "paper_2604_25378_amd/csrc/pass.hip",
}


def source_hash(rel):
    import hashlib
    with open(os.path.join(ROOT, rel), "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()


def measured_traffic(kernel, workload, precision):
    """HBM bytes per launch from the committed rocprofv3 PMC summary
    (FETCH_SIZE + WRITE_SIZE, each scaled by the same counter's reading for
    a plain device copy of known size), or None when no summary exists for
    this kernel and workload or the kernel source changed since."""
    path = os.path.join(ROOT, "profiles",
                        f"traffic_{kernel}_{workload}_{precision}.json")
    if kernel not in TRAFFIC_SOURCES or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha1") != source_hash(TRAFFIC_SOURCES[kernel]):
        return None
    return rec["bytes_per_launch"]


def copy_calibration(nbytes=1 << 30):
    """One plain device copy of nbytes (the PMC scale reference)."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy calibration: {nbytes} bytes read, {nbytes} written")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp64", choices=list(ESIZE))
    ap.add_argument("--workload", default="n5440_T12000")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-frontier", action="store_true")
    ap.add_argument("--frontier-points", type=int, default=256)
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the built-in launch shapes")
    ap.add_argument("--only", default=None,
                    help="run the headline step and this one block only "
                         "(frontier_n1000, frontier_n1000_pcg, ragged, warmstart, warmstart_hard, simplex, "
                         "conditioning, line_search, return_floor, regime, "
                         "precision, probe)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with one 1 GiB device copy (PMC scale reference)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is "
              "not supported (the multi-GPU sharding is design only)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_2604_25378_amd import binding as yb

    wl = synth.WORKLOADS[args.workload]
    R = synth.workload_returns(args.workload)
    T, n = R.shape
    c = np.array(wl["c"])
    Rd = torch.from_numpy(R).cuda()
    ctx = yb.Context(Rd, args.precision)
    del Rd
    torch.cuda.synchronize()
    tuned = None if args.no_autotune else ctx.autotune()
    opts = yb.default_opts(max_iter=1, eps=0.0)
    w = torch.full((n,), 1.0 / n, dtype=torch.float64, device="cuda")

    def step(w):
        w2, info = ctx.solve(c, w0=w, opts=opts)
        assert info.iterations == 1, info
        return w2, info

    for _ in range(args.warmup):
        w, _ = step(w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        w, info = step(w)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # Per-kernel times from HIP events on the library stream, in as many
    # steps again after the timed ones, so that recording and reading the
    # events stays out of the timed region.
    ctx.profile(True)
    for _ in range(args.steps):
        w, info = step(w)
    torch.cuda.synchronize()
    prof = ctx.profile_read()
    ctx.profile(False)
    gn = info.gnorm

    # HVP pass bandwidth (a4), timed on the library stream: a fused read of A
    # per product at the current iterate.
    v = torch.randn(n, dtype=torch.float64, device="cuda")
    ctx.hvp(c, w, v)
    ctx.profile(True)
    for _ in range(10):
        ctx.hvp(c, w, v)
    torch.cuda.synchronize()
    hprof = ctx.profile_read()
    ctx.profile(False)
    if "hvp_pass" in hprof:
        prof_h = {"hvp_pass": hprof["hvp_pass"]}
    else:
        prof_h = {}

    # Oracle pass (a2, value and gradient, one fused read of A) with the
    # 256 MB MALL defeated: the eval calls rotate over enough contexts of the
    # same workload that their matrices total more than 512 MB, so each pass
    # finds its A evicted by the others.
    a_bytes = T * n * ESIZE[args.precision]
    ring_k = max(1, math.ceil(512e6 / a_bytes))
    ring = [ctx]
    if ring_k > 1:
        Rd = torch.from_numpy(R).cuda()
        for _ in range(ring_k - 1):
            cx = yb.Context(Rd, args.precision)
            if tuned is not None:
                cx.tuning(ctx.tuning())
            ring.append(cx)
        del Rd
    for cx in ring:
        cx.eval(c, w)
    torch.cuda.synchronize()
    for cx in ring:
        cx.profile(True)
    for i in range(4 * ring_k):
        ring[i % ring_k].eval(c, w)
    torch.cuda.synchronize()
    ms_r, cnt_r = 0.0, 0
    for cx in ring:
        p_ = cx.profile_read()
        cx.profile(False)
        if "oracle_pass" in p_:
            ms_r += p_["oracle_pass"][0]
            cnt_r += p_["oracle_pass"][1]
    for cx in ring[1:]:
        cx.close()
    oracle_ring = None
    if cnt_r:
        _, work_r = kernel_model("oracle_pass", T, n, ESIZE[args.precision])
        gbps_r = work_r / (ms_r / cnt_r / 1e3) / 1e9
        oracle_ring = {"contexts": ring_k,
                       "bytes_rotated": ring_k * a_bytes,
                       "avg_ms": round(ms_r / cnt_r, 4), "launches": cnt_r,
                       "gbps": round(gbps_r, 1),
                       "frac_hbm": round(gbps_r / PEAK_HBM_GBS, 3)}

    kernels = {}
    for name, (ms, cnt) in prof.items():
        kind, work = kernel_model(name, T, n, ESIZE[args.precision])
        avg_s = ms / cnt / 1e3
        entry = {"avg_ms": round(ms / cnt, 4), "launches": cnt,
                 "share": round(ms / (el * 1e3), 4)}  # same step count
        if kind == "hbm":
            entry["gbps"] = round(work / avg_s / 1e9, 1)
            entry["frac_hbm"] = round(work / avg_s / 1e9 / PEAK_HBM_GBS, 3)
        elif kind == "mfma":
            entry["tflops"] = round(work / avg_s / 1e12, 2)
        kernels[name] = entry
    for name, (ms, cnt) in prof_h.items():
        kind, work = kernel_model(name, T, n, ESIZE[args.precision])
        avg_s = ms / cnt / 1e3
        kernels[name] = {"avg_ms": round(ms / cnt, 4), "launches": cnt,
                         "share": None,
                         "gbps": round(work / avg_s / 1e9, 1),
                         "frac_hbm": round(work / avg_s / 1e9 / PEAK_HBM_GBS, 3)}
    # Dominant single kernel (potrf_trtri is a sequence of ~3 launches per
    # 128-column step, reported in the table but not as a kernel roofline).
    singles = {k: v for k, v in prof.items() if k != "potrf_trtri"}
    dom = max(singles, key=lambda k: singles[k][0])
    kind, work = kernel_model(dom, T, n, ESIZE[args.precision])
    avg_s = prof[dom][0] / prof[dom][1] / 1e3
    if kind == "hbm":
        roof = {"kernel": dom, "bound": "hbm", "achieved": work / avg_s / 1e9,
                "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    else:
        # FP32 / BF16 storage forms the dense products on the matrix cores
        # with FP32 / BF16 inputs (FP32 accumulation); FP64 on FP64 MFMA
        peak = PEAK_TFLOPS[args.precision]
        roof = {"kernel": dom, "bound": "mfma",
                "achieved": work / avg_s / 1e12, "peak": peak,
                "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(dom, args.workload, args.precision)
    roof["share_of_step"] = round(prof[dom][0] / (el * 1e3), 4)
    hv = kernels.get("hvp_pass")

    out = {
        "metric": "YAND iters/s + frontier solves/s at n=5440,T=12000; HVP HBM GB/s vs peak",
        "value": args.steps / el,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE_NAME[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: n={n} T={T} factor model "
                               f"K={wl['K']} S={wl['S']} nu={wl['nu']} "
                               f"jumps={wl['p_jump']}, c={tuple(float(v) for v in wl['c'])}, "
                               "budget set, direct exact-trace solve",
                   "precision": args.precision},
        "roofline": roof,
        "autotune": tuned,
        "pass_gbps": {k: v.get("gbps") for k, v in kernels.items() if "gbps" in v},
        "hvp_pass_frac_hbm": hv.get("frac_hbm") if hv else None,
        "oracle_pass_mall_defeated": oracle_ring,
        "frontier_solves_per_s": None,
        "kernels": kernels,
        "gnorm_after": gn,
    }
    ctx.close()
    del ctx
    blocks = {"precision": precision_bench, "probe": probe_bench,
              "frontier_n1000": lambda: frontier_bench(
                  "n1000_T12000_frontier", 16, 8, args.precision,
                  not args.no_autotune),
              "frontier_n1000_pcg": lambda: frontier_bench(
                  "n1000_T12000_frontier", 16, 8, args.precision,
                  not args.no_autotune, pcg=True),
              "warmstart_hard": lambda: warmstart_hard_bench(args.precision),
              "ragged": lambda: ragged_bench(32, 6000, args.precision,
                                             not args.no_autotune),
              "warmstart": lambda: warmstart_bench(
                  args.workload, 16, args.frontier_points, 16, args.precision,
                  not args.no_autotune),
              "simplex": lambda: simplex_bench(args.precision),
              "conditioning": lambda: conditioning_bench(args.precision),
              "line_search": lambda: line_search_bench(args.precision),
              "return_floor": lambda: return_floor_bench(args.precision),
              "regime": lambda: regime_bench(args.precision)}
    if args.only:
        out[args.only] = blocks[args.only]()
    elif not args.no_frontier:
        tune = not args.no_autotune
        fr = {"n1000_T12000": frontier_bench("n1000_T12000_frontier", 16, 8,
                                             args.precision, tune),
              "n1000_T12000_pcg": frontier_bench("n1000_T12000_frontier", 16,
                                                 8, args.precision, tune,
                                                 pcg=True),
              "ragged_T6000": ragged_bench(32, 6000, args.precision, tune),
              "n5440_T12000": warmstart_bench(args.workload, 16,
                                              args.frontier_points, 16,
                                              args.precision, tune)}
        out["frontier"] = fr
        out["warmstart_hard"] = warmstart_hard_bench(args.precision)
        out["simplex"] = simplex_bench(args.precision)
        out["conditioning"] = conditioning_bench(args.precision)
        out["line_search"] = line_search_bench(args.precision)
        out["return_floor"] = return_floor_bench(args.precision)
        out["regime"] = regime_bench(args.precision)
        out["precision"] = precision_bench()
        out["probe"] = probe_bench()
        out["frontier_solves_per_s"] = fr["n5440_T12000"]["warm_batched_solves_per_s"]
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(R, c)
    if args.copy_calibration:
        copy_calibration()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
