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
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2500.0}
DTYPE_NAME = {"fp64": "f64", "fp32": "f64 (A stored f32)", "bf16": "f64 (A stored bf16)"}
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


def frontier_bench(workload, n_targets, n_plain, precision="fp64"):
    """Frontier solves/s: batched (one call, lanes advancing together with
    graph-replayed iterations) vs plain single-instance solves of the same
    instances, at ||reduced gradient|| <= 1e-8."""
    import torch

    import synth
    from paper_2604_25378_amd import binding as yb

    R = synth.workload_returns(workload)
    T, n = R.shape
    targets = synth.frontier_targets(R, n_targets)
    C4 = np.array([synth.crra_coefficients(g) for g in (2.0, 4.0, 6.0, 10.0)
                   for _ in targets])
    tg = np.tile(targets, 4)
    ctx = yb.Context(torch.from_numpy(R).cuda(), precision)
    ctx.frontier(C4[:2], tg[:2])            # warm-up (graph path, allocations)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    W, infos = ctx.frontier(C4, tg)
    torch.cuda.synchronize()
    el_b = time.perf_counter() - t0
    ok = sum(1 for i in infos if i.status == 0 and i.gnorm <= 1e-8)
    its = [i.iterations for i in infos]
    t0 = time.perf_counter()
    plain_its = []
    for b in range(n_plain):
        _, inf = ctx.solve(C4[b], target=tg[b])
        plain_its.append(inf.iterations)
    torch.cuda.synchronize()
    el_p = time.perf_counter() - t0
    ctx.close()
    return {"workload": f"{workload}: n={n} T={T}, {len(tg)} instances "
                        f"({n_targets} targets x 4 CRRA gamma)",
            "batched_solves_per_s": len(tg) / el_b,
            "plain_solves_per_s": n_plain / el_p,
            "speedup": (len(tg) / el_b) / (n_plain / el_p),
            "converged": f"{ok}/{len(tg)}",
            "iterations_mean": float(np.mean(its)),
            "plain_sample": n_plain,
            "plain_iterations_mean": float(np.mean(plain_its))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp64", choices=list(ESIZE))
    ap.add_argument("--workload", default="n5440_T12000")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-frontier", action="store_true")
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
    opts = yb.default_opts(max_iter=1, eps=0.0)
    w = torch.full((n,), 1.0 / n, dtype=torch.float64, device="cuda")

    def step(w):
        w2, info = ctx.solve(c, w0=w, opts=opts)
        assert info.iterations == 1, info
        return w2, info

    for _ in range(args.warmup):
        w, _ = step(w)
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        w, info = step(w)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
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

    kernels = {}
    for name, (ms, cnt) in prof.items():
        kind, work = kernel_model(name, T, n, ESIZE[args.precision])
        avg_s = ms / cnt / 1e3
        entry = {"avg_ms": round(ms / cnt, 4), "launches": cnt,
                 "share": round(ms / (el * 1e3), 4)}
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
    dom = max(prof, key=lambda k: prof[k][0])
    kind, work = kernel_model(dom, T, n, ESIZE[args.precision])
    avg_s = prof[dom][0] / prof[dom][1] / 1e3
    if kind == "hbm":
        roof = {"kernel": dom, "bound": "hbm", "achieved": work / avg_s / 1e9,
                "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    else:
        peak = PEAK_TFLOPS["fp64"]      # the dense trace runs on FP64 MFMA
        roof = {"kernel": dom, "bound": "mfma",
                "achieved": work / avg_s / 1e12, "peak": peak,
                "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
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
                               f"jumps={wl['p_jump']}, c={tuple(wl['c'])}, "
                               "budget set, direct exact-trace solve",
                   "precision": args.precision},
        "roofline": roof,
        "pass_gbps": {k: v.get("gbps") for k, v in kernels.items() if "gbps" in v},
        "hvp_pass_frac_hbm": hv.get("frac_hbm") if hv else None,
        "frontier_solves_per_s": None,
        "kernels": kernels,
        "gnorm_after": gn,
    }
    ctx.close()
    del ctx
    if not args.no_frontier:
        fr = {"n1000_T12000": frontier_bench("n1000_T12000_frontier", 16, 8,
                                             args.precision),
              "n5440_T12000": frontier_bench(args.workload, 4, 2,
                                             args.precision)}
        out["frontier"] = fr
        out["frontier_solves_per_s"] = fr["n5440_T12000"]["batched_solves_per_s"]
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(R, c)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
