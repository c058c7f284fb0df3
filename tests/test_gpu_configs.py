"""Solve-level parity on the single-solve workloads in every storage
precision, against the FP64 oracle run on the matrix each precision stores.

 - n = 400, T = 4800 (10 factors, nu = 4, c = (1, 5, 2, 10)), budget set:
   the direct and the PCG configurations, FP64 and FP32 storage.
 - n = 2000, T = 12000 (20 factors plus 20 sectors, nu = 4,
   c = (1, 5, 2, 10)), budget set: the PCG configuration with stall
   recovery, FP64, FP32 and BF16 storage.

FP32 and BF16 storage form the exact trace's products on the matrix cores
with FP32 accumulation, so their iterates follow their own path; every
solve is judged where it ends: objective relative error <= 1e-10 against
the oracle's solve of the same stored problem, weights within
kappa_w = 10 eps / lambda_min of its reduced Hessian (the accuracy that
|gbar| <= eps implies under strong convexity), and the oracle's own reduced
gradient at the returned weights.  The distance to the FP64 minimiser and
the FP64 reduced gradient at the returned weights are reported per
precision and bounded by what the storage rounding implies.
"""

import numpy as np
import pytest

import oracle as O
import synth
from storage import round_storage

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2604_25378_amd import binding as yb  # noqa: E402

EPS = 1e-8


def _reduced(A, mu, c, x):
    U = O.tangent_basis(O.constraints(mu)[0])
    H = A.T @ (O.d2psi(c, A @ x)[:, None] * A) / A.shape[0]
    lmin = np.linalg.eigvalsh(U.T @ H @ U)[0]
    gbar = np.linalg.norm(U.T @ O.gradient(A, mu, c, x))
    return lmin, gbar


_CACHE = {}


def _oracle(wl, prec, solver):
    key = (wl, prec, solver)
    if key not in _CACHE:
        R = synth.workload_returns(wl)
        mu, A = O.center(R)
        Ar = round_storage(A, prec)
        opts = O.Options.large() if solver == "pcg" else O.Options()
        x, info = O.solve(R, synth.WORKLOADS[wl]["c"], opts=opts,
                          centered=(mu, Ar))
        _CACHE[key] = (R, mu, A, Ar, x, info)
    return _CACHE[key]


_CTX = {}


def _ctx(wl, prec):
    if (wl, prec) not in _CTX:
        R = synth.workload_returns(wl)
        _CTX[(wl, prec)] = yb.Context(torch.from_numpy(R).cuda(), prec)
    return _CTX[(wl, prec)]


def _check(wl, prec, solver, fp64_ref):
    print(f"[case] {wl} {prec} {solver}", flush=True)
    R, mu, A, Ar, xr, ir = _oracle(wl, prec, solver)
    c = np.array(synth.WORKLOADS[wl]["c"])
    ctx = _ctx(wl, prec)
    w, info = ctx.solve(c, opts=yb.default_opts(large=solver == "pcg"))
    w = w.cpu().numpy()
    assert info.status == 0 and info.gnorm <= EPS, info
    assert ir.status == 0
    lmin, gbar = _reduced(Ar, mu, c, xr)
    kappa_w = 10 * EPS / lmin
    f = O.objective(Ar, mu, c, w)
    assert abs(f - ir.f) <= 1e-10 * abs(ir.f)
    assert np.abs(w - xr).max() <= kappa_w
    _, gbar_w = _reduced(Ar, mu, c, w)
    assert gbar_w <= 2 * EPS
    # budget invariant up to the rounding of the steps' sums
    assert abs(w.sum() - 1.0) <= 1e-14 * max(1.0, np.abs(w).sum())
    # against the FP64 problem
    x64 = fp64_ref
    _, g64 = _reduced(A, mu, c, w)
    dist = float(np.abs(w - x64).max())
    print(f"[precision] {wl} {prec} {solver}: iterations {info.iterations} "
          f"(oracle {ir.iterations}), |w - w_oracle|_inf {np.abs(w - xr).max():.2e} "
          f"(kappa_w {kappa_w:.1e}), |w - w*_fp64|_inf {dist:.2e}, "
          f"FP64 |gbar| {g64:.2e}", flush=True)
    return dist, g64


@pytest.mark.parametrize("solver", ["direct", "pcg"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_n400_T4800(prec, solver):
    wl = "n400_T4800"
    x64 = _oracle(wl, "fp64", "direct")[4]
    dist, g64 = _check(wl, prec, solver, x64)
    if prec == "fp32":
        # FP32 rounding of A (2^-24 relative) moves the minimiser by about
        # that much relative to the weights' scale
        assert dist <= 1e-4 * np.abs(x64).max()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_n2000_T12000_pcg(prec):
    wl = "n2000_T12000"
    x64 = _oracle(wl, "fp64", "pcg")[4]
    dist, g64 = _check(wl, prec, "pcg", x64)
    bound = {"fp64": 1e-6, "fp32": 1e-4, "bf16": 5e-1}[prec]
    assert dist <= bound * np.abs(x64).max()
