"""GPU parity in the FP32 and BF16 storage modes of A.

The library rounds A = R - 1 mu^T to the storage type once (round to
nearest even; BF16 through FP32).  The streaming passes (objective,
gradient, HVP, line-search sums) read the stored values and accumulate in
FP64, so the oracle runs on the same rounded matrix, built here from its
own centering with NumPy, and the GPU must match it to FP64 accumulation
accuracy.  The exact trace's products (B = A^T diag(psi'') A / T and the
rows of L^-1 A^T) run on the matrix cores with FP32 or BF16 inputs and FP32
accumulation, so the direction carries their rounding: it is compared with
the oracle's direction on the rounded matrix to a measured per-precision
bound, and to 1e-8 with those products in FP64 (dense_fp64 = 1).  The
error of each storage mode against the unrounded FP64 problem is also
measured and bounded (BF16 perturbs A by up to 2^-9 relative, FP32 by
2^-24).
"""

import numpy as np
import pytest

import oracle as O
import synth
from storage import round_storage

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2604_25378_amd import binding as yb  # noqa: E402


# error of the rounded problem against FP64, relative (measured bound)
F_BOUND = {"fp32": 1e-8, "bf16": 1e-3}


@pytest.fixture(scope="module", params=["fp32", "bf16"])
def pcase(request):
    prec = request.param
    R = synth.factor_returns(300, 1000, 5, 0, 5.0, 0.0, 7)
    c = np.array([1.0, 5.0, 2.0, 10.0])
    mu, A = O.center(R)
    Ar = round_storage(A, prec)
    print(f"[case] precision={prec} T=1000 n=300", flush=True)
    ctx = yb.Context(torch.from_numpy(R).cuda(), prec)
    yield dict(prec=prec, R=R, c=c, mu=mu, A=A, Ar=Ar, ctx=ctx)
    ctx.close()


def _x(mu, seed):
    n = mu.shape[0]
    x = np.full(n, 1.0 / n) + 0.1 / n * np.random.default_rng(seed).normal(size=n)
    return x - (x.sum() - 1.0) / n


def _rel(got, ref):
    return float(np.abs(np.asarray(got) - ref).max() / np.abs(ref).max())


def test_eval_hvp_ls_on_rounded_matrix(pcase):
    c, mu, A, Ar, ctx = pcase["c"], pcase["mu"], pcase["A"], pcase["Ar"], pcase["ctx"]
    x = _x(mu, 1)
    f, g, mom = ctx.eval(c, x)
    assert f == pytest.approx(O.objective(Ar, mu, c, x), rel=1e-11)
    assert _rel(g.cpu().numpy(), O.gradient(Ar, mu, c, x)) <= 1e-11
    # measured error of the storage mode against the FP64 problem
    assert abs(f - O.objective(A, mu, c, x)) <= F_BOUND[pcase["prec"]] * abs(f)
    v = np.random.default_rng(2).normal(size=mu.shape[0])
    assert _rel(ctx.hvp(c, x, v).cpu().numpy(), O.hvp(Ar, c, x, v)) <= 1e-11
    d = v - v.mean()
    coef = ctx.linesearch_coeffs(c, x, d)
    ref = O.linesearch_coeffs(Ar, mu, c, x, d)
    assert np.abs(coef - ref).max() <= 1e-11 * np.abs(ref).max()


# direction error of the matrix-core products (relative to |d|_inf),
# measured bound per storage precision
D_BOUND = {"fp32": 3e-4, "bf16": 5e-2}


@pytest.mark.parametrize("dense_fp64", [1, 0])
def test_direction_on_rounded_matrix(pcase, dense_fp64):
    c, mu, Ar, ctx = pcase["c"], pcase["mu"], pcase["Ar"], pcase["ctx"]
    Cm, b = O.constraints(mu)
    U = O.tangent_basis(Cm)
    x = O.feasible_start(Cm, b, _x(mu, 3))
    ref = O.affine_normal(Ar, mu, c, x, U)
    d, gn = ctx.affine_normal(c, x, opts=yb.default_opts(dense_fp64=dense_fp64))
    assert gn == pytest.approx(ref.gnorm, rel=1e-11)
    err = _rel(d.cpu().numpy(), ref.d)
    print(f"[precision] {pcase['prec']} dense_fp64={dense_fp64}: direction "
          f"error {err:.2e} relative to |d|_inf", flush=True)
    # the direction is a descent direction whatever the products' rounding:
    # g^T d = -|gbar| exactly in exact arithmetic
    g = O.gradient(Ar, mu, c, x)
    assert float(g @ d.cpu().numpy()) == pytest.approx(-ref.gnorm, rel=1e-6)
    assert err <= (1e-8 if dense_fp64 else D_BOUND[pcase["prec"]])


def test_solve_on_rounded_matrix(pcase):
    c, mu, A, Ar, ctx = pcase["c"], pcase["mu"], pcase["A"], pcase["Ar"], pcase["ctx"]
    w, info = ctx.solve(c)
    w = w.cpu().numpy()
    assert info.status == 0 and info.gnorm <= 1e-8
    Cm, _ = O.constraints(mu)
    U = O.tangent_basis(Cm)
    # stationary for the rounded problem, judged by the oracle
    assert np.linalg.norm(U.T @ O.gradient(Ar, mu, c, w)) <= 2e-8
    assert abs(w.sum() - 1.0) < 1e-12
    # distance to the FP64 minimiser is what the rounding of A implies:
    # report it through the FP64 reduced gradient at the returned weights
    g64 = np.linalg.norm(U.T @ O.gradient(A, mu, c, w))
    print(f"[precision] {pcase['prec']}: FP64 |gbar| at the {pcase['prec']} "
          f"solution = {g64:.3e}", flush=True)
    assert g64 <= {"fp32": 1e-8, "bf16": 1e-4}[pcase["prec"]]
