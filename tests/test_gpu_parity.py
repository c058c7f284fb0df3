"""GPU parity: every libyand entry point against the FP64 CPU oracle.

Tolerances (FP64 storage): pass results (f, gradient, HVP, line-search
coefficients) agree to 1e-12 relative to the vector's scale; the direction
involves a factorisation of the tangent Hessian, so it is compared to
1e-8 relative to |d|_inf (condition number ~1e3 times rounding); solves are
compared through the objective (relative 1e-10) and the weights within
10 eps / lambda_min of the reduced Hessian, the accuracy that stationarity
|gbar| <= eps implies under strong convexity.
"""

import math

import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2604_25378_amd import binding as yb  # noqa: E402


def _inst(name):
    if name == "n12_T500":
        R = synth.workload_returns("n12_T500")
        c = np.array(synth.WORKLOADS["n12_T500"]["c"])
    elif name == "n300_T1000":          # 3 column tiles with a ragged edge,
        R = synth.factor_returns(300, 1000, 5, 0, 5.0, 0.0, 7)   # ragged rows
        c = np.array([1.0, 5.0, 2.0, 10.0])
    elif name == "n2_T40":              # smallest universe: m = 1
        R = synth.factor_returns(2, 40, 1, 0, 5.0, 0.0, 9)
        c = np.array([1.0, 1.0, 1.0, 1.0])
    else:
        raise KeyError(name)
    return R, c


INSTANCES = ["n12_T500", "n300_T1000", "n2_T40"]


@pytest.fixture(scope="module", params=INSTANCES)
def case(request):
    R, c = _inst(request.param)
    print(f"[case] {request.param} T={R.shape[0]} n={R.shape[1]}", flush=True)
    mu, A = O.center(R)
    ctx = yb.Context(torch.from_numpy(R).cuda(), "fp64")
    yield dict(name=request.param, R=R, c=c, mu=mu, A=A, ctx=ctx)
    ctx.close()


def _feasible_point(mu, seed, scale=0.3):
    n = mu.shape[0]
    rng = np.random.default_rng(seed)
    x = np.full(n, 1.0 / n) + scale / n * rng.normal(size=n)
    return x - (x.sum() - 1.0) / n


def _close(got, ref, rtol):
    got = np.asarray(got)
    ref = np.asarray(ref)
    scale = max(np.abs(ref).max(), 1e-300)
    err = np.abs(got - ref).max() / scale
    assert err <= rtol, f"relative error {err:.3e} > {rtol:.1e}"


def test_mu(case):
    _close(case["ctx"].mu().cpu().numpy(), case["mu"], 1e-14)


def test_eval(case):
    A, mu, c, ctx = case["A"], case["mu"], case["c"], case["ctx"]
    for seed in range(2):
        x = _feasible_point(mu, seed)
        f, g, mom = ctx.eval(c, x)
        assert f == pytest.approx(O.objective(A, mu, c, x), rel=1e-12)
        _close(g.cpu().numpy(), O.gradient(A, mu, c, x), 1e-12)
        _close(mom, O.moments(A, mu, x), 1e-12)


def test_hvp(case):
    A, mu, c, ctx = case["A"], case["mu"], case["c"], case["ctx"]
    x = _feasible_point(mu, 3)
    v = np.random.default_rng(4).normal(size=mu.shape[0])
    _close(ctx.hvp(c, x, v).cpu().numpy(), O.hvp(A, c, x, v), 1e-12)


def test_linesearch_coeffs(case):
    A, mu, c, ctx = case["A"], case["mu"], case["c"], case["ctx"]
    x = _feasible_point(mu, 5)
    d = np.random.default_rng(6).normal(size=mu.shape[0])
    d -= d.mean()
    got = ctx.linesearch_coeffs(c, x, d)
    ref = O.linesearch_coeffs(A, mu, c, x, d)
    for i in range(5):
        assert got[i] == pytest.approx(ref[i], rel=1e-11, abs=1e-13 * np.abs(ref).max())


def test_select_step_matches_oracle(case):
    ctx = case["ctx"]
    rng = np.random.default_rng(11)
    for k in range(40):
        coef = rng.normal(size=5) * 10.0 ** rng.integers(-6, 2, size=5)
        coef[1] = -abs(coef[1])
        coef[4] = abs(coef[4])
        amax = math.inf if k % 2 == 0 else float(rng.uniform(0.1, 50.0))
        try:
            ref = O.select_step(coef, amax)
        except O.Unbounded:
            with pytest.raises(yb.YandError):
                ctx.select_step(coef, amax)
            continue
        got = ctx.select_step(coef, amax)
        vr, vg = O.quartic_value(coef, ref), O.quartic_value(coef, got)
        assert got == pytest.approx(ref, rel=1e-10, abs=1e-300) or \
            abs(vg - vr) <= 1e-14 * (abs(coef[0]) + 1e-300)


def test_select_step_unbounded(case):
    with pytest.raises(yb.YandError) as e:
        case["ctx"].select_step([0.0, -1.0, 0.5, -0.2, 0.0], math.inf)
    assert e.value.code == -6


@pytest.mark.parametrize("with_target", [False, True])
def test_affine_normal(case, with_target):
    A, mu, c, ctx = case["A"], case["mu"], case["c"], case["ctx"]
    if with_target and mu.shape[0] < 3:
        pytest.skip("target needs n >= 3")
    target = float(np.quantile(mu, 0.6)) if with_target else None
    Cm, b = O.constraints(mu, target)
    U = O.tangent_basis(Cm)
    x = O.feasible_start(Cm, b, _feasible_point(mu, 8))
    ref = O.affine_normal(A, mu, c, x, U)
    d, gn = ctx.affine_normal(c, x, target=target)
    assert gn == pytest.approx(ref.gnorm, rel=1e-12)
    _close(d.cpu().numpy(), ref.d, 1e-8)


def _kappa_w(A, mu, c, x, target, eps):
    Cm, _ = O.constraints(mu, target)
    U = O.tangent_basis(Cm)
    z = A @ x
    Hr = U.T @ (A.T @ (O.d2psi(c, z)[:, None] * A) / A.shape[0]) @ U
    return 10.0 * eps / np.linalg.eigvalsh(Hr)[0]


@pytest.mark.parametrize("with_target", [False, True])
def test_solve_direct(case, with_target):
    R, A, mu, c, ctx = case["R"], case["A"], case["mu"], case["c"], case["ctx"]
    if with_target and mu.shape[0] < 3:
        pytest.skip("target needs n >= 3")
    target = float(np.quantile(mu, 0.6)) if with_target else None
    xr, ir = O.solve(R, c, target=target)
    w, info = ctx.solve(c, target=target)
    w = w.cpu().numpy()
    assert info.status == 0 and info.gnorm <= 1e-8
    assert info.f == pytest.approx(ir.f, rel=1e-10)
    assert abs(w.sum() - 1.0) < 1e-12
    if target is not None:
        assert abs(mu @ w - target) < 1e-12 * max(1.0, abs(target)) + 1e-15
    kw = _kappa_w(A, mu, c, xr, target, 1e-8)
    assert np.abs(w - xr).max() <= kw
    # stationarity judged by the oracle at the returned weights
    Cm, _ = O.constraints(mu, target)
    U = O.tangent_basis(Cm)
    assert np.linalg.norm(U.T @ O.gradient(A, mu, c, w)) <= 2e-8


def test_solve_pcg_matches_unique_minimiser(case):
    R, A, mu, c, ctx = case["R"], case["A"], case["mu"], case["c"], case["ctx"]
    xr, _ = O.solve(R, c)
    w, info = ctx.solve(c, opts=yb.default_opts(large=True))
    w = w.cpu().numpy()
    assert info.status == 0 and info.gnorm <= 1e-8
    assert np.abs(w - xr).max() <= _kappa_w(A, mu, c, xr, None, 1e-8)


def test_first_step_matches_oracle(case):
    """One outer iteration from equal weights, element by element."""
    R, A, mu, c, ctx = case["R"], case["A"], case["mu"], case["c"], case["ctx"]
    o = O.Options(max_iter=1, eps=0.0)
    xr, _ = O.solve(R, c, opts=o)
    w, info = ctx.solve(c, opts=yb.default_opts(max_iter=1, eps=0.0))
    assert info.iterations == 1
    _close(w.cpu().numpy(), xr, 1e-9)


def test_nonfinite_and_bad_coefficients():
    R = synth.factor_returns(5, 30, 1, 0, 5.0, 0.0, 1)
    R[3, 2] = np.nan
    with pytest.raises(yb.YandError) as e:
        yb.Context(torch.from_numpy(R).cuda())
    assert e.value.code == -2
    R[3, 2] = 0.0
    ctx = yb.Context(torch.from_numpy(R).cuda())
    with pytest.raises(yb.YandError) as e:
        ctx.eval([1.0, -1.0, 0.0, 1.0], np.full(5, 0.2))
    assert e.value.code == -1
    ctx.close()


def test_solve_R_wrapper():
    R, c = _inst("n12_T500")
    w = yb.solve_R(torch.from_numpy(R).cuda(), c).cpu().numpy()
    xr, _ = O.solve(R, c)
    mu, A = O.center(R)
    assert np.abs(w - xr).max() <= _kappa_w(A, mu, c, xr, None, 1e-8)


@pytest.mark.parametrize("iters", [1, 2, 4])
def test_simplex_iterations_match_oracle(iters):
    """SIMPLEX set with capped raw steps only (eta = 0): the interior-safe
    step cap binds from the first step on n12_T500 with c = (1,1,1,1) (the
    budget minimiser holds weights near -21); the GPU iterates follow the
    oracle's element by element."""
    R = synth.workload_returns("n12_T500")
    c = np.array([1.0, 1.0, 1.0, 1.0])
    print(f"[case] simplex n12_T500 iters={iters}", flush=True)
    xr, _ = O.solve(R, c, opts=O.Options(feasible_set="simplex", max_iter=iters, eps=0.0,
                                         eta=0.0))
    ctx = yb.Context(torch.from_numpy(R).cuda())
    w, info = ctx.solve(c, opts=yb.default_opts(feasible_set="simplex", max_iter=iters,
                                                eps=0.0, eta=0.0))
    w = w.cpu().numpy()
    assert info.iterations == iters
    assert np.abs(w - xr).max() <= 1e-9
    assert w.min() >= 1e-8 * (1 - 1e-6) and abs(w.sum() - 1.0) <= 1e-12
    assert xr.min() < 1e-7          # the cap is active
    ctx.close()
