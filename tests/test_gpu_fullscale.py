"""GPU parity at the full benchmark size, n = 5440 assets x T = 12000 bars,
FP64 storage, through the same entry points and kernels the benchmark times.

The FP64 oracle still finishes at this size in seconds per call (one outer
iteration is a few dense products of 12000 x 5440 matrices), so whole outputs
are compared, not samples:
  - f, gradient and moments at two points: relative 1e-12 (sums of 12000
    terms in a different order);
  - Hessian-vector product: relative 1e-11 of the vector's scale;
  - line-search coefficients: relative 1e-10 of the largest coefficient;
  - affine-normal direction and one full outer iteration from equal weights:
    relative 1e-9 of |d|_inf (observed ~2e-11; the bound leaves room for the
    condition of the tangent Hessian times FP64 rounding);
  - a complete solve and twelve frontier instances: stationarity judged by the
    oracle, |U^T grad f(w)| <= 2e-8 with the oracle's own tangent basis, and
    the constraints to rounding.
"""

import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2604_25378_amd import binding as yb  # noqa: E402

WORKLOAD = "n5440_T12000"


@pytest.fixture(scope="module")
def full():
    print(f"[case] full scale {WORKLOAD}", flush=True)
    R = synth.workload_returns(WORKLOAD)
    c = np.array(synth.WORKLOADS[WORKLOAD]["c"])
    mu, A = O.center(R)
    ctx = yb.Context(torch.from_numpy(R).cuda(), "fp64")
    yield dict(R=R, c=c, mu=mu, A=A, ctx=ctx)
    ctx.close()


def _rel(got, ref):
    got, ref = np.asarray(got), np.asarray(ref)
    return np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)


def _point(mu, seed):
    n = mu.shape[0]
    x = np.full(n, 1.0 / n) + 0.3 / n * np.random.default_rng(seed).normal(size=n)
    return x - (x.sum() - 1.0) / n


def test_fullscale_passes(full):
    A, mu, c, ctx = full["A"], full["mu"], full["c"], full["ctx"]
    for seed in (None, 1):
        x = np.full(mu.shape[0], 1.0 / mu.shape[0]) if seed is None else _point(mu, seed)
        f, g, mom = ctx.eval(c, x)
        assert f == pytest.approx(O.objective(A, mu, c, x), rel=1e-12)
        assert _rel(g.cpu().numpy(), O.gradient(A, mu, c, x)) <= 1e-12
        assert _rel(mom, O.moments(A, mu, x)) <= 1e-12
    x = _point(mu, 2)
    v = np.random.default_rng(3).normal(size=mu.shape[0])
    assert _rel(ctx.hvp(c, x, v).cpu().numpy(), O.hvp(A, c, x, v)) <= 1e-11
    d = np.random.default_rng(4).normal(size=mu.shape[0])
    d -= d.mean()
    got = ctx.linesearch_coeffs(c, x, d)
    ref = O.linesearch_coeffs(A, mu, c, x, d)
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()


def test_fullscale_direction_and_first_iteration(full):
    R, A, mu, c, ctx = full["R"], full["A"], full["mu"], full["c"], full["ctx"]
    Cm, b = O.constraints(mu)
    U = O.tangent_basis(Cm)
    x = O.feasible_start(Cm, b)
    ref = O.affine_normal(A, mu, c, x, U)
    d, gn = ctx.affine_normal(c, x)
    err = _rel(d.cpu().numpy(), ref.d)
    print(f"direction relative error {err:.2e}", flush=True)
    assert gn == pytest.approx(ref.gnorm, rel=1e-12)
    assert err <= 1e-9
    xr, _ = O.solve(R, c, opts=O.Options(max_iter=1, eps=0.0))
    w, info = ctx.solve(c, opts=yb.default_opts(max_iter=1, eps=0.0))
    assert info.iterations == 1
    assert _rel(w.cpu().numpy() - 1.0 / mu.shape[0], xr - 1.0 / mu.shape[0]) <= 1e-9


def _oracle_gnorm(A, mu, c, w, target):
    Cm, _ = O.constraints(mu, target)
    U = O.tangent_basis(Cm)
    return float(np.linalg.norm(U.T @ O.gradient(A, mu, c, w)))


def test_fullscale_solve_certified_by_oracle(full):
    A, mu, c, ctx = full["A"], full["mu"], full["c"], full["ctx"]
    w, info = ctx.solve(c)
    w = w.cpu().numpy()
    print(f"solve: {info.iterations} iterations, |g| {info.gnorm:.2e}", flush=True)
    assert info.status == 0 and info.gnorm <= 1e-8
    assert abs(w.sum() - 1.0) <= 1e-12
    assert _oracle_gnorm(A, mu, c, w, None) <= 2e-8
    x0 = np.full(mu.shape[0], 1.0 / mu.shape[0])
    assert O.objective(A, mu, c, w) < O.objective(A, mu, c, x0)


def test_fullscale_solve_objective_matches_oracle_solve(full):
    """The full-scale solve against the oracle's own solve of the same
    instance: the same iterations and the objective to a relative error of
    1e-10 (FP64); the weights are certified separately by the oracle's
    reduced gradient."""
    R, A, mu, c, ctx = full["R"], full["A"], full["mu"], full["c"], full["ctx"]
    w, info = ctx.solve(c)
    w = w.cpu().numpy()
    xr, ir = O.solve(R, c)
    print(f"oracle: {ir.iterations} iterations, f {ir.f:.12e}; GPU: "
          f"{info.iterations} iterations, f {info.f:.12e}", flush=True)
    assert ir.status == 0 and info.status == 0
    assert info.iterations == ir.iterations
    f = O.objective(A, mu, c, w)
    assert abs(f - ir.f) <= 1e-10 * abs(ir.f)
    assert abs(info.f - ir.f) <= 1e-10 * abs(ir.f)
    assert _oracle_gnorm(A, mu, c, w, None) <= 2e-8


def test_fullscale_frontier_certified_by_oracle(full):
    """Twelve frontier instances in lockstep (four return targets x CRRA
    gamma 3, 5, 8): each stationary by the oracle's reduced gradient, on
    its budget and return constraints."""
    R, A, mu, ctx = full["R"], full["A"], full["mu"], full["ctx"]
    targets = synth.frontier_targets(R, 6)[1:5]
    gammas = (3.0, 5.0, 8.0)
    C4 = np.array([synth.crra_coefficients(g) for g in gammas for _ in targets])
    tg = np.tile(targets, len(gammas))
    W, infos = ctx.frontier(C4, tg)
    W = W.cpu().numpy()
    for b in range(len(tg)):
        assert infos[b].status == 0 and infos[b].gnorm <= 1e-8, infos[b]
        assert abs(W[b].sum() - 1.0) <= 1e-12
        assert abs(mu @ W[b] - tg[b]) <= 1e-12 * max(1.0, abs(tg[b]))
        assert _oracle_gnorm(A, mu, C4[b], W[b], tg[b]) <= 2e-8
