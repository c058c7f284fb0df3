"""GPU parity of the T < n push-through exact trace (PCG configuration with
2 T <= n) against the FP64 oracle, which factors the reduced tangent
Hessian explicitly.

Direction level: both sides run the PCG u-solve to convergence
(krylov_tol 1e-13), so the direction d = Q u - nu depends on the exact
trace alone and not on the two preconditioners (the library's Jacobi
preconditioner lives in ambient coordinates, the oracle's in reduced ones);
compared to 1e-8 of |d|_inf, the direction tolerance of the dense path.
Solve level: the PCG configuration with stall recovery on the simplex,
the converged minimiser to 1e-7.  Indefinite S: where psi'' < 0 at some
bars the identity runs on the signed factorisation of lambda S^-1 + G, with
the dense route's escalation of lambda.
"""

import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2604_25378_amd import binding as yb  # noqa: E402


def _close(got, ref, rtol):
    scale = max(np.abs(ref).max(), 1e-300)
    err = np.abs(np.asarray(got) - ref).max() / scale
    assert err <= rtol, f"relative error {err:.3e} > {rtol:.1e}"


CASES = {
    # uniform [-0.1, 0.4] returns, CRRA gamma = 6 (certified, psi'' > 0)
    "uniform_n400_T120": lambda: (synth.uniform_returns(400, 120, seed=4),
                                  synth.crra_coefficients(6.0)),
    # heavy-tailed factor panel, ragged T against the 32-row Gram tiles
    "factor_n640_T200": lambda: (synth.factor_returns(640, 200, 3, 0, 5.0,
                                                      0.0, 11),
                                 np.array([1.0, 5.0, 2.0, 10.0])),
}
# Relative regularisation 1e-2 in the direction tests.  With n > T the
# directions outside A's row space carry only lambda, so at the default
# 1e-4 the reduced system has cond ~ 1e4 and the converged PCG solves still
# differ by ~1e-8 in u on the two sides (residual floor ~1e-12 times the
# condition number), which would mask the trace; 1e-2 brings cond to ~1e2.
REG = {"uniform_n400_T120": 1e-2, "factor_n640_T200": 1e-2}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("with_target", [False, True])
def test_thin_direction_matches_oracle(name, with_target):
    print(f"[case] thin direction {name} target={with_target}", flush=True)
    R, c = CASES[name]()
    mu, A = O.center(R)
    n = mu.size
    target = float(np.quantile(mu, 0.6)) if with_target else None
    Cm, b = O.constraints(mu, target)
    U = O.tangent_basis(Cm)
    rng = np.random.default_rng(8)
    x0 = np.full(n, 1.0 / n) + 0.3 / n * rng.normal(size=n)
    x = O.feasible_start(Cm, b, x0 - (x0.sum() - 1.0) / n)
    ref = O.affine_normal(A, mu, c, x, U, solver="pcg", reg=REG[name],
                          krylov_tol=1e-13, krylov_maxit=4000)
    ctx = yb.Context(torch.from_numpy(R).cuda())
    opts = yb.default_opts(large=True, krylov_tol=1e-13, krylov_maxit=4000,
                           regularization=REG[name])
    d, gn = ctx.affine_normal(c, x, target=target, opts=opts)
    ctx.close()
    assert gn == pytest.approx(ref.gnorm, rel=1e-12)
    _close(d.cpu().numpy(), ref.d, 1e-8)


def test_thin_solve_matches_oracle():
    """Simplex, PCG configuration with stall recovery: a certified-convex
    instance with a unique minimiser; the per-iteration PCG solves stop at
    krylov_tol 1e-3 under different preconditioners, so the runs are
    compared at their converged point."""
    print("[case] thin solve uniform n400 T120 simplex", flush=True)
    R, c = CASES["uniform_n400_T120"]()
    mu, A = O.center(R)
    oo = O.Options.large()
    oo.feasible_set = "simplex"
    xr, ir = O.solve(R, c, opts=oo)
    ctx = yb.Context(torch.from_numpy(R).cuda())
    w, info = ctx.solve(c, opts=yb.default_opts(large=True,
                                                feasible_set="simplex"))
    ctx.close()
    w = w.cpu().numpy()
    print(f"GPU {info.status} {info.iterations} it kkt {info.kkt:.1e}; "
          f"oracle {ir.status} {ir.iterations} it", flush=True)
    assert info.status == 0 and ir.status == 0
    assert info.iterations == ir.iterations
    assert info.kkt <= 1e-8
    assert np.abs(w - xr).max() <= 1e-8
    assert O.objective(A, mu, c, w) == pytest.approx(
        O.objective(A, mu, c, xr), rel=1e-10)


@pytest.mark.parametrize("route", ["thin", "dense"])
@pytest.mark.parametrize("iters", [1, 4])
def test_pcg_iterates_match_oracle(route, iters):
    """Default PCG settings (krylov_tol 1e-3, 15 iterations): both sides use
    the Jacobi inverse of the ambient Hessian diagonal on the tangent space,
    so the truncated inner solves, and with them the outer iterates, agree
    element by element.  thin: n = 400, T = 120 (2 T <= n) on the simplex
    (on the budget hull with n > T the iterates run off along A's null
    space, where every difference grows); dense: n = 300, T = 1000 on the
    budget hull."""
    print(f"[case] PCG iterates route={route} iters={iters}", flush=True)
    if route == "thin":
        R, c = CASES["uniform_n400_T120"]()
        fs = "simplex"
    else:
        R = synth.factor_returns(300, 1000, 5, 0, 5.0, 0.0, 7)
        c = np.array([1.0, 5.0, 2.0, 10.0])
        fs = "budget"
    oo = O.Options.large()
    oo.max_iter, oo.eps, oo.stall_recovery = iters, 0.0, False
    oo.feasible_set = fs
    xr, ir = O.solve(R, c, opts=oo)
    ctx = yb.Context(torch.from_numpy(R).cuda())
    w, info = ctx.solve(c, opts=yb.default_opts(large=True, max_iter=iters,
                                                eps=0.0, stall_recovery=0,
                                                feasible_set=fs))
    ctx.close()
    assert info.iterations == iters and info.cg_iters == ir.cg_iters
    # the direction tolerance: a different preconditioner would differ at
    # the truncation level (krylov_tol 1e-3), rounding stays near 1e-9
    _close(w.cpu().numpy(), xr, 1e-8)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_thin_reduced_storage_matches_rounded_oracle(precision):
    """FP32/BF16 storage: the Gram and diagonal kernels read the stored A;
    the oracle runs on the same rounded matrix."""
    print(f"[case] thin direction storage={precision}", flush=True)
    R, c = CASES["factor_n640_T200"]()
    mu, A = O.center(R)
    f32 = A.astype(np.float32)
    if precision == "fp32":
        Ar = f32.astype(np.float64)
    else:
        bits = f32.view(np.uint32).astype(np.uint64)
        bits = (bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000
        Ar = bits.astype(np.uint32).view(np.float32).astype(np.float64)
    n = mu.size
    Cm, b = O.constraints(mu, None)
    U = O.tangent_basis(Cm)
    x = np.full(n, 1.0 / n)
    ref = O.affine_normal(Ar, mu, c, x, U, solver="pcg", reg=1e-2,
                          krylov_tol=1e-13, krylov_maxit=4000)
    ctx = yb.Context(torch.from_numpy(R).cuda(), precision)
    opts = yb.default_opts(large=True, krylov_tol=1e-13, krylov_maxit=4000,
                           regularization=1e-2)
    d, _ = ctx.affine_normal(c, x, opts=opts)
    ctx.close()
    _close(d.cpu().numpy(), ref.d, 1e-8)


def _concentrated_indefinite():
    """c = (10, 1, 10, 1): psi''(s) = 2 - 60 s + 12 s^2 is negative for
    0.034 < s < 4.97, which the centred uniform returns reach from a
    concentrated portfolio (|z_t| up to 0.2): S is indefinite."""
    R = synth.uniform_returns(300, 120, seed=5)
    c = np.array([10.0, 1.0, 10.0, 1.0])
    mu, A = O.center(R)
    x = np.full(mu.size, 0.1 / mu.size)
    x[7] += 0.9
    s2 = O.d2psi(c, A @ x)
    assert s2.min() < 0.0 < s2.max()
    return R, c, mu, A, x, int((s2 < 0).sum())


@pytest.mark.parametrize("reg", [1e-4, 1e-9])
def test_thin_indefinite_matches_oracle(reg):
    """psi'' < 0 at some bars: the push-through runs on the signed
    factorisation of W = lambda S^-1 + G (no n x n matrix; the profile shows
    the signed factorisation and no SYRK) and gives the oracle's direction,
    whose explicit reduced factorisation escalates lambda on failure.  At
    reg 1e-9 the tangent Hessian plus lambda is indefinite at first, so both
    sides escalate; a different number of escalations would move the
    direction by far more than the tolerance."""
    print(f"[case] thin indefinite reg={reg}", flush=True)
    R, c, mu, A, x, nneg = _concentrated_indefinite()
    print(f"  {nneg} of {R.shape[0]} bars with psi'' < 0", flush=True)
    U = O.tangent_basis(O.constraints(mu, None)[0])
    ref = O.affine_normal(A, mu, c, x, U, solver="pcg", reg=reg,
                          krylov_tol=1e-13, krylov_maxit=4000)
    ctx = yb.Context(torch.from_numpy(R).cuda())
    ctx.profile(True)
    opts = yb.default_opts(large=True, krylov_tol=1e-13, krylov_maxit=4000,
                           regularization=reg)
    d, gn = ctx.affine_normal(c, x, opts=opts)
    prof = {k: v[1] for k, v in ctx.profile_read().items()}
    ctx.close()
    print(f"  oracle lambda {ref.lam:.3e}; kernels {sorted(prof)}", flush=True)
    assert "thin_indef_factor" in prof and "syrk" not in prof
    assert gn == pytest.approx(ref.gnorm, rel=1e-12)
    _close(d.cpu().numpy(), ref.d, 1e-8)
    if reg == 1e-9:
        assert prof["thin_indef_factor"] >= 2       # escalated at least once


def test_thin_indefinite_simplex_solve():
    """Simplex, PCG configuration, c = (10, 1, 10, 1) on the uniform n = 300,
    T = 120 panel (2T <= n): directions with psi'' < 0 on some bars take the
    signed factorisation.  Outside the convexity certificate the two runs
    need not take the same path to a stationary point, so the check is the
    outcome: the run ends without error on the push-through route only
    (thin_traces = dense_traces), at a point of the slice whose projected
    KKT residual and objective the oracle recomputes to the library's."""
    print("[case] thin indefinite simplex solve n=300 T=120", flush=True)
    R = synth.uniform_returns(300, 120, seed=5)
    c = np.array([10.0, 1.0, 10.0, 1.0])
    mu, A = O.center(R)
    ctx = yb.Context(torch.from_numpy(R).cuda())
    w, info = ctx.solve(c, opts=yb.default_opts(large=True,
                                                feasible_set="simplex"))
    ctx.close()
    w = w.cpu().numpy()
    print(f"  status {info.status} iterations {info.iterations} traces "
          f"{info.dense_traces} thin {info.thin_traces} kkt {info.kkt:.1e}",
          flush=True)
    assert info.status in (0, 1, 2)
    assert info.thin_traces == info.dense_traces > 0
    assert abs(w.sum() - 1.0) <= 1e-12 and w.min() >= 1e-8 - 1e-15
    g = O.gradient(A, mu, c, w)
    kkt = float(np.linalg.norm(w - O.project_simplex(w - g, 1e-8)))
    assert kkt == pytest.approx(info.kkt, rel=1e-6, abs=1e-14)
    assert O.objective(A, mu, c, w) == pytest.approx(info.f, rel=1e-12)
    # lower than the equal-weight start
    x0 = np.full(300, 1.0 / 300)
    assert info.f < O.objective(A, mu, c, x0)
