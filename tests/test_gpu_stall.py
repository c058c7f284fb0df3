"""GPU parity of the stall handling of yand_mvsk_solve against the oracle:
the stall-recovery restarts of Table "YAND-MVSK parameter settings" (budget
set: twice the Krylov budget, then the direct solve; simplex boundary block:
projected trial steps 0.045, then 0.02), the stall test, the time budget,
the Krylov tolerance option and the unbounded line model.

Each case forces the path from the options (a Krylov budget of 1, an outer
budget of 2, a restart budget of 1 or 2, eps = 0, a tiny time budget) and
compares restarts, the iterations of every phase, the status and the
iterates.  The PCG iterates follow the oracle's element by element (same
preconditioner), so iterates are compared to 1e-9 like the other iterate
parity tests.
"""

import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2604_25378_amd import binding as yb  # noqa: E402


def _n12():
    R = synth.workload_returns("n12_T500")
    c = np.array(synth.WORKLOADS["n12_T500"]["c"])
    return R, c


def _both(R, c, oo, **kw):
    xr, ir = O.solve(R, c, opts=oo)
    ctx = yb.Context(torch.from_numpy(R).cuda())
    w, info = ctx.solve(c, opts=yb.default_opts(**kw))
    ctx.close()
    return xr, ir, w.cpu().numpy(), info


def _kappa_w(R, c, x, eps=1e-8):
    mu, A = O.center(R)
    U = O.tangent_basis(O.constraints(mu)[0])
    H = A.T @ (O.d2psi(c, A @ x)[:, None] * A) / A.shape[0]
    return 10 * eps / np.linalg.eigvalsh(U.T @ H @ U)[0]


def _phase_its(ir):
    its = [p[4] for p in ir.phases]
    return tuple(its + [0] * (3 - len(its)))


@pytest.mark.parametrize("restart_max_iter", [1, 120])
def test_budget_restarts_match_oracle(restart_max_iter):
    """krylov_maxit = 1, max_iter = 2: the baseline PCG phase ends above eps;
    with a restart budget of 1 both restarts run (the direct one converges),
    with 120 the first restart converges."""
    print(f"[case] budget stall restarts n12 restart_max_iter={restart_max_iter}",
          flush=True)
    R, c = _n12()
    oo = O.Options.large()
    oo.krylov_maxit, oo.max_iter, oo.restart_max_iter = 1, 2, restart_max_iter
    xr, ir, w, info = _both(R, c, oo, large=True, krylov_maxit=1, max_iter=2,
                            restart_max_iter=restart_max_iter)
    assert ir.restarts >= 1
    assert info.restarts == ir.restarts
    assert info.iterations == ir.iterations
    assert info.phase_iterations == _phase_its(ir)
    assert info.status == ir.status == 0
    assert info.cg_iters == ir.cg_iters
    assert np.abs(w - xr).max() <= 1e-9
    assert abs(info.f - ir.f) <= 1e-10 * abs(ir.f)


@pytest.mark.parametrize("restart_max_iter", [2, 120])
def test_simplex_restarts_match_oracle(restart_max_iter):
    """Simplex with the boundary block, max_iter = 2: the restarts lower the
    projected trial step to 0.045 and then 0.02.  With a restart budget of 2
    the solve is still above eps after both (a stall, status 2); with 120
    the first restart converges."""
    print(f"[case] simplex stall restarts n12 restart_max_iter={restart_max_iter}",
          flush=True)
    R, c = _n12()
    oo = O.Options.large()
    oo.feasible_set = "simplex"
    oo.max_iter, oo.restart_max_iter = 2, restart_max_iter
    xr, ir, w, info = _both(R, c, oo, large=True, feasible_set="simplex",
                            max_iter=2, restart_max_iter=restart_max_iter)
    assert ir.restarts >= 1
    assert info.restarts == ir.restarts
    assert info.iterations == ir.iterations
    assert info.phase_iterations == _phase_its(ir)
    assert info.projected_steps == ir.projected_steps
    assert info.status == ir.status
    assert ir.status == (2 if restart_max_iter == 2 else 0)
    assert np.abs(w - xr).max() <= 1e-9
    assert info.kkt == pytest.approx(ir.kkt, rel=1e-6, abs=1e-12)


def test_stall_test_reports_a_stall():
    """eps = 0 (direct configuration): the run ends at the stall test on both
    sides with status YAND_WARN_STALL, at the same minimum.  The decreases
    that trigger the test are a few ulps of f, so the iteration counts may
    differ by the rounding of those last steps."""
    print("[case] stall test eps=0 n12 direct", flush=True)
    R, c = _n12()
    xr, ir, w, info = _both(R, c, O.Options(eps=0.0), eps=0.0)
    assert ir.status == 2 and info.status == yb.YAND_WARN_STALL
    assert abs(info.iterations - ir.iterations) <= 2
    assert info.iterations < 300
    assert abs(info.f - ir.f) <= 1e-14 * abs(ir.f)
    assert np.abs(w - xr).max() <= 1e-9


def test_time_budget():
    """A time budget of 1e-9 s ends every phase before its first direction:
    no iteration runs; the PCG configuration runs both restarts and reports
    a stall, the direct one reports the budget.  max_elapsed = 0 means no
    limit."""
    print("[case] time budget n12", flush=True)
    R, c = _n12()
    oo = O.Options.large()
    oo.max_elapsed = 1e-9
    xr, ir, w, info = _both(R, c, oo, large=True, max_elapsed=1e-9)
    assert info.iterations == ir.iterations == 0
    assert info.restarts == ir.restarts == 2
    assert info.status == ir.status == yb.YAND_WARN_STALL
    assert np.abs(w - xr).max() == 0.0 or np.abs(w - xr).max() <= 1e-15
    xr, ir, w, info = _both(R, c, O.Options(max_elapsed=1e-9), max_elapsed=1e-9)
    assert info.iterations == ir.iterations == 0
    assert info.status == ir.status == yb.YAND_WARN_MAXITER
    xr, ir, w, info = _both(R, c, O.Options(max_elapsed=0.0), max_elapsed=0.0)
    assert info.status == ir.status == 0
    assert info.iterations == ir.iterations


def test_krylov_tol_option_is_honoured():
    """The PCG configuration runs at the caller's Krylov tolerance: with
    krylov_tol = 1e-10 the GPU solve follows the oracle's (same iterations,
    Krylov counts and weights) and differs from the default 1e-3."""
    print("[case] krylov_tol 1e-10 n300 PCG budget", flush=True)
    R = synth.factor_returns(300, 1000, 5, 0, 5.0, 0.0, 7)
    c = np.array([1.0, 5.0, 2.0, 10.0])
    oo = O.Options.large()
    oo.krylov_tol = 1e-10
    xr, ir, w, info = _both(R, c, oo, large=True, krylov_tol=1e-10)
    assert info.status == ir.status == 0
    assert info.iterations == ir.iterations
    assert info.cg_iters == ir.cg_iters
    # both solves stop at |gbar| <= eps: weights within 10 eps / lambda_min
    assert np.abs(w - xr).max() <= _kappa_w(R, c, xr)
    assert abs(info.f - ir.f) <= 1e-10 * abs(ir.f)
    _, ir3 = O.solve(R, c, opts=O.Options.large())
    ctx = yb.Context(torch.from_numpy(R).cuda())
    _, i3 = ctx.solve(c, opts=yb.default_opts(large=True))
    ctx.close()
    assert i3.cg_iters == ir3.cg_iters < info.cg_iters


def test_bad_krylov_tol_is_an_argument_error():
    R, c = _n12()
    ctx = yb.Context(torch.from_numpy(R).cuda())
    for tol in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(yb.YandError) as e:
            ctx.solve(c, opts=yb.default_opts(large=True, krylov_tol=tol))
        assert e.value.code == -1
    ctx.close()


@pytest.mark.parametrize("c", [(1.0, 1.0, 1.0, 0.0), (0.0, 1.0, 10.0, 0.0)])
def test_budget_line_without_kurtosis_is_unbounded(c):
    """c4 = 0 with c3 > 0 on the budget set: the oracle meets a line model
    that is a falling cubic and raises; the library returns
    YAND_ERR_UNBOUNDED."""
    print(f"[case] unbounded c={c}", flush=True)
    R, _ = _n12()
    c = np.array(c)
    with pytest.raises(O.Unbounded):
        O.solve(R, c)
    ctx = yb.Context(torch.from_numpy(R).cuda())
    with pytest.raises(yb.YandError) as e:
        ctx.solve(c)
    assert e.value.code == -6
    ctx.close()
