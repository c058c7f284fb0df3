"""Pins of the oracle's stall handling: the stall test, the time and
iteration budgets, and the stall-recovery restarts of Table "YAND-MVSK
parameter settings" (restarts with twice the Krylov budget and then the
direct solve on the budget set; projected trial steps 0.045 and then 0.02
on the simplex; 120 iterations per restart).

The schedule is checked by recording what the outer loop and the direction
actually receive, and every recovered solve is checked against a minimiser
computed another way: Newton's method on the explicit moment tensors for the
budget set, SLSQP over the simplex.
"""

import math

import numpy as np
import pytest
from scipy.optimize import minimize

import oracle as O
import oracle.mvsk as M
import synth


def _n12():
    R = synth.workload_returns("n12_T500")
    c = np.array(synth.WORKLOADS["n12_T500"]["c"])
    return R, c


def _tensor_newton(A, mu, c, U, x):
    """Newton's method on f written with the explicit covariance,
    coskewness and cokurtosis tensors (Section 2), in the tangent space."""
    T = A.shape[0]
    Sig = A.T @ A / T
    S = np.einsum("ti,tj,tk->ijk", A, A, A) / T
    K = np.einsum("ti,tj,tk,tl->ijkl", A, A, A, A) / T
    for _ in range(60):
        g = (-c[0] * mu + 2 * c[1] * Sig @ x
             - 3 * c[2] * np.einsum("ijk,i,j->k", S, x, x)
             + 4 * c[3] * np.einsum("ijkl,i,j,k->l", K, x, x, x))
        H = (2 * c[1] * Sig - 6 * c[2] * np.einsum("ijk,i->jk", S, x)
             + 12 * c[3] * np.einsum("ijkl,i,j->kl", K, x, x))
        step = U @ np.linalg.solve(U.T @ H @ U, U.T @ g)
        x = x - step
        if np.linalg.norm(step) < 1e-15:
            break
    return x


class _Spy:
    """Records the arguments of the outer-loop phases and of the direction
    calls while delegating to the oracle's own functions."""

    def __init__(self, monkeypatch):
        self.phases, self.dirs = [], []
        it, an = M._iterate, M.affine_normal

        def iterate(A, mu, c, x, U, opts, solver, krylov_maxit, max_iter,
                    info, t0, eta=None):
            self.phases.append((solver, krylov_maxit, max_iter, eta))
            return it(A, mu, c, x, U, opts, solver, krylov_maxit, max_iter,
                      info, t0, eta)

        def affine(*a, **k):
            self.dirs.append((len(self.phases) - 1, k.get("solver"),
                              k.get("krylov_maxit"), k.get("reg")))
            return an(*a, **k)

        monkeypatch.setattr(M, "_iterate", iterate)
        monkeypatch.setattr(M, "affine_normal", affine)


def test_budget_restarts_double_krylov_then_direct(monkeypatch):
    """krylov_maxit = 1 and max_iter = 2 force the baseline PCG phase to end
    above eps; the restarts then run PCG with 2 Krylov iterations and the
    direct solve (no regularisation), each for restart_max_iter iterations."""
    R, c = _n12()
    spy = _Spy(monkeypatch)
    o = O.Options.large()
    o.krylov_maxit, o.max_iter, o.restart_max_iter = 1, 2, 1
    x, info = O.solve(R, c, opts=o)
    assert spy.phases == [("pcg", 1, 2, 0.05), ("pcg", 2, 1, 0.05),
                          ("direct", 0, 1, 0.05)]
    # every direction of a phase uses that phase's solver and budget
    want = {0: ("pcg", 1, 1e-4), 1: ("pcg", 2, 1e-4), 2: ("direct", 0, 0.0)}
    assert [d[0] for d in spy.dirs] == [0, 0, 1, 2]
    for ph, solver, kmax, reg in spy.dirs:
        assert (solver, kmax, reg) == want[ph]
    assert info.restarts == 2 and info.iterations == 4
    assert [p[4] for p in info.phases] == [2, 1, 1]
    assert [p[5] for p in info.phases] == ["budget", "budget", "converged"]
    assert info.status == 0 and info.gnorm <= o.eps


def test_budget_restart_reaches_the_tensor_newton_minimiser():
    """With the paper's restart budget (120) the first restart converges to
    the minimiser that Newton's method finds on the explicit tensors."""
    R, c = _n12()
    mu, A = O.center(R)
    o = O.Options.large()
    o.krylov_maxit, o.max_iter = 1, 2
    assert o.restart_max_iter == 120
    x, info = O.solve(R, c, opts=o)
    assert info.restarts == 1 and info.status == 0
    assert info.phases[1][:3] == ("pcg", 2, 120)
    C, b = O.constraints(mu)
    U = O.tangent_basis(C)
    xn = _tensor_newton(A, mu, c, U, O.feasible_start(C, b))
    Hr = U.T @ (A.T @ (O.d2psi(c, A @ xn)[:, None] * A) / A.shape[0]) @ U
    lmin = np.linalg.eigvalsh(Hr)[0]
    assert np.linalg.norm(x - xn) <= 2 * o.eps / lmin + 1e-12


def _slsqp(A, mu, c):
    n = mu.size
    r = minimize(lambda x: O.objective(A, mu, c, x), np.full(n, 1.0 / n),
                 jac=lambda x: O.gradient(A, mu, c, x), method="SLSQP",
                 bounds=[(0.0, 1.0)] * n,
                 constraints=[{"type": "eq", "fun": lambda x: x.sum() - 1.0,
                               "jac": lambda x: np.ones_like(x)}],
                 options={"ftol": 1e-15, "maxiter": 1000})
    return r.x, r.fun


def test_simplex_restarts_use_the_projected_steps_0045_then_002(monkeypatch):
    """On the simplex with the boundary block the restarts keep the PCG
    configuration and lower the nominal projected trial step to 0.045 and
    then 0.02; a solve still above eps after both reports a stall."""
    R, c = _n12()
    spy = _Spy(monkeypatch)
    o = O.Options.large()
    o.feasible_set = "simplex"
    o.max_iter, o.restart_max_iter = 2, 2
    x, info = O.solve(R, c, opts=o)
    assert spy.phases == [("pcg", 15, 2, 0.05), ("pcg", 15, 2, 0.045),
                          ("pcg", 15, 2, 0.02)]
    assert all(d[1:] == ("pcg", 15, 1e-4) for d in spy.dirs)
    assert info.restarts == 2 and info.iterations == 6
    assert info.status == 2 and info.kkt > o.eps


def test_simplex_restart_reaches_the_slsqp_minimiser():
    R, c = _n12()
    mu, A = O.center(R)
    o = O.Options.large()
    o.feasible_set = "simplex"
    o.max_iter = 2
    x, info = O.solve(R, c, opts=o)
    assert info.restarts == 1 and info.status == 0
    assert info.phases[1][3] == 0.045
    xs, fs = _slsqp(A, mu, c)
    g = O.gradient(A, mu, c, x)
    assert info.f <= fs + 2.0 * mu.size * 1e-8 * np.abs(g).max() + 1e-12 * abs(fs)
    assert np.abs(x - xs).max() <= 1e-5


def test_stall_test_needs_three_small_decreases():
    """With eps = 0 the gradient test never fires; the run ends at the stall
    test once three iterations in a row decrease f by less than 1e-14 |f|,
    and not before, at the tensor-Newton minimum."""
    R, c = _n12()
    mu, A = O.center(R)
    x, info = O.solve(R, c, opts=O.Options(eps=0.0))
    assert info.status == 2 and info.phases[0][5] == "stall"
    assert info.iterations < 300
    f = [O.objective(A, mu, c, O.feasible_start(*O.constraints(mu)))]
    f += [h[2] for h in info.history]
    small = [f[i] - f[i + 1] < 1e-14 * abs(f[i]) for i in range(len(f) - 1)]
    assert small[-3:] == [True, True, True]
    assert not any(all(small[i:i + 3]) for i in range(len(small) - 3))
    C, b = O.constraints(mu)
    xn = _tensor_newton(A, mu, c, O.tangent_basis(C), O.feasible_start(C, b))
    fn = O.objective(A, mu, c, xn)
    assert abs(info.f - fn) <= 1e-14 * abs(fn)


def test_time_budget():
    """max_elapsed > 0 ends a phase before its next direction once that many
    seconds have passed (here at once: no iteration runs); with the PCG
    configuration every restart times out too and the solve reports a
    stall.  max_elapsed <= 0 means no time limit."""
    R, c = _n12()
    o = O.Options.large()
    o.max_elapsed = 1e-9
    x, info = O.solve(R, c, opts=o)
    assert info.iterations == 0 and info.restarts == 2 and info.status == 2
    assert [p[5] for p in info.phases] == ["time"] * 3
    x, info = O.solve(R, c, opts=O.Options(max_elapsed=1e-9))
    assert info.iterations == 0 and info.status == 1
    x, info = O.solve(R, c, opts=O.Options(max_elapsed=0.0))
    assert info.status == 0 and info.gnorm <= 1e-8


@pytest.mark.parametrize("c", [(1.0, 1.0, 1.0, 0.0), (0.0, 1.0, 10.0, 0.0)])
def test_budget_line_without_kurtosis_is_unbounded(c):
    """c4 = 0 with c3 > 0 on the budget set: once a direction meets a line
    model that is a cubic with a negative leading coefficient, f has no
    minimiser on that ray (checked on f itself) and the solve raises."""
    R, _ = _n12()
    mu, A = O.center(R)
    c = np.array(c)
    C, b = O.constraints(mu)
    U = O.tangent_basis(C)
    x = O.feasible_start(C, b)
    for _ in range(50):
        d = O.affine_normal(A, mu, c, x, U).d
        coef = O.linesearch_coeffs(A, mu, c, x, d)
        assert coef[4] == 0.0
        if coef[3] < 0.0:
            break
        x = x + O.select_step(coef) * d
    else:
        pytest.fail("no unbounded line within 50 iterations")
    # past a0 the cubic term dominates: f falls without bound along the ray
    a0 = 10.0 * max(1.0, abs(coef[2] / coef[3]),
                    math.sqrt(abs(coef[1] / coef[3])))
    f0 = O.objective(A, mu, c, x)
    fs = [O.objective(A, mu, c, x + a * d) for a in (a0, 10 * a0, 100 * a0)]
    assert fs[0] > fs[1] > fs[2] and fs[2] < -1e3 * abs(f0)
    with pytest.raises(O.Unbounded):
        O.select_step(coef)
    with pytest.raises(O.Unbounded):
        O.solve(R, c)
    assert math.isinf(O.Options().max_elapsed)
