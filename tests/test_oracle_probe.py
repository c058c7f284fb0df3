"""Pins of the oracle's probe estimate of the trace (the Krylov reduced
solve of Appendix C with Hutchinson's diagonal estimator): the counter-based
sign generator against SplitMix64's published outputs, the estimator's
unbiasedness and variance against the exact diagonal computed from explicit
matrices, the descent identity g^T d = -|gbar| of the resulting direction,
and solves that reach the tensor-Newton minimiser."""

import numpy as np
import pytest

import oracle as O
import oracle.mvsk as M
import synth

GAMMA = 0x9E3779B97F4A7C15


def test_splitmix64_published_outputs():
    """SplitMix64 (Steele, Lea and Flood 2014) seeded with 1234567 gives
    6457827717110365317, 3203168211198807973, 9817491932198370423,
    4593380528125082431, 16408922859458223821: the generator's widely
    reproduced reference sequence."""
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    states = np.array([(1234567 + i * GAMMA) % (1 << 64) for i in range(5)],
                      dtype=np.uint64)
    assert [int(v) for v in O.splitmix64(states)] == want


def test_rademacher_signs():
    X = O.rademacher(7, 3, 4000, 64)
    assert X.shape == (4000, 64) and set(np.unique(X)) == {-1.0, 1.0}
    # balanced and uncorrelated across rows, columns and draws
    assert abs(X.mean()) < 4.0 / np.sqrt(X.size)
    Cc = X.T @ X / 4000.0
    assert np.abs(Cc - np.eye(64)).max() < 5.0 / np.sqrt(4000)
    Y = O.rademacher(7, 4, 4000, 64)
    assert abs(np.mean(X * Y)) < 4.0 / np.sqrt(X.size)
    assert np.array_equal(X, O.rademacher(7, 3, 4000, 64))
    assert not np.array_equal(X, O.rademacher(8, 3, 4000, 64))
    # a column does not depend on how many columns are drawn
    assert np.array_equal(X[:, :5], O.rademacher(7, 3, 4000, 5))


def _instance(n=8, T=60, seed=4):
    R = synth.factor_returns(n, T, 2, 0, 5.0, 0.0, seed)
    mu, A = O.center(R)
    c = np.array([1.0, 3.0, 7.0, 14.0])
    C, b = O.constraints(mu)
    U = O.tangent_basis(C)
    rng = np.random.default_rng(seed)
    x = O.feasible_start(C, b, np.full(n, 1.0 / n) + 0.05 * rng.standard_normal(n) / n)
    return R, mu, A, c, U, x


def _explicit_M(A, mu, c, x, U, reg):
    """P H^-1 P^T with P = A U Q from explicit matrices (Section 4.2)."""
    T = A.shape[0]
    g = O.gradient(A, mu, c, x)
    gbar = U.T @ g
    nu = gbar / np.linalg.norm(gbar)
    # an orthonormal basis of nu-perp in the reduced space, from an SVD
    # (any basis gives the same P H^-1 P^T)
    W = np.linalg.svd(np.eye(len(nu)) - np.outer(nu, nu))[0][:, :len(nu) - 1]
    P = A @ U @ W
    B0 = P.T @ (O.d2psi(c, A @ x)[:, None] * P) / T
    lam = reg * np.trace(B0) / B0.shape[0]
    return P @ np.linalg.solve(B0 + lam * np.eye(B0.shape[0]), P.T)


def test_probe_estimate_is_unbiased_with_the_hutchinson_variance():
    """With exact inner solves, q_t averaged over many draws converges to
    the diagonal of P H^-1 P^T; single-draw estimates scatter with variance
    k^-1 sum_{s != t} M_ts^2 (independent signs)."""
    R, mu, A, c, U, x = _instance()
    Mx = _explicit_M(A, mu, c, x, U, 1e-4)
    q_exact = np.diag(Mx)
    ex = O.affine_normal(A, mu, c, x, U, solver="pcg", reg=1e-4,
                         krylov_tol=1e-15, krylov_maxit=200)
    assert np.allclose(ex.q, q_exact, rtol=1e-9, atol=0.0)
    k, draws = 16, 600
    est = np.array([O.affine_normal(A, mu, c, x, U, solver="pcg", reg=1e-4,
                                    krylov_tol=1e-15, krylov_maxit=200,
                                    trace="probe", probes=k, seed=11,
                                    draw=i).q for i in range(draws)])
    var = (np.sum(Mx * Mx, axis=1) - q_exact ** 2) / k
    zt = (est.mean(axis=0) - q_exact) / np.sqrt(var / draws)
    assert np.abs(zt).max() < 5.0
    ratio = est.var(axis=0, ddof=1) / var
    assert np.all((ratio > 0.7) & (ratio < 1.3))


def test_probe_direction_is_a_descent_direction():
    R, mu, A, c, U, x = _instance(n=12, T=80, seed=5)
    g = O.gradient(A, mu, c, x)
    dr = O.affine_normal(A, mu, c, x, U, solver="pcg", reg=1e-4,
                         trace="probe", probes=8, seed=1, draw=0)
    assert g @ dr.d == pytest.approx(-dr.gnorm, rel=1e-9)
    assert abs(dr.d.sum()) < 1e-13
    assert dr.probe_iters > 0


def test_many_probes_approach_the_exact_direction():
    R, mu, A, c, U, x = _instance(n=10, T=70, seed=6)
    kw = dict(solver="pcg", reg=1e-4, krylov_tol=1e-14, krylov_maxit=200)
    de = O.affine_normal(A, mu, c, x, U, **kw).d
    errs = []
    for k in (16, 1024):     # 1024: the largest block the counter covers
        dp = O.affine_normal(A, mu, c, x, U, trace="probe", probes=k, seed=2,
                             **kw).d
        errs.append(np.abs(dp - de).max() / np.abs(de).max())
    # Monte Carlo error of the correction shrinks about like 1 / sqrt(k)
    assert errs[1] < errs[0] / 3.0 and errs[1] < 0.05


def test_probe_solve_reaches_the_tensor_newton_minimiser():
    from test_oracle_stall import _tensor_newton
    R = synth.workload_returns("n12_T500")
    c = np.array(synth.WORKLOADS["n12_T500"]["c"])
    mu, A = O.center(R)
    o = O.Options.large()
    o.trace, o.probes, o.probe_seed = "probe", 32, 5
    x, info = O.solve(R, c, opts=o)
    assert info.status == 0 and info.gnorm <= 1e-8
    assert info.directions == info.iterations and info.probe_iters > 0
    C, b = O.constraints(mu)
    U = O.tangent_basis(C)
    xn = _tensor_newton(A, mu, c, U, O.feasible_start(C, b))
    Hr = U.T @ (A.T @ (O.d2psi(c, A @ xn)[:, None] * A) / A.shape[0]) @ U
    assert np.linalg.norm(x - xn) <= 2e-8 / np.linalg.eigvalsh(Hr)[0] + 1e-12


def test_pcg_stops_at_nonpositive_curvature():
    """Truncated CG: the first search direction with p^T B p <= 0 ends the
    iteration without a step along it."""
    Bm = np.diag([2.0, -1.0])
    u, it = M._pcg(Bm, np.array([0.0, 1.0]), 1e-12, 10, lambda r: r)
    assert it == 1 and np.array_equal(u, np.zeros(2))
    u, it = M._pcg(np.diag([2.0, 1.0]), np.array([1.0, 1.0]), 1e-14, 10,
                   lambda r: r)
    assert np.allclose(u, [0.5, 1.0]) and it == 2
