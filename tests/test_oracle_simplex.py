"""Pins of the oracle's simplex boundary block: the projection onto
Delta(tau), the projected-KKT residual, the face rule and the solve loop.

Independent references: exhaustive search over supports for the projection,
the optimality conditions of the projection, a linear objective whose
minimiser over the simplex is a known vertex, and scipy's SLSQP minimiser of
the same objective over the simplex.
"""

import itertools
import math

import numpy as np
import pytest

import oracle as O
import synth


def _brute_project(y, tau):
    """min |x - y| over Delta(tau) by trying every support: on a support S
    the free coordinates are y_S - theta_S with theta_S fixed by the budget;
    keep the feasible candidate nearest to y."""
    n = y.size
    best, bd = None, math.inf
    for k in range(1, n + 1):
        for S in itertools.combinations(range(n), k):
            S = list(S)
            x = np.full(n, tau)
            theta = (y[S].sum() - (1.0 - (n - k) * tau)) / k
            x[S] = y[S] - theta
            if np.all(x >= tau - 1e-15):
                dist = float(np.sum((x - y) ** 2))
                if dist < bd:
                    best, bd = x, dist
    return best


@pytest.mark.parametrize("n", [1, 2, 3, 5, 6])
@pytest.mark.parametrize("tau", [0.0, 1e-3])
def test_projection_matches_exhaustive_search(n, tau):
    rng = np.random.default_rng(10 * n + int(tau > 0))
    for scale in (0.1, 1.0, 10.0):
        y = scale * rng.standard_normal(n)
        assert np.abs(O.project_simplex(y, tau) - _brute_project(y, tau)).max() <= 1e-13 * max(1.0, scale)


@pytest.mark.parametrize("n", [7, 64, 1000, 5440])
def test_projection_optimality_conditions(n):
    """x = Pi(y) iff x in Delta(tau) and y - x = theta 1 - lambda with
    lambda >= 0 vanishing off the bound (y - x constant on free coordinates,
    not larger on bound ones)."""
    rng = np.random.default_rng(n)
    tau = 1e-8
    for y in (rng.standard_normal(n) / n, rng.standard_normal(n), np.full(n, 3.0)):
        x = O.project_simplex(y, tau)
        assert x.min() >= tau * (1 - 1e-12)
        # x_i = y_i - theta loses an ulp of |y| per coordinate
        ulp_y = np.finfo(float).eps * max(1.0, np.abs(y).max())
        assert abs(x.sum() - 1.0) <= 4 * n * ulp_y
        r = y - x
        free = x > tau * (1 + 1e-9)
        theta = r[free].mean()
        assert np.abs(r[free] - theta).max() <= 1e-12 * max(1.0, np.abs(y).max())
        assert np.all(r[~free] <= theta + 1e-12 * max(1.0, np.abs(y).max()))


def test_projection_fixed_points_and_invariances():
    rng = np.random.default_rng(3)
    n, tau = 9, 1e-8
    x = rng.random(n) + 0.1
    x /= x.sum()
    assert np.abs(O.project_simplex(x, tau) - x).max() <= 1e-15
    y = rng.standard_normal(n)
    p = O.project_simplex(y, tau)
    assert np.abs(O.project_simplex(y + 7.25, tau) - p).max() <= 1e-14
    perm = rng.permutation(n)
    assert np.abs(O.project_simplex(y[perm], tau) - p[perm]).max() <= 1e-15


def test_kkt_residual_linear_objective_vertex():
    """c = (c1, 0, 0, 0): f = -c1 mu^T x is minimised over the simplex at the
    vertex of the largest mean, where the residual vanishes; it is positive
    at every other vertex."""
    R = synth.workload_returns("n12_T500")
    mu, A = O.center(R)
    c = np.array([2.0, 0.0, 0.0, 0.0])
    order = np.argsort(mu)[::-1]
    k, j, third = int(order[0]), int(order[1]), int(order[2])
    assert O.kkt_residual(A, mu, c, np.eye(mu.size)[k]) <= 1e-15
    for i in range(mu.size):
        if i != k:
            assert O.kkt_residual(A, mu, c, np.eye(mu.size)[i]) > 0.0
    # at the second vertex the projection of e_j + c1 mu splits the unit
    # mass between j and k (theta = c1 (mu_j + mu_k) / 2 lies above the
    # third mean), so the residual is c1 (mu_k - mu_j) / sqrt(2)
    assert mu[third] < 0.5 * (mu[j] + mu[k])
    assert O.kkt_residual(A, mu, c, np.eye(mu.size)[j]) == pytest.approx(
        c[0] * (mu[k] - mu[j]) / math.sqrt(2.0), rel=1e-9)


def test_kkt_residual_equals_tangent_gradient_inside():
    """At an interior point whose unit projected-gradient step stays inside,
    the residual is |P_1 grad f| (the budget tangent gradient)."""
    R = synth.workload_returns("n12_T500")
    mu, A = O.center(R)
    c = np.array([1e-4, 1e-3, 1e-3, 1e-3])
    x = np.full(mu.size, 1.0 / mu.size)
    g = O.gradient(A, mu, c, x)
    assert np.abs(g - g.mean()).max() < 0.5 / mu.size
    assert O.kkt_residual(A, mu, c, x) == pytest.approx(np.linalg.norm(g - g.mean()), rel=1e-12)


def test_face_rule_and_basis():
    tau = 1e-8
    x = np.array([0.5, tau, 0.3, tau, 0.2])
    g = np.array([1.0, 0.0, 1.0, 5.0, 1.0])  # multiplier of coordinate 1 is -1
    free = O.face_free(x, g, tau)
    assert free.tolist() == [True, True, True, False, True]
    U = O.face_basis(free)
    assert U.shape == (5, 3)
    assert np.abs(U.T @ U - np.eye(3)).max() <= 1e-15
    assert np.abs(U[3]).max() == 0.0 and np.abs(U.sum(axis=0)).max() <= 1e-15
    assert O.face_basis(np.array([False, True, False])).shape == (3, 0)


def _slsqp(A, mu, c):
    from scipy.optimize import minimize
    n = mu.size
    res = minimize(lambda x: O.objective(A, mu, c, x), np.full(n, 1.0 / n),
                   jac=lambda x: O.gradient(A, mu, c, x), method="SLSQP",
                   bounds=[(0.0, 1.0)] * n,
                   constraints=[{"type": "eq", "fun": lambda x: x.sum() - 1.0,
                                 "jac": lambda x: np.ones(n)}],
                   options={"ftol": 1e-16, "maxiter": 2000})
    return res.x, res.fun


@pytest.mark.parametrize("c", [(1.0, 1.0, 1.0, 1.0), (1.0, 10.0, 1.0, 10.0), (10.0, 1.0, 10.0, 1.0)])
def test_boundary_block_reaches_the_simplex_minimiser(c):
    """The boundary block (projected trial step, face continuation) ends at
    SLSQP's minimiser over the simplex, up to the tau offsets of the bound
    coordinates; every iterate stays in Delta(tau) and f never increases."""
    R = synth.workload_returns("n12_T500")
    mu, A = O.center(R)
    c = np.array(c)
    x, info = O.solve(R, c, opts=O.Options(feasible_set="simplex", max_iter=300))
    xs, fs = _slsqp(A, mu, c)
    assert info.status == 0
    assert x.min() >= 1e-8 * (1 - 1e-9) and abs(x.sum() - 1.0) <= 1e-13
    # the bound coordinates sit at tau = 1e-8, not 0: that costs at most
    # n tau |grad f|_inf against the minimiser over the closed simplex
    g = O.gradient(A, mu, c, x)
    assert info.f <= fs + 2.0 * mu.size * 1e-8 * np.abs(g).max() + 1e-12 * abs(fs)
    assert np.abs(x - xs).max() <= 1e-5
    fh = [h[2] for h in info.history]
    assert all(b <= a + 1e-15 * abs(a) for a, b in zip(fh, fh[1:]))
    assert info.kkt <= 1e-6


def test_eta_zero_keeps_capped_steps():
    R = synth.workload_returns("n12_T500")
    x, info = O.solve(R, [1.0, 1.0, 1.0, 1.0],
                      opts=O.Options(feasible_set="simplex", eta=0.0, max_iter=50))
    # the cap-only run ends at the stall test (three steps without decrease)
    assert info.projected_steps == 0 and info.status == 2
    assert info.phases[0][5] == "stall"


def test_armijo_step_conditions():
    """The accepted step satisfies the sufficient-decrease condition on the
    quartic, and the step twice as long (when tried) did not."""
    rng = np.random.default_rng(11)
    for _ in range(200):
        A = rng.standard_normal(5)
        A[1] = -abs(A[1]) - 1e-3          # descent
        A[4] = abs(A[4])
        amax = rng.choice([math.inf, 0.3, 2.0])
        a = O.armijo_step(A, amax)
        phi = lambda t: A[1] * t + A[2] * t**2 + A[3] * t**3 + A[4] * t**4
        assert 0.0 < a <= min(1.0, amax)
        assert phi(a) <= 1e-4 * a * A[1] + 1e-15
        if a < min(1.0, amax):
            assert phi(2 * a) > 1e-4 * 2 * a * A[1]


def test_armijo_solves_reach_the_exact_rule_minimiser():
    """Budget set, certified-convex CRRA: Armijo and exact steps end within
    the stopping tolerance of the same unique minimiser, |x - x*| <=
    |gbar| / lambda_min of the reduced Hessian for both runs; on n12_T500
    simplex both end on the same two-asset face."""
    R = synth.workload_returns("n400_T4800")
    mu, A = O.center(R)
    c = synth.crra_coefficients(6.0)
    xe, ie = O.solve(R, c)
    xa, ia = O.solve(R, c, opts=O.Options(linesearch="armijo"))
    assert ie.status == 0 and ia.status == 0
    U = O.tangent_basis(np.ones((mu.size, 1)))
    H = U.T @ (A.T @ (O.d2psi(c, A @ xe)[:, None] * A) / A.shape[0]) @ U
    lam = float(np.linalg.eigvalsh(H)[0])
    assert np.linalg.norm(xa - xe) <= 1.1 * (ie.gnorm + ia.gnorm) / lam
    R = synth.workload_returns("n12_T500")
    xe, ie = O.solve(R, [1.0, 1.0, 1.0, 1.0], opts=O.Options(feasible_set="simplex"))
    xa, ia = O.solve(R, [1.0, 1.0, 1.0, 1.0],
                     opts=O.Options(feasible_set="simplex", linesearch="armijo"))
    assert ia.status == 0
    assert np.array_equal(xa > 1e-6, xe > 1e-6)


def test_kkt_on_the_slice_and_the_floor_against_delta0():
    """At the boundary block's solution on n12_T500 (two free coordinates,
    ten on the bound tau), the residual on the slice vanishes to the
    stopping tolerance, while against Delta(0) it keeps the floor
    tau sqrt(n_b^2 / n_free + n_b): the bound coordinates drop to 0 and
    their mass n_b tau spreads over the free ones."""
    R = synth.workload_returns("n12_T500")
    mu, A = O.center(R)
    c = np.array([1.0, 1.0, 1.0, 1.0])
    x, info = O.solve(R, c, opts=O.Options(feasible_set="simplex"))
    tau = 1e-8
    nb = int(np.count_nonzero(x <= tau * (1 + 1e-6)))
    assert nb == 10
    assert O.kkt_residual(A, mu, c, x, tau) <= 1e-8
    assert info.kkt == pytest.approx(O.kkt_residual(A, mu, c, x, tau), rel=1e-12, abs=1e-20)
    floor = tau * math.sqrt(nb * nb / 2.0 + nb)
    assert O.kkt_residual(A, mu, c, x, 0.0) == pytest.approx(floor, rel=1e-3)


def test_face_solver_takes_over_when_no_segment_descends():
    # A crash-skewed panel where the direction on the released face drives a
    # bound coordinate further down and the projected segment is no descent
    # direction either: without handing those coordinates to the face solver
    # the run stalls at zero steps with f = 10.92 and a KKT residual near 1.
    # With the hand-off it must reach the simplex KKT point.
    R = synth.priced_factor_returns(60, 600, 3, 5.0, 3)
    mu, A = O.center(R)
    n = R.shape[1]
    m = O.moments(A, mu, np.full(n, 1.0 / n))
    c = np.array([4434.270595, 1.0 / m[1], 1.0 / abs(m[2]), 10.0 / m[3]])
    x, info = O.solve(R, c, opts=O.Options(feasible_set="simplex"))
    assert info.status == 0
    assert O.kkt_residual(A, mu, c, x, 1e-8) <= 1e-8
    assert O.objective(A, mu, c, x) < 10.0
    # KKT on Delta(tau) read off directly: one multiplier on the support,
    # nothing below it on the bound coordinates
    g = O.gradient(A, mu, c, x)
    sup = x > 1e-8 * (1.0 + 1e-6)
    nu = g[sup].mean()
    assert np.max(np.abs(g[sup] - nu)) <= 1e-7 * np.max(np.abs(g))
    assert np.all(g[~sup] >= nu - 1e-7 * np.max(np.abs(g)))


@pytest.mark.parametrize("n", [60, 1000])
def test_short_projected_segments_hand_off_to_the_face_solver(n):
    # The paper's T = 252 stress generator with the certified profile
    # [1, 10, 1, 10]: taking every descent segment, however short its step,
    # crept to a stall at KKT 1e-3 (n = 60) and 7e-3 (n = 1000).  With the
    # usable-step rule the run must reach the simplex KKT point, checked
    # here from the gradient directly.
    R = synth.uniform_returns(n, 252, seed=n)
    mu, A = O.center(R)
    c = np.array([1.0, 10.0, 1.0, 10.0])
    x, info = O.solve(R, c, opts=O.Options(feasible_set="simplex"))
    assert info.status == 0
    g = O.gradient(A, mu, c, x)
    sup = x > 1e-8 * (1.0 + 1e-6)
    nu = g[sup].mean()
    scale = np.max(np.abs(g))
    assert np.max(np.abs(g[sup] - nu)) <= 1e-8 * scale
    assert np.all(g[~sup] >= nu - 1e-8 * scale)
    # a step capped at alpha_max lands on the bound up to rounding
    assert abs(x.sum() - 1.0) <= 1e-12 and x.min() >= 1e-8 * (1 - 1e-9)
