"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these tests re-types the oracle's formulas: each compares it with a
different route to the same quantity (explicit comoment tensors, complex-step
derivatives, polynomial fits, brute-force scans, the centroid definition of
the affine normal, the closed-form mean-variance portfolio, printed values).
"""

import math

import numpy as np
import pytest

import oracle as O
import synth

C_CONVEX = np.array([1.0, 10.0, 1.0, 10.0])   # [1,10,1,10] profile, Section 6.1
C_NONCVX = np.array([10.0, 1.0, 10.0, 1.0])


def small_instance(n=5, T=40, seed=3):
    R = synth.uniform_returns(n, T, seed)
    mu, A = O.center(R)
    return R, mu, A


def tensors(A):
    """Explicit comoment tensors Sigma, S, K of Section 2 (n <= 8 only)."""
    T = A.shape[0]
    Sig = np.einsum("ti,tj->ij", A, A) / T
    S = np.einsum("ti,tj,tk->ijk", A, A, A) / T
    K = np.einsum("ti,tj,tk,tl->ijkl", A, A, A, A) / T
    return Sig, S, K


# --------------------------------------------------------------- centering --

def test_center_column_means_fsum():
    R = synth.uniform_returns(6, 33, 0)
    mu, A = O.center(R)
    for j in range(6):
        assert mu[j] == pytest.approx(math.fsum(R[:, j]) / 33, rel=1e-15)
        # 1^T A = 0 (Remark on the curvature decomposition: rank A <= T-1)
        assert abs(math.fsum(A[:, j])) < 4 * 33 * abs(mu[j]) * 2**-53


def test_moments_match_definition():
    """m_p(x) = T^-1 sum (r_t^T x - mu^T x)^p, computed with fsum from R."""
    R, mu, A = small_instance(4, 25, 1)
    x = np.array([0.1, 0.2, 0.3, 0.4])
    T = R.shape[0]
    m1 = math.fsum(math.fsum(R[:, j]) / T * x[j] for j in range(4))
    rx = [math.fsum(R[t, j] * x[j] for j in range(4)) for t in range(T)]
    ref = [m1] + [math.fsum((v - m1) ** p for v in rx) / T for p in (2, 3, 4)]
    got = O.moments(A, mu, x)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-18)
    c = np.array([1.3, 2.0, 0.7, 5.0])
    f_ref = -c[0] * ref[0] + c[1] * ref[1] - c[2] * ref[2] + c[3] * ref[3]
    assert O.objective(A, mu, c, x) == pytest.approx(f_ref, rel=1e-12)


# ------------------------------------------- tensor route (Section 2, n<=8) --

@pytest.mark.parametrize("c", [C_CONVEX, C_NONCVX, np.array([1, 1, 1, 1.])])
def test_oracle_matches_tensor_route(c):
    R, mu, A = small_instance(5, 40, 4)
    Sig, S, K = tensors(A)
    rng = np.random.default_rng(0)
    x = rng.dirichlet(np.ones(5))
    u, v = rng.normal(size=5), rng.normal(size=5)
    f_t = (-c[0] * mu @ x + c[1] * x @ Sig @ x
           - c[2] * np.einsum("ijk,i,j,k->", S, x, x, x)
           + c[3] * np.einsum("ijkl,i,j,k,l->", K, x, x, x, x))
    g_t = (-c[0] * mu + 2 * c[1] * Sig @ x
           - 3 * c[2] * np.einsum("ijk,i,j->k", S, x, x)
           + 4 * c[3] * np.einsum("ijkl,i,j,k->l", K, x, x, x))
    H_t = (2 * c[1] * Sig - 6 * c[2] * np.einsum("ijk,i->jk", S, x)
           + 12 * c[3] * np.einsum("ijkl,i,j->kl", K, x, x))
    T3_t = (-6 * c[2] * S + 24 * c[3] * np.einsum("ijkl,i->jkl", K, x))
    assert O.objective(A, mu, c, x) == pytest.approx(f_t, rel=1e-12)
    np.testing.assert_allclose(O.gradient(A, mu, c, x), g_t, rtol=1e-11,
                               atol=1e-15)
    np.testing.assert_allclose(O.hvp(A, c, x, v), H_t @ v, rtol=1e-11,
                               atol=1e-14)
    np.testing.assert_allclose(O.third(A, c, x, u, v),
                               np.einsum("ijk,i,j->k", T3_t, u, v),
                               rtol=1e-10, atol=1e-13)


# ------------------------------------------------- complex-step derivatives --

def test_gradient_hvp_third_by_complex_step():
    """f is a polynomial, so complex-step derivatives are exact to rounding."""
    R, mu, A = small_instance(7, 60, 5)
    c = np.array([0.8, 3.0, 4.0, 6.0])
    rng = np.random.default_rng(1)
    x = rng.dirichlet(np.ones(7))
    u, v = rng.normal(size=7), rng.normal(size=7)
    h = 1e-30
    g_cs = np.array([O.objective(A, mu, c, x + 1j * h * e).imag / h
                     for e in np.eye(7)])
    np.testing.assert_allclose(O.gradient(A, mu, c, x), g_cs, rtol=1e-13,
                               atol=1e-16)
    hv_cs = O.gradient(A, mu, c, x + 1j * h * v).imag / h
    np.testing.assert_allclose(O.hvp(A, c, x, v), hv_cs, rtol=1e-13,
                               atol=1e-15)
    t_cs = O.hvp(A, c, x + 1j * h * u, v).imag / h
    np.testing.assert_allclose(O.third(A, c, x, u, v), t_cs, rtol=1e-12,
                               atol=1e-14)


# ------------------------------------------------- quartic line search -----

def test_linesearch_coeffs_fit_quartic():
    """A0..A4 equal the quartic through f(x + alpha_i d) at 5 distinct steps."""
    R, mu, A = small_instance(6, 50, 6)
    c = np.array([1.0, 2.0, 3.0, 4.0])
    rng = np.random.default_rng(2)
    x = rng.dirichlet(np.ones(6))
    d = rng.normal(size=6)
    d -= d.mean()
    al = np.array([-1.0, -0.5, 0.0, 0.5, 1.0])
    V = np.vander(al, 5, increasing=True)
    vals = [O.objective(A, mu, c, x + a * d) for a in al]
    fit = np.linalg.solve(V, vals)
    coef = O.linesearch_coeffs(A, mu, c, x, d)
    np.testing.assert_allclose(coef, fit, rtol=1e-9, atol=1e-14)
    assert coef[0] == pytest.approx(O.objective(A, mu, c, x), rel=1e-15)
    assert coef[1] == pytest.approx(O.gradient(A, mu, c, x) @ d, rel=1e-12)


def _golden_min(coef, lo, hi, grid=200001):
    al = np.linspace(lo, hi, grid)
    vals = O.quartic_value(coef, al)
    i = int(np.argmin(vals))
    a, b = al[max(i - 1, 0)], al[min(i + 1, grid - 1)]
    gr = (math.sqrt(5) - 1) / 2
    for _ in range(200):
        c1, c2 = b - gr * (b - a), a + gr * (b - a)
        if O.quartic_value(coef, c1) < O.quartic_value(coef, c2):
            b = c2
        else:
            a = c1
    return 0.5 * (a + b), vals.min()


@pytest.mark.parametrize("seed", range(6))
def test_select_step_brute_force(seed):
    rng = np.random.default_rng(seed)
    coef = rng.normal(size=5)
    coef[1] = -abs(coef[1])           # descent direction: A1 < 0
    coef[4] = abs(coef[4]) + 0.1
    amax = float(rng.uniform(0.5, 3.0)) if seed % 2 else math.inf
    hi = amax if math.isfinite(amax) else 20.0
    a_star = O.select_step(coef, amax)
    a_ref, vmin = _golden_min(coef, 0.0, hi)
    assert O.quartic_value(coef, a_star) <= vmin + 1e-12
    if not (math.isfinite(amax) and abs(a_ref - amax) < 1e-6):
        assert a_star == pytest.approx(a_ref, abs=1e-6)


def test_select_step_unbounded():
    with pytest.raises(O.Unbounded):
        O.select_step([0.0, -1.0, 0.5, -0.2, 0.0])     # c4 = 0, c3 > 0 line
    # c3 = c4 = 0 with positive curvature: the quadratic minimiser
    assert O.select_step([0.0, -1.0, 0.5, 0.0, 0.0]) == pytest.approx(1.0)


def test_alpha_max_property():
    rng = np.random.default_rng(3)
    x = rng.dirichlet(np.ones(9))
    d = rng.normal(size=9)
    d -= d.mean()
    tau = 1e-8
    am = O.alpha_max(x, d, tau)
    y = x + am * d
    assert y.min() == pytest.approx(tau, abs=1e-14)
    assert abs(y.sum() - 1.0) < 1e-14
    for a in np.linspace(0, am, 7):
        assert (x + a * d).min() >= tau - 1e-15


# --------------------------------------------------------- reduced frames --

def test_bases():
    mu = np.random.default_rng(4).normal(size=8)
    for target in (None, 0.3):
        C, b = O.constraints(mu, target)
        U = O.tangent_basis(C)
        np.testing.assert_allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-14)
        np.testing.assert_allclose(C.T @ U, 0, atol=1e-14)
        P = np.eye(8) - C @ np.linalg.solve(C.T @ C, C.T)
        np.testing.assert_allclose(U @ U.T, P, atol=1e-14)
        x0 = O.feasible_start(C, b)
        np.testing.assert_allclose(C.T @ x0, b, atol=1e-15)
    nu = np.random.default_rng(5).normal(size=6)
    nu /= np.linalg.norm(nu)
    Q = O.householder_frame(nu)
    np.testing.assert_allclose(Q.T @ Q, np.eye(5), atol=1e-14)
    np.testing.assert_allclose(Q.T @ nu, 0, atol=1e-15)


# ------------------------------------------------ affine-normal direction --

def _delta_f(A, mu, c, x0, v):
    """f(x0 + v) - f(x0) by the Taylor expansion in w = A v (no cancellation)."""
    T = A.shape[0]
    z = A @ x0
    w = A @ v
    p1 = 2 * c[1] * z - 3 * c[2] * z**2 + 4 * c[3] * z**3
    p2 = 2 * c[1] - 6 * c[2] * z + 12 * c[3] * z**2
    p3 = -6 * c[2] + 24 * c[3] * z
    dpsi = p1 * w + p2 * w**2 / 2 + p3 * w**3 / 6 + c[3] * w**4
    return np.sum(dpsi) / T - c[0] * (mu @ v)


def _ray_root(A, mu, c, x0, v0, e):
    """Smallest positive r with f(x0 + v0 + r e) = f(x0) (exact quartic)."""
    rs = np.array([-2.0, -1.0, 0.0, 1.0, 2.0]) * 50 * np.linalg.norm(v0)
    p = np.polyfit(rs, [_delta_f(A, mu, c, x0, v0 + r * e) for r in rs], 4)
    rt = np.roots(p)
    rt = rt[np.abs(rt.imag) < 1e-9 * np.abs(rt)].real
    return rt[rt > 0].min()


def _centroid_normal(A, mu, c, x0, C, eps, N=96):
    """Affine normal as the limit of section centroids (Blaschke's
    characterisation): cut the sublevel set at depth eps below the tangent
    plane and join x0 to the centroid of the section."""
    g = O.gradient(A, mu, c, x0)
    P0 = np.eye(len(x0)) - C @ np.linalg.solve(C.T @ C, C.T)
    nu = P0 @ g
    nu /= np.linalg.norm(nu)
    E = np.column_stack([C, nu])
    Qc, _ = np.linalg.qr(E, mode="complete")
    Tb = Qc[:, E.shape[1]:]
    v0 = -eps * nu
    if Tb.shape[1] == 1:
        e = Tb[:, 0]
        off = 0.5 * (_ray_root(A, mu, c, x0, v0, e)
                     - _ray_root(A, mu, c, x0, v0, -e)) * e
    else:
        num = np.zeros(len(x0))
        den = 0.0
        for th in 2 * np.pi * np.arange(N) / N:
            e = np.cos(th) * Tb[:, 0] + np.sin(th) * Tb[:, 1]
            r = _ray_root(A, mu, c, x0, v0, e)
            num += r**3 / 3 * e
            den += r**2 / 2
        off = num / den
    return -nu + off / eps


@pytest.mark.parametrize("with_target", [False, True])
def test_direction_is_centroid_affine_normal(with_target):
    """m = 3 (budget, n = 4) and m = 2 (budget + target, n = 4).  With the
    target, m + 1 = 3 differs from n = 4, so the factor 1/(m+1) of Appendix B
    is checked against the 1/n of Section 4.2."""
    R = synth.uniform_returns(4, 252, 7)
    mu, A = O.center(R)
    target = float(mu.mean() + 0.3 * (mu.max() - mu.mean())) if with_target else None
    C, b = O.constraints(mu, target)
    U = O.tangent_basis(C)
    x0 = O.feasible_start(C, b)
    dr = O.affine_normal(A, mu, C_CONVEX, x0, U)
    e1 = _centroid_normal(A, mu, C_CONVEX, x0, C, 5e-4 * dr.gnorm / 0.1)
    e2 = _centroid_normal(A, mu, C_CONVEX, x0, C, 2.5e-4 * dr.gnorm / 0.1)
    rich = 2 * e2 - e1                                   # Richardson, O(eps)
    np.testing.assert_allclose(dr.d, rich, atol=1e-8)
    assert np.abs(e2 - dr.d).max() > 1e-8                # the limit is needed


def test_direction_invariants_and_basis_invariance():
    R, mu, A = small_instance(7, 80, 8)
    c = C_CONVEX
    for target in (None, float(mu.mean())):
        C, b = O.constraints(mu, target)
        U = O.tangent_basis(C)
        x0 = O.feasible_start(C, b)
        dr = O.affine_normal(A, mu, c, x0, U)
        g = O.gradient(A, mu, c, x0)
        assert g @ dr.d == pytest.approx(-dr.gnorm, rel=1e-12)   # g^T d = -|G|
        np.testing.assert_allclose(C.T @ dr.d, 0, atol=1e-14)
        Rm, _ = np.linalg.qr(np.random.default_rng(9).normal(size=(U.shape[1],) * 2))
        dr2 = O.affine_normal(A, mu, c, x0, U @ Rm)
        np.testing.assert_allclose(dr2.d, dr.d, rtol=1e-10, atol=1e-13)


def test_trace_matches_tensor_contraction():
    """a_l = sum_ij (H_T^-1)_ij D^3 phi[Q e_i, Q e_j, Q e_l] with explicit S, K."""
    R, mu, A = small_instance(6, 70, 10)
    c = np.array([1.0, 4.0, 3.0, 8.0])
    _, S, K = tensors(A)
    C, b = O.constraints(mu)
    U = O.tangent_basis(C)
    x = O.feasible_start(C, b) + U @ np.random.default_rng(1).normal(size=5) * 0.05
    dr = O.affine_normal(A, mu, c, x, U)
    g = O.gradient(A, mu, c, x)
    nu = U.T @ g / dr.gnorm
    V = U @ O.householder_frame(nu)
    H = (2 * c[1] * np.einsum("ti,tj->ij", A, A) / A.shape[0]
         - 6 * c[2] * np.einsum("ijk,i->jk", S, x)
         + 12 * c[3] * np.einsum("ijkl,i,j->kl", K, x, x))
    D3 = -6 * c[2] * S + 24 * c[3] * np.einsum("ijkl,i->jkl", K, x)
    Binv = np.linalg.inv(V.T @ H @ V)
    a_ref = np.einsum("ij,abc,ai,bj,cl->l", Binv, D3, V, V, V)
    np.testing.assert_allclose(dr.a, a_ref, rtol=1e-9, atol=1e-12)


def test_trace_is_logdet_derivative():
    """a = d/d eta log det(Q^T H_red(y + Q eta) Q) at eta = 0 (central FD)."""
    R, mu, A = small_instance(6, 70, 11)
    c = np.array([1.0, 4.0, 3.0, 8.0])
    C, b = O.constraints(mu)
    U = O.tangent_basis(C)
    x = O.feasible_start(C, b)
    dr = O.affine_normal(A, mu, c, x, U)
    nu = U.T @ O.gradient(A, mu, c, x) / dr.gnorm
    V = U @ O.householder_frame(nu)
    T = A.shape[0]

    def logdet(xx):
        z = A @ xx
        Hm = V.T @ (A.T @ (O.d2psi(c, z)[:, None] * A)) @ V / T
        return np.linalg.slogdet(Hm)[1]

    h = 1e-5
    fd = np.array([(logdet(x + h * V[:, l]) - logdet(x - h * V[:, l])) / (2 * h)
                   for l in range(V.shape[1])])
    np.testing.assert_allclose(dr.a, fd, rtol=1e-6, atol=1e-8)


# --------------------------------------- closed-form mean-variance optimum --

def _mv_optimum(A, mu, c, target=None):
    """Merton (1972): minimiser of -c1 mu^T x + c2 x^T Sigma x on C^T x = b."""
    T, n = A.shape
    Sig = A.T @ A / T
    one = np.ones(n)
    if target is None:
        si1, sim = np.linalg.solve(Sig, one), np.linalg.solve(Sig, mu)
        eta = (c[0] * one @ sim - 2 * c[1]) / (one @ si1)
        return (c[0] * sim - eta * si1) / (2 * c[1])
    Cm = np.stack([one, mu], 1)
    SiC = np.linalg.solve(Sig, Cm)
    return SiC @ np.linalg.solve(Cm.T @ SiC, np.array([1.0, target]))


@pytest.mark.parametrize("with_target", [False, True])
def test_quadric_case_one_step_to_mv_optimum(with_target):
    R = synth.workload_returns("n12_T500")
    mu, A = O.center(R)
    c = np.array([1.0, 5.0, 0.0, 0.0])
    target = float(np.median(mu)) if with_target else None
    C, b = O.constraints(mu, target)
    U = O.tangent_basis(C)
    x0 = O.feasible_start(C, b)
    dr = O.affine_normal(A, mu, c, x0, U)
    alpha = O.select_step(O.linesearch_coeffs(A, mu, c, x0, dr.d))
    xs = _mv_optimum(A, mu, c, target)
    np.testing.assert_allclose(x0 + alpha * dr.d, xs, rtol=1e-9, atol=1e-10)


# ----------------------------------------------------------- whole solves --

def _tensor_newton(A, mu, c, U, x):
    """Independent minimiser: Newton on the reduced tensor-form objective."""
    Sig, S, K = tensors(A)
    for _ in range(60):
        g = (-c[0] * mu + 2 * c[1] * Sig @ x - 3 * c[2] * np.einsum("ijk,i,j->k", S, x, x)
             + 4 * c[3] * np.einsum("ijkl,i,j,k->l", K, x, x, x))
        H = (2 * c[1] * Sig - 6 * c[2] * np.einsum("ijk,i->jk", S, x)
             + 12 * c[3] * np.einsum("ijkl,i,j->kl", K, x, x))
        step = U @ np.linalg.solve(U.T @ H @ U, U.T @ g)
        x = x - step
        if np.linalg.norm(step) < 1e-15:
            break
    return x


@pytest.mark.parametrize("solver", ["direct", "pcg"])
def test_solve_matches_tensor_newton(solver):
    R = synth.factor_returns(6, 300, 2, 0, 5.0, 0.0, 21)
    mu, A = O.center(R)
    c = np.array([1.0, 1.0, 1.0, 1.0])
    opts = O.Options.large() if solver == "pcg" else O.Options()
    opts.eps = 1e-13
    x, info = O.solve(R, c, opts=opts)
    assert info.status == 0 and info.gnorm <= opts.eps
    C, b = O.constraints(mu)
    U = O.tangent_basis(C)
    xn = _tensor_newton(A, mu, c, U, O.feasible_start(C, b))
    # strong convexity on the tangent space: |x - x*| <= |gbar| / lambda_min
    Hr = U.T @ (A.T @ (O.d2psi(c, A @ xn)[:, None] * A) / A.shape[0]) @ U
    lmin = np.linalg.eigvalsh(Hr)[0]
    assert np.linalg.norm(x - xn) <= 2 * opts.eps / lmin + 1e-12
    assert abs(x.sum() - 1.0) < 1e-12


def test_solve_workload_n12_budget_and_target():
    R = synth.workload_returns("n12_T500")
    c = np.array(synth.WORKLOADS["n12_T500"]["c"])
    x, info = O.solve(R, c)
    assert info.status == 0 and info.gnorm <= 1e-8
    assert abs(x.sum() - 1.0) < 1e-12
    mu, _ = O.center(R)
    r = float(np.quantile(mu, 0.7))
    xt, it = O.solve(R, c, target=r)
    assert it.status == 0 and it.gnorm <= 1e-8
    assert abs(mu @ xt - r) < 1e-12 and abs(xt.sum() - 1) < 1e-12


def test_simplex_mode_stays_in_slice():
    R = synth.uniform_returns(8, 252, 2)
    c = np.array([1.0, 10.0, 1.0, 10.0])
    x, info = O.solve(R, c, opts=O.Options(feasible_set="simplex", max_iter=50))
    assert x.min() >= 1e-8 - 1e-15 and abs(x.sum() - 1) < 1e-12


# ------------------------------------------------------ printed values -----

def test_crra_golden(golden_dir):
    rows = np.loadtxt(f"{golden_dir}/crra_calibration.txt")
    rows = np.atleast_2d(rows)
    for g, *cv in rows:
        np.testing.assert_allclose(synth.crra_coefficients(g), cv, rtol=1e-15)
        assert 8 * cv[1] * cv[3] - 3 * cv[2] ** 2 == pytest.approx(
            g**2 * (g + 1) * (g + 3) / 12)
        assert O.certified_convex(cv)
    assert not O.certified_convex(C_NONCVX)


def test_reduced_hessian_table(golden_dir):
    """Distribution-level match of Table 'Supporting reduced-Hessian
    conditioning diagnostic' (medians; the paper has three draws per n)."""
    tab = np.loadtxt(f"{golden_dir}/hessian_conditioning_T252.txt")
    profiles = [np.array(p, float) for p in ([10, 1, 10, 1], [1, 10, 1, 10],
                                             [10, 10, 10, 10])]
    for n, lmin, lmax, kap in tab[[0, 2, 5]]:
        n = int(n)
        vals = []
        for seed in range(5):
            R = synth.uniform_returns(n, 252, 100 + seed)
            mu, A = O.center(R)
            C, b = O.constraints(mu)
            U = O.tangent_basis(C)
            z = A @ O.feasible_start(C, b)
            for c in profiles:
                Hr = U.T @ (A.T @ (O.d2psi(c, z)[:, None] * A) / 252) @ U
                ev = np.linalg.eigvalsh(Hr)
                vals.append((ev[0], ev[-1], ev[-1] / ev[0]))
        med = np.median(np.array(vals), axis=0)
        assert med[0] == pytest.approx(lmin, rel=0.2)
        assert med[1] == pytest.approx(lmax, rel=0.1)
        assert med[2] == pytest.approx(kap, rel=0.25)
