"""GPU parity of the simplex boundary block: the projection onto Delta(tau),
the projected-KKT residual, and solves whose iterates use face continuation
and projected trial steps, all through the C-ABI against the FP64 oracle.

Tolerances: the projection's threshold comes from a block sum instead of a
correctly rounded one, so outputs agree to a few ulps of max|y| per
coordinate (bound 1e-13 max(1, |y|_inf)); the KKT residual is a norm of
such differences plus the gradient's rounding (relative 1e-9); iterates of
a solve agree to 1e-9 like the other solve-level parity tests.
"""

import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2604_25378_amd import binding as yb  # noqa: E402


@pytest.mark.parametrize("n", [1, 2, 13, 1000, 1024, 1025, 5440])
@pytest.mark.parametrize("tau", [0.0, 1e-8, 1e-4])
def test_projection_matches_oracle(n, tau):
    if tau * n >= 1.0:
        pytest.skip("tau >= 1/n")
    print(f"[case] projection n={n} tau={tau}", flush=True)
    rng = np.random.default_rng(n + int(1e9 * tau))
    for y in (rng.standard_normal(n), rng.standard_normal(n) / n, np.full(n, 2.5),
              O.project_simplex(rng.random(n), tau)):
        got = yb.project_simplex(torch.from_numpy(y), tau).cpu().numpy()
        ref = O.project_simplex(y, tau)
        assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(y).max())
        assert got.min() >= tau * (1 - 1e-12)


@pytest.mark.parametrize("wl", ["n12_T500", "n400_T4800"])
def test_kkt_residual_matches_oracle(wl):
    print(f"[case] kkt {wl}", flush=True)
    R = synth.workload_returns(wl)
    mu, A = O.center(R)
    n = mu.size
    c = np.array(synth.WORKLOADS[wl]["c"])
    ctx = yb.Context(torch.from_numpy(R).cuda())
    rng = np.random.default_rng(5)
    x = rng.random(n)
    x /= x.sum()
    for w in (np.full(n, 1.0 / n), np.eye(n)[int(np.argmax(mu))], x):
        for tau in (0.0, 1e-8):
            got = ctx.kkt_residual(c, w, tau)
            assert got == pytest.approx(O.kkt_residual(A, mu, c, w, tau), rel=1e-9, abs=1e-18)
    ctx.close()


@pytest.mark.parametrize("iters", [1, 3, 6, 11])
def test_boundary_block_iterates_match_oracle(iters):
    """n12_T500 with c = (1,1,1,1): the optimum sits on a two-asset face;
    the run takes projected trial steps and then continues on that face."""
    print(f"[case] simplex boundary block iters={iters}", flush=True)
    R = synth.workload_returns("n12_T500")
    c = np.array([1.0, 1.0, 1.0, 1.0])
    xr, ir = O.solve(R, c, opts=O.Options(feasible_set="simplex", max_iter=iters, eps=0.0))
    ctx = yb.Context(torch.from_numpy(R).cuda())
    w, info = ctx.solve(c, opts=yb.default_opts(feasible_set="simplex", max_iter=iters, eps=0.0))
    w = w.cpu().numpy()
    assert info.iterations == iters
    assert info.projected_steps == ir.projected_steps
    assert np.abs(w - xr).max() <= 1e-9
    assert w.min() >= 1e-8 - 1e-15 and abs(w.sum() - 1.0) <= 1e-12
    ctx.close()


def test_boundary_block_solve_reaches_simplex_minimiser():
    R = synth.workload_returns("n12_T500")
    mu, A = O.center(R)
    c = np.array([1.0, 1.0, 1.0, 1.0])
    xr, ir = O.solve(R, c, opts=O.Options(feasible_set="simplex"))
    ctx = yb.Context(torch.from_numpy(R).cuda())
    w, info = ctx.solve(c, opts=yb.default_opts(feasible_set="simplex"))
    w = w.cpu().numpy()
    print(f"GPU {info.iterations} it, {info.projected_steps} projected, kkt {info.kkt:.2e}", flush=True)
    assert info.status == 0 and ir.status == 0
    assert info.iterations == ir.iterations
    assert np.abs(w - xr).max() <= 1e-9
    assert info.kkt == pytest.approx(O.kkt_residual(A, mu, c, w, 1e-8), rel=1e-8, abs=1e-12)
    assert info.kkt <= 1e-8
    ctx.close()


@pytest.mark.parametrize("gamma", [3.0, 8.0])
def test_boundary_block_certified_convex_direct_and_pcg(gamma):
    """CRRA coefficients (certified convex): a unique minimiser over the
    simplex, reached by the direct and the PCG configurations alike and by
    the oracle."""
    print(f"[case] simplex CRRA gamma={gamma} n400_T4800", flush=True)
    R = synth.workload_returns("n400_T4800")
    mu, A = O.center(R)
    c = synth.crra_coefficients(gamma)
    xr, ir = O.solve(R, c, opts=O.Options(feasible_set="simplex"))
    ctx = yb.Context(torch.from_numpy(R).cuda())
    wd, idr = ctx.solve(c, opts=yb.default_opts(feasible_set="simplex"))
    wp, ipc = ctx.solve(c, opts=yb.default_opts(large=True, feasible_set="simplex"))
    wd, wp = wd.cpu().numpy(), wp.cpu().numpy()
    print(f"direct {idr.iterations} it kkt {idr.kkt:.2e}; pcg {ipc.iterations} it "
          f"kkt {ipc.kkt:.2e}; oracle {ir.iterations} it kkt {ir.kkt:.2e}", flush=True)
    assert idr.status == 0 and ir.status == 0
    assert np.abs(wd - xr).max() <= 1e-6
    # the PCG configuration against the oracle's PCG run: same outcome and
    # iterations (the Krylov steps agree element by element), the same
    # stationary point of the face up to its KKT tolerance
    oo = O.Options.large()
    oo.feasible_set = "simplex"
    xp, ip = O.solve(R, c, opts=oo)
    assert ipc.status == ip.status == 0
    assert ipc.iterations == ip.iterations and ipc.restarts == ip.restarts
    assert np.abs(wp - xp).max() <= 1e-6
    assert ipc.kkt <= 1e-8
    assert O.objective(A, mu, c, wp) <= O.objective(A, mu, c, xr) + 1e-9
    ctx.close()


@pytest.mark.parametrize("n,large,c", [
    (60, False, (10.0, 1.0, 10.0, 1.0)),
    (60, False, (10.0, 10.0, 10.0, 10.0)),
    (300, True, (10.0, 10.0, 10.0, 10.0)),
])
def test_uniform_T252_matches_oracle(n, large, c):
    """The paper's synthetic coefficient-stress generator (returns uniform on
    [-0.1, 0.4], T = 252), direct configuration below T and the PCG
    configuration with stall recovery above it (n > T: the regularised
    stress regime).  Same outcome, iterations and iterates as the oracle."""
    print(f"[case] uniform T=252 n={n} {'PCG' if large else 'direct'} c={c}", flush=True)
    R = synth.uniform_returns(n, 252, seed=n)
    if large:
        oo = O.Options.large()
        oo.feasible_set = "simplex"
    else:
        oo = O.Options(feasible_set="simplex")
    xr, ir = O.solve(R, c, opts=oo)
    ctx = yb.Context(torch.from_numpy(R).cuda())
    w, info = ctx.solve(c, opts=yb.default_opts(large=large, feasible_set="simplex"))
    w = w.cpu().numpy()
    assert info.status == ir.status and info.iterations == ir.iterations
    assert info.restarts == ir.restarts
    # same iterations; both runs stop inside the KKT tolerance 1e-8, which
    # leaves up to ~1e-8 between the two final iterates on the optimal face
    assert np.abs(w - xr).max() <= 1e-8
    # the residual is dominated by the bound coordinates' tau = 1e-8, so it
    # is compared through the projection's nonexpansiveness:
    # |kkt(w) - kkt(xr)| <= 2 |w - xr| + |grad f(w) - grad f(xr)|
    mu, A = O.center(R)
    bound = (2.0 * np.linalg.norm(w - xr)
             + np.linalg.norm(O.gradient(A, mu, np.array(c), w)
                              - O.gradient(A, mu, np.array(c), xr)))
    assert abs(info.kkt - ir.kkt) <= bound + 1e-12 * ir.kkt + 1e-15
    ctx.close()


@pytest.mark.parametrize("n,T,large,c", [
    (30, 252, False, (1.0, 10.0, 1.0, 10.0)),
    (120, 252, False, (10.0, 10.0, 10.0, 10.0)),
    (400, 252, True, (1.0, 10.0, 1.0, 10.0)),
    (700, 252, True, (10.0, 10.0, 10.0, 10.0)),
    (1000, 252, False, (1.0, 10.0, 1.0, 10.0)),
    (150, 2000, True, (1.0, 10.0, 1.0, 10.0)),
])
def test_stress_generator_reaches_the_oracle_minimiser(n, T, large, c):
    """Certified profiles on the uniform stress generator, both
    configurations, n below and above T: the library reaches the simplex
    KKT target and the oracle's objective (a unique minimum value)."""
    print(f"[case] stress n={n} T={T} {'PCG' if large else 'direct'} c={c}",
          flush=True)
    R = synth.uniform_returns(n, T, seed=n + T)
    mu, A = O.center(R)
    if large:
        oo = O.Options.large()
        oo.feasible_set = "simplex"
    else:
        oo = O.Options(feasible_set="simplex")
    xr, ir = O.solve(R, c, opts=oo)
    ctx = yb.Context(torch.from_numpy(R).cuda())
    w, info = ctx.solve(c, opts=yb.default_opts(large=large,
                                                feasible_set="simplex"))
    ctx.close()
    w = w.cpu().numpy()
    print(f"GPU {info.status} {info.iterations} it kkt {info.kkt:.1e}; oracle "
          f"{ir.status} {ir.iterations} it kkt {ir.kkt:.1e}", flush=True)
    assert info.kkt <= 1e-6 and ir.kkt <= 1e-6
    fr, fw = O.objective(A, mu, np.array(c), xr), O.objective(A, mu, np.array(c), w)
    assert fw == pytest.approx(fr, rel=1e-9, abs=1e-12)


def test_single_free_coordinate_face_takes_a_zero_step():
    """A face with one free coordinate has a zero direction: the step must
    be 0 (constant quartic model), not an unbounded-model error.  Factor
    panel n = 2000, T = 500, profile [10,1,10,1] outside the certificate,
    direct configuration, where such a face occurs on the way."""
    print("[case] zero-direction face n=2000 T=500", flush=True)
    R = synth.factor_returns(2000, 500, 3, 2, 4.0, 0.01, 7)
    ctx = yb.Context(torch.from_numpy(R).cuda())
    w, info = ctx.solve([10.0, 1.0, 10.0, 1.0],
                        opts=yb.default_opts(feasible_set="simplex"))
    ctx.close()
    w = w.cpu().numpy()
    # n > T: the tangent Hessian has rank <= T, the direct configuration
    # factors it at the escalated lam = 1e-12 of its mean curvature, and its
    # null-space components are then set by rounding (eigenvalues ~1e-18
    # against lam ~1e-17), so the library's and the oracle's directions part
    # by ~1% from the first iteration.  Only the outcome class is checked: no
    # error, a point of the slice.
    assert info.status in (0, 1, 2)
    assert np.isfinite(w).all() and abs(w.sum() - 1.0) <= 1e-12
    assert w.min() >= 1e-8 - 1e-15
    # the zero direction of a one-coordinate face is a constant quartic
    # model; the library and the oracle both take the step 0
    coef = np.array([info.f, 0.0, 0.0, 0.0, 0.0])
    ctx2 = yb.Context(torch.from_numpy(R[:, :4]).cuda())
    assert ctx2.select_step(coef, float("inf")) == 0.0
    assert ctx2.select_step(coef, 0.25) == 0.0
    ctx2.close()
    assert O.select_step(coef) == 0.0 and O.select_step(coef, 0.25) == 0.0
