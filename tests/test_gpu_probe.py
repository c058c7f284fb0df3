"""GPU parity of the probe estimate of the trace (trace_mode = probe) against
the oracle's, through the C-ABI.

Both sides draw the same SplitMix64 signs and run the probe solves and the
tangent solve with the same projected PCG (same preconditioner, tolerance
and budget), so the two estimates differ only by rounding.  The probe solves
usually stop at the iteration budget (15) with their residuals still above
the tolerance, and CG's rounding grows over those steps by about the
condition number per step, so directions are compared to 1e-5 relative to
|d|_inf (measured 7.5e-7 to 2.3e-6, the larger with fewer probes) and solve
iterates to 1e-6 of |w|_inf, with the
same iteration and Krylov counts.  The probe direction is a descent
direction (g^T d = -|gbar|) and the solve ends at the exact route's
minimiser (objective relative error 1e-10).
"""

import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2604_25378_amd import binding as yb  # noqa: E402


def _inst():
    R = synth.factor_returns(300, 1000, 5, 0, 5.0, 0.0, 7)
    return R, np.array([1.0, 5.0, 2.0, 10.0])


def _x(mu, seed):
    n = mu.shape[0]
    x = np.full(n, 1.0 / n) + 0.1 / n * np.random.default_rng(seed).normal(size=n)
    return x - (x.sum() - 1.0) / n


@pytest.mark.parametrize("k,target,seed", [(64, False, 0), (7, False, 3),
                                           (33, True, 12345678901234567)])
def test_probe_direction_matches_oracle(k, target, seed):
    print(f"[case] probe direction n=300 T=1000 k={k} target={target}", flush=True)
    R, c = _inst()
    mu, A = O.center(R)
    r = float(np.quantile(mu, 0.6)) if target else None
    Cm, b = O.constraints(mu, r)
    U = O.tangent_basis(Cm)
    x = O.feasible_start(Cm, b, _x(mu, 5))
    ref = O.affine_normal(A, mu, c, x, U, solver="pcg", reg=1e-4,
                          trace="probe", probes=k, seed=seed, draw=0)
    ctx = yb.Context(torch.from_numpy(R).cuda())
    opts = yb.default_opts(large=True, trace_mode="probe", probes=k,
                           probe_seed=seed)
    d, gn = ctx.affine_normal(c, x, target=r, opts=opts)
    d = d.cpu().numpy()
    ctx.close()
    assert gn == pytest.approx(ref.gnorm, rel=1e-11)
    err = np.abs(d - ref.d).max() / np.abs(ref.d).max()
    print(f"  direction error {err:.2e}", flush=True)
    assert err <= 1e-5
    g = O.gradient(A, mu, c, x)
    assert float(g @ d) == pytest.approx(-ref.gnorm, rel=1e-9)
    # the estimate differs from the exact trace's direction
    ex = O.affine_normal(A, mu, c, x, U, solver="pcg", reg=1e-4).d
    assert np.abs(ex - ref.d).max() > 1e2 * err * np.abs(ref.d).max()


def test_probe_solve_matches_oracle():
    """Budget set, PCG configuration with the probe trace: the same
    iterations, Krylov counts and iterates as the oracle's probe solve, and
    the exact route's minimiser."""
    print("[case] probe solve n=300 T=1000", flush=True)
    R, c = _inst()
    mu, A = O.center(R)
    oo = O.Options.large()
    oo.trace, oo.probes, oo.probe_seed = "probe", 64, 9
    xr, ir = O.solve(R, c, opts=oo)
    ctx = yb.Context(torch.from_numpy(R).cuda())
    w, info = ctx.solve(c, opts=yb.default_opts(large=True, trace_mode="probe",
                                                probes=64, probe_seed=9))
    w = w.cpu().numpy()
    assert info.status == ir.status == 0
    assert info.iterations == ir.iterations
    assert info.cg_iters == ir.cg_iters
    assert info.probe_cg_iters == ir.probe_iters
    assert info.probe_traces == ir.directions and info.dense_traces == 0
    assert np.abs(w - xr).max() <= 1e-6 * np.abs(xr).max()
    assert abs(O.objective(A, mu, c, w) - ir.f) <= 1e-10 * abs(ir.f)
    we, ie = ctx.solve(c, opts=yb.default_opts(large=True))
    ctx.close()
    fe = O.objective(A, mu, c, we.cpu().numpy())
    assert abs(O.objective(A, mu, c, w) - fe) <= 1e-10 * abs(fe)


def test_probe_simplex_solve_matches_oracle():
    """Simplex set with the boundary block (faces mask the probe solves),
    the paper's uniform T = 252 generator with n > T."""
    print("[case] probe simplex n=300 T=252", flush=True)
    R = synth.uniform_returns(300, 252, seed=300)
    c = np.array([10.0, 10.0, 10.0, 10.0])
    oo = O.Options.large()
    oo.feasible_set = "simplex"
    oo.trace, oo.probes, oo.probe_seed = "probe", 16, 4
    xr, ir = O.solve(R, c, opts=oo)
    ctx = yb.Context(torch.from_numpy(R).cuda())
    w, info = ctx.solve(c, opts=yb.default_opts(
        large=True, feasible_set="simplex", trace_mode="probe", probes=16,
        probe_seed=4))
    w = w.cpu().numpy()
    ctx.close()
    print(f"  GPU {info.status} {info.iterations} it kkt {info.kkt:.1e}; "
          f"oracle {ir.status} {ir.iterations} it kkt {ir.kkt:.1e}", flush=True)
    assert info.status == ir.status and info.iterations == ir.iterations
    assert info.probe_cg_iters == ir.probe_iters
    assert np.abs(w - xr).max() <= 1e-6 * np.abs(xr).max()


def test_probe_options_are_checked():
    R, c = _inst()
    ctx = yb.Context(torch.from_numpy(R).cuda())
    for kw in ({"probes": 0}, {"probes": 65}, {"trace_mode": 2}):
        with pytest.raises(yb.YandError) as e:
            ctx.solve(c, opts=yb.default_opts(large=True, **kw))
        assert e.value.code == -1
    ctx.close()
