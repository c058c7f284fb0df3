"""GPU parity of the return-floor protocol (yand_return_floor) and of the
face-solver hand-off in the simplex boundary block, through the C-ABI
against the FP64 oracle.

Tolerances.  The floor is an order statistic interpolation of mu, whose
device sum differs from numpy's in rounding order only (relative 1e-13);
c2..c4 divide the profile by equal-weight moments from a device reduction
(relative 1e-12).  The calibrated c1 is the root of mu^T x(c1) = floor,
which both sides bracket to 1e-9 (max mu - min mu) in the mean return; two
solves differ by about 1e-12 in mu^T x, which moves the root by a relative
1e-8 or so on these panels, so c1 is compared to 1e-6 and the weights to
1e-7.  Bisection paths may differ where a comparison with the floor flips
on rounding; only the outcome is compared.
"""

import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2604_25378_amd import binding as yb  # noqa: E402

KURT = (1.0, 1.0, 10.0)
BAL = (1.0, 1.0, 1.0)
SKEW = (1.0, 10.0, 1.0)


def _compare(R, profile, q, large):
    oo = O.Options.large() if large else O.Options()
    oo.feasible_set = "simplex"
    ref = O.return_floor(R, profile, q, opts=oo)
    ctx = yb.Context(torch.from_numpy(R).cuda())
    c, w, floor, ret, info, solves = ctx.return_floor(
        profile, q, opts=yb.default_opts(large=large, feasible_set="simplex"))
    w = w.cpu().numpy()
    ctx.close()
    mu = R.mean(axis=0)
    spread = mu.max() - mu.min()
    print(f"GPU c1 {c[0]:.10g} ({solves} solves, {info.iterations} it, kkt "
          f"{info.kkt:.1e}); oracle c1 {ref.c[0]:.10g} ({ref.solves} solves)",
          flush=True)
    assert floor == pytest.approx(ref.floor, rel=1e-13)
    for k in (1, 2, 3):
        assert c[k] == pytest.approx(ref.c[k], rel=1e-12)
    # the study's projected-KKT target (a solve may end at the stall test
    # just above eps = 1e-8 when n > T)
    assert info.kkt <= 1e-6 and ref.info.kkt <= 1e-6
    if ref.c[0] == 0.0:
        assert c[0] == 0.0 and solves == 1
    else:
        assert c[0] == pytest.approx(ref.c[0], rel=1e-6)
        assert abs(ret - floor) <= 1e-9 * spread
    assert ret == pytest.approx(float(mu @ w), rel=1e-12)
    assert np.abs(w - ref.x).max() <= 1e-7
    assert abs(w.sum() - 1.0) <= 1e-12 and w.min() >= 1e-8 - 1e-15


@pytest.mark.parametrize("profile,q", [(KURT, 0.4), (KURT, 0.6), (BAL, 0.6)])
def test_return_floor_direct_matches_oracle(profile, q):
    print(f"[case] return floor direct n=60 T=600 profile={profile} q={q}",
          flush=True)
    _compare(synth.priced_factor_returns(60, 600, 3, 5.0, 3), profile, q,
             large=False)


def test_return_floor_pcg_matches_oracle():
    print("[case] return floor PCG n=200 T=1000 balanced q=0.6", flush=True)
    _compare(synth.priced_factor_returns(200, 1000, 3, 5.0, 3), BAL, 0.6,
             large=True)


def test_return_floor_pcg_thin_route_matches_oracle():
    # n = 600 > 2 T = 504: every PCG direction takes the T x T exact trace
    print("[case] return floor PCG n=600 T=252 kurtosis q=0.9", flush=True)
    _compare(synth.priced_factor_returns(600, 252, 3, 5.0, 3), KURT, 0.9,
             large=True)


@pytest.mark.parametrize("q", [0.5, 0.8])
def test_return_floor_two_assets_closed_form(q):
    # the floor fixes the two-asset portfolio: t mu_1 + (1 - t) mu_2 = floor
    print(f"[case] return floor two assets q={q}", flush=True)
    R = synth.priced_factor_returns(2, 400, 3, 5.0, 4)
    mu = R.mean(axis=0)
    ctx = yb.Context(torch.from_numpy(R).cuda())
    c, w, floor, ret, info, solves = ctx.return_floor(KURT, q)
    ctx.close()
    t = (floor - mu[1]) / (mu[0] - mu[1])
    assert c[0] > 0.0
    assert w.cpu().numpy()[0] == pytest.approx(t, abs=1e-9)


def test_return_floor_slack_floor_keeps_c1_zero():
    print("[case] return floor q=0", flush=True)
    R = synth.priced_factor_returns(20, 300, 3, 5.0, 5)
    ctx = yb.Context(torch.from_numpy(R).cuda())
    c, w, floor, ret, info, solves = ctx.return_floor(KURT, 0.0)
    ctx.close()
    assert c[0] == 0.0 and solves == 1 and ret >= floor


def test_return_floor_outside_certificate_matches_oracle():
    # the skew-focused profile normalised on this panel lies outside the
    # convexity certificate; regularisation escalation keeps the directions
    # defined on both sides, which follow the same iterates
    print("[case] return floor skew-focused n=20", flush=True)
    _compare(synth.priced_factor_returns(20, 300, 3, 5.0, 5), SKEW, 0.5,
             large=False)


def test_return_floor_rejects_bad_arguments():
    print("[case] return floor bad arguments", flush=True)
    R = synth.priced_factor_returns(20, 300, 3, 5.0, 5)
    ctx = yb.Context(torch.from_numpy(R).cuda())
    for args, kw in (((KURT, 1.5), {}), (((1.0, -1.0, 1.0), 0.5), {}),
                     ((KURT, 0.5), {"opts": yb.default_opts()}),
                     ((KURT, 0.5), {"max_rounds": -1})):
        with pytest.raises(yb.YandError) as e:
            ctx.return_floor(*args, **kw)
        assert e.value.code == -1
    ctx.close()


def test_face_solver_handoff_matches_oracle():
    """A solve where the direction on the released face drives a bound
    coordinate down and no segment descends: both sides hand the coordinate
    to the face solver and reach the simplex KKT point with the same
    iterations and iterates."""
    print("[case] face-solver hand-off n=60 T=600", flush=True)
    R = synth.priced_factor_returns(60, 600, 3, 5.0, 3)
    mu, A = O.center(R)
    n = R.shape[1]
    m = O.moments(A, mu, np.full(n, 1.0 / n))
    c = np.array([4434.270595, 1.0 / m[1], 1.0 / abs(m[2]), 10.0 / m[3]])
    xr, ir = O.solve(R, c, opts=O.Options(feasible_set="simplex"))
    ctx = yb.Context(torch.from_numpy(R).cuda())
    w, info = ctx.solve(c, opts=yb.default_opts(feasible_set="simplex"))
    ctx.close()
    w = w.cpu().numpy()
    print(f"GPU {info.iterations} it kkt {info.kkt:.1e}; oracle "
          f"{ir.iterations} it kkt {ir.kkt:.1e}", flush=True)
    assert info.status == 0 and ir.status == 0
    assert info.iterations == ir.iterations
    assert info.projected_steps == ir.projected_steps
    # the iterations agree step for step; the last one lands inside the KKT
    # tolerance 1e-8 on both sides, and on this stiff instance (c4 ~ 3e9)
    # that leaves about 1e-9 of slack in the weights
    assert np.abs(w - xr).max() <= 1e-8
    assert info.kkt <= 1e-8
