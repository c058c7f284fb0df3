"""GPU parity of the Armijo step rule and of solves on the controlled-
conditioning generator, through the C-ABI against the FP64 oracle.

Iterates are compared element by element (1e-9, like the other solve-level
parity tests); the Armijo decisions compare the same Horner-form decrease
on both sides, so equal coefficients to rounding give equal steps except at
an exact tie of the sufficient-decrease test.
"""

import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2604_25378_amd import binding as yb  # noqa: E402


@pytest.mark.parametrize("fs", ["budget", "simplex"])
@pytest.mark.parametrize("iters", [1, 5, 300])
def test_armijo_iterates_match_oracle(fs, iters):
    print(f"[case] armijo {fs} iters={iters}", flush=True)
    R = synth.workload_returns("n12_T500")
    c = np.array([1.0, 1.0, 1.0, 1.0])
    eps = 0.0 if iters < 300 else 1e-8
    xr, ir = O.solve(R, c, opts=O.Options(feasible_set=fs, linesearch="armijo",
                                         max_iter=iters, eps=eps))
    ctx = yb.Context(torch.from_numpy(R).cuda())
    w, info = ctx.solve(c, opts=yb.default_opts(feasible_set=fs, linesearch="armijo",
                                                max_iter=iters, eps=eps))
    w = w.cpu().numpy()
    assert info.iterations == ir.iterations
    assert np.abs(w - xr).max() <= 1e-9
    if iters == 300:
        assert info.status == 0 and ir.status == 0
    ctx.close()


@pytest.mark.parametrize("kappa", [1.0, 1e3])
def test_conditioned_crra_matches_oracle(kappa):
    """The controlled-conditioning generator (kappa_+(AU) = kappa, A x0 = 0),
    CRRA gamma = 6, simplex with the boundary block: same iterations and
    iterates as the oracle (direct configuration), and the PCG
    configuration ends at the same minimiser."""
    print(f"[case] conditioned n=120 T=240 kappa={kappa}", flush=True)
    R = synth.conditioned_returns(120, 240, kappa, seed=3)
    mu, A = O.center(R)
    c = synth.crra_coefficients(6.0)
    xr, ir = O.solve(R, c, opts=O.Options(feasible_set="simplex"))
    ctx = yb.Context(torch.from_numpy(R).cuda())
    w, info = ctx.solve(c, opts=yb.default_opts(feasible_set="simplex"))
    w = w.cpu().numpy()
    assert info.status == ir.status and info.iterations == ir.iterations
    assert np.abs(w - xr).max() <= 1e-9
    wp, ip = ctx.solve(c, opts=yb.default_opts(large=True, feasible_set="simplex"))
    wp = wp.cpu().numpy()
    assert O.objective(A, mu, c, wp) <= O.objective(A, mu, c, xr) + 1e-10 * abs(O.objective(A, mu, c, xr))
    ctx.close()
