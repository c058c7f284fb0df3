"""yand_mvsk_solve_R_noalloc, the allocation-free variant of the stateless
solve, against yand_mvsk_solve_R through the C-ABI: two calls in a row, the
second on a smaller instance (the fixed scratch array then still holds the
first call's contents), each compared element by element with the existing
entry point (same kernels, same reduction order: the results agree to the
last bit up to 1e-15 of |w|_inf) and with the FP64 oracle's solve (objective
relative error 1e-10, weights within 10 eps / lambda_min of the reduced
Hessian, as in the other solve-level parity tests).  An instance beyond the
array is refused before any device work.
"""

import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2604_25378_amd import binding as yb  # noqa: E402


def _kappa_w(R, c, x):
    mu, A = O.center(R)
    C, _ = O.constraints(mu)
    U = O.tangent_basis(C)
    H = A.T @ (O.d2psi(c, A @ x)[:, None] * A) / A.shape[0]
    return 10 * 1e-8 / np.linalg.eigvalsh(U.T @ H @ U)[0]


@pytest.mark.parametrize("first,second", [("n400_T4800", "n12_T500")])
def test_noalloc_matches_stateless_solve_twice(first, second):
    for wl in (first, second):
        print(f"[case] noalloc solve {wl}", flush=True)
        R = synth.workload_returns(wl)
        c = np.array(synth.WORKLOADS[wl]["c"])
        Rd = torch.from_numpy(R).cuda()
        n = R.shape[1]
        ref = yb.solve_R(Rd, c).cpu().numpy()
        out = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        got = yb.solve_R_noalloc(Rd, c, out=out).cpu().numpy()
        diff = float(np.abs(got - ref).max())
        print(f"  |w_noalloc - w_R|_inf = {diff:.3e}", flush=True)
        assert diff <= 1e-15 * np.abs(ref).max()
        xr, ir = O.solve(R, c)
        mu, A = O.center(R)
        f = O.objective(A, mu, c, got)
        assert abs(f - ir.f) <= 1e-10 * abs(ir.f)
        assert np.abs(got - xr).max() <= _kappa_w(R, c, xr)
        assert abs(got.sum() - 1.0) <= 1e-12


def test_noalloc_with_target_matches_stateless_solve():
    print("[case] noalloc solve n12_T500 with a return target", flush=True)
    R = synth.workload_returns("n12_T500")
    c = np.array(synth.WORKLOADS["n12_T500"]["c"])
    mu, _ = O.center(R)
    r = float(np.quantile(mu, 0.7))
    Rd = torch.from_numpy(R).cuda()
    ref = yb.solve_R(Rd, c, target=r).cpu().numpy()
    got = yb.solve_R_noalloc(Rd, c, target=r).cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-15 * np.abs(ref).max()
    assert abs(mu @ got - r) <= 1e-12


def test_noalloc_refuses_instances_beyond_the_array():
    print("[case] noalloc too large", flush=True)
    Rd = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    lib = yb.load()
    import ctypes as C
    c = (1.0, 1.0, 1.0, 1.0)
    # the size check runs before R is read: a 12000 x 2000 instance needs
    # more than the 256 MiB array
    rc = lib.yand_mvsk_solve_R_noalloc(C.c_void_p(Rd.data_ptr()), 12000, 2000,
                                       *c, None, C.c_void_p(out.data_ptr()))
    assert rc == -7
