"""The launch-shape autotuner: chosen shapes come from the candidate sets,
results under any shape agree with the default shapes to rounding order
(1e-13 relative; only the grouping of the FP64 sums changes), and solves
after tuning still reach the oracle's unique minimiser."""

import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2604_25378_amd import binding as yb  # noqa: E402


def test_autotune_shapes_and_results():
    R = synth.factor_returns(300, 2000, 5, 0, 5.0, 0.0, 7)
    print("[case] autotune n=300 T=2000", flush=True)
    c = np.array([1.0, 5.0, 2.0, 10.0])
    mu, A = O.center(R)
    ctx = yb.Context(torch.from_numpy(R).cuda())
    assert ctx.tuning() == [0] * 7
    x = np.full(300, 1.0 / 300) + 1e-3 * np.random.default_rng(1).normal(size=300)
    x -= (x.sum() - 1.0) / 300
    v = np.random.default_rng(2).normal(size=300)
    f0, g0, _ = ctx.eval(c, x)
    h0 = ctx.hvp(c, x, v).cpu().numpy()
    rep = ctx.autotune()
    assert set(rep["pass_groups"].values()) <= {256, 384, 512, 768, 1024}
    assert rep["chol_group"] in (2, 4, 8)
    assert all(t > 0 for t in rep["ms"].values())
    assert ctx.tuning() == [*rep["pass_groups"].values(), rep["chol_group"]]
    for shape in ([1024] * 6 + [2], [256] * 6 + [8], None):
        if shape is not None:
            ctx.tuning(shape)
        f, g, _ = ctx.eval(c, x)
        h = ctx.hvp(c, x, v).cpu().numpy()
        assert f == pytest.approx(f0, rel=1e-13)
        assert np.abs(g.cpu().numpy() - g0.cpu().numpy()).max() <= 1e-13 * np.abs(g0.cpu().numpy()).max()
        assert np.abs(h - h0).max() <= 1e-13 * np.abs(h0).max()
        w, info = ctx.solve(c)
        assert info.status == 0 and info.gnorm <= 1e-8
        xr, _ = O.solve(R, c)
        Cm, _ = O.constraints(mu)
        U = O.tangent_basis(Cm)
        assert np.linalg.norm(U.T @ O.gradient(A, mu, c, w.cpu().numpy())) <= 2e-8
        Hr = U.T @ (A.T @ (O.d2psi(c, A @ xr)[:, None] * A) / A.shape[0]) @ U
        assert np.abs(w.cpu().numpy() - xr).max() <= 10 * 1e-8 / np.linalg.eigvalsh(Hr)[0]
    with pytest.raises(yb.YandError):
        ctx.tuning([-1, 0, 0, 0, 0, 0, 0])
    ctx.close()
