"""The launch-shape autotuner: chosen shapes come from the candidate sets,
results under any shape agree with the default shapes to rounding order
(1e-13 relative; workgroup counts and block heights only regroup the FP64
sums), the Cholesky's sub-block and band widths change no bit of a solve,
and solves after tuning still reach the oracle's unique minimiser."""

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
    assert ctx.tuning() == [0] * 15
    x = np.full(300, 1.0 / 300) + 1e-3 * np.random.default_rng(1).normal(size=300)
    x -= (x.sum() - 1.0) / 300
    v = np.random.default_rng(2).normal(size=300)
    f0, g0, _ = ctx.eval(c, x)
    h0 = ctx.hvp(c, x, v).cpu().numpy()
    rep = ctx.autotune()
    assert set(rep["pass_groups"].values()) <= {256, 384, 512, 768, 1024}
    assert rep["chol_group"] in (2, 3, 4, 5, 6, 8)
    assert set(rep["pass_rows"].values()) <= {0, 1, 2, 4}
    assert rep["chol_step_tm"] in (0, 32, 64) and rep["chol_band"] in (0, 32, 64)
    assert all(t > 0 for t in rep["ms"].values())
    assert ctx.tuning() == [*rep["pass_groups"].values(), rep["chol_group"],
                            *rep["pass_rows"].values(), rep["chol_step_tm"],
                            rep["chol_band"]]
    print(f"tuned {ctx.tuning()}", flush=True)
    for shape in ([1024] * 6 + [2] + [1] * 6 + [64, 64],
                  [256] * 6 + [8] + [4] * 6 + [32, 64],
                  [384] * 6 + [4] + [2] * 6 + [64, 32], None):
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
    for bad in ([-1] + [0] * 14, [0] * 7 + [3] + [0] * 7, [0] * 13 + [48, 0],
                [0] * 14 + [128]):
        with pytest.raises(yb.YandError):
            ctx.tuning(bad)
    with pytest.raises(ValueError):
        ctx.tuning([0] * 7)
    ctx.close()


@pytest.mark.parametrize("grp", [2, 4])
def test_cholesky_widths_change_no_bit(grp):
    """Every entry of the factor and its inverse is the same product over the
    same reduction whatever the sub-block and band widths, so three
    iterations of a solve (n = 1000: eight tile columns, in-group updates
    and group updates) end on the same weights bit for bit."""
    print(f"[case] cholesky widths n=1000 T=3000 group {grp}", flush=True)
    R = synth.factor_returns(1000, 3000, 5, 3, 5.0, 0.0, 11)
    c = [1.0, 5.0, 2.0, 10.0]
    ctx = yb.Context(torch.from_numpy(R).cuda())
    opts = yb.default_opts(max_iter=3, eps=0.0)
    ref = None
    for tm, band in ((0, 0), (64, 32), (32, 64), (64, 64)):
        ctx.tuning([0] * 6 + [grp] + [0] * 6 + [tm, band])
        w, info = ctx.solve(c, opts=opts)
        assert info.iterations == 3
        w = w.cpu().numpy()
        if ref is None:
            ref = w
        else:
            assert np.array_equal(w, ref), (tm, band)
    ctx.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_block_heights_regroup_sums_only(precision):
    """Every block height of every pass (1, 2 and 4 rows, each capped by
    the storage type's register budget) gives the default shape's value,
    gradient and Hessian-vector product to rounding order (1e-13)."""
    print(f"[case] block heights n=300 T=2000 {precision}", flush=True)
    R = synth.factor_returns(300, 2000, 5, 0, 5.0, 0.0, 7)
    c = np.array([1.0, 5.0, 2.0, 10.0])
    ctx = yb.Context(torch.from_numpy(R).cuda(), precision)
    x = np.full(300, 1.0 / 300) + 1e-3 * np.random.default_rng(3).normal(size=300)
    x -= (x.sum() - 1.0) / 300
    v = np.random.default_rng(4).normal(size=300)
    f0, g0, _ = ctx.eval(c, x)
    g0 = g0.cpu().numpy()
    h0 = ctx.hvp(c, x, v).cpu().numpy()
    # two iterations run the value, line-search and third-order passes too
    opts = yb.default_opts(max_iter=2, eps=0.0)
    w0, _ = ctx.solve(c, opts=opts)
    w0 = w0.cpu().numpy()
    for rows in (1, 2, 4):
        ctx.tuning([0] * 7 + [rows] * 6 + [0, 0])
        f, g, _ = ctx.eval(c, x)
        h = ctx.hvp(c, x, v).cpu().numpy()
        assert f == pytest.approx(f0, rel=1e-13)
        assert np.abs(g.cpu().numpy() - g0).max() <= 1e-13 * np.abs(g0).max()
        assert np.abs(h - h0).max() <= 1e-13 * np.abs(h0).max()
        w, info = ctx.solve(c, opts=opts)
        assert info.iterations == 2
        assert np.abs(w.cpu().numpy() - w0).max() <= 1e-10
    ctx.close()
