"""GPU parity of the batched solves (frontier on a shared A, ragged universes).

Every instance of a batch must reach the same unique minimiser as a single
solve of that instance and as the FP64 oracle (weights within
10 eps / lambda_min of the reduced Hessian).  Graph replay and eager
enqueueing run identical kernels in identical order, so their results must be
bit-identical.
"""

import numpy as np
import pytest

import oracle as O
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2604_25378_amd import binding as yb  # noqa: E402


def _kappa_w(R, c, x, target, eps=1e-8):
    mu, A = O.center(R)
    Cm, _ = O.constraints(mu, target)
    U = O.tangent_basis(Cm)
    Hr = U.T @ (A.T @ (O.d2psi(c, A @ x)[:, None] * A) / A.shape[0]) @ U
    return 10.0 * eps / np.linalg.eigvalsh(Hr)[0]


def _frontier_instances(R, k_targets):
    mu, _ = O.center(R)
    targets = np.linspace(np.quantile(mu, 0.3), np.quantile(mu, 0.9), k_targets)
    C4, tg = [], []
    for g in (2.0, 6.0):
        for r in targets:
            C4.append(synth.crra_coefficients(g))
            tg.append(r)
    return np.array(C4), np.array(tg)


@pytest.mark.parametrize("n,T,seed", [(12, 500, 0), (300, 1000, 7)])
def test_frontier_matches_single_and_oracle(n, T, seed):
    R = synth.factor_returns(n, T, 3, 0, 5.0, 0.0, seed)
    print(f"[case] frontier n={n} T={T}", flush=True)
    C4, tg = _frontier_instances(R, 3)
    ctx = yb.Context(torch.from_numpy(R).cuda())
    W, infos = ctx.frontier(C4, tg)
    W = W.cpu().numpy()
    for b in range(C4.shape[0]):
        assert infos[b].status == 0 and infos[b].gnorm <= 1e-8, infos[b]
        ws, _ = ctx.solve(C4[b], target=tg[b])
        xr, _ = O.solve(R, C4[b], target=tg[b])
        kw = _kappa_w(R, C4[b], xr, tg[b])
        assert np.abs(W[b] - ws.cpu().numpy()).max() <= kw
        assert np.abs(W[b] - xr).max() <= kw
        assert abs(W[b].sum() - 1.0) < 1e-12
    ctx.close()


def test_frontier_budget_only_and_waves():
    R = synth.factor_returns(40, 400, 2, 0, 5.0, 0.0, 3)
    C4 = np.array([synth.crra_coefficients(g) for g in (1.0, 2.0, 4.0, 6.0, 10.0)])
    ctx = yb.Context(torch.from_numpy(R).cuda())
    W, infos = ctx.frontier(C4)
    W = W.cpu().numpy()
    # the same batch in waves of two lanes, eager and with graph replay
    Wg, _ = yb.batch_solve([ctx] * 5, C4, max_lanes=2, use_graph=True)
    We, _ = yb.batch_solve([ctx] * 5, C4, max_lanes=2, use_graph=False)
    for b in range(5):
        assert infos[b].status == 0
        xr, _ = O.solve(R, C4[b])
        assert np.abs(W[b] - xr).max() <= _kappa_w(R, C4[b], xr, None)
        a, e = Wg[b].cpu().numpy(), We[b].cpu().numpy()
        assert np.array_equal(a, e), "graph replay differs from eager enqueue"
    ctx.close()


@pytest.mark.parametrize("n,T", [(300, 1000), (520, 600)])
def test_grouped_lanes_match_separate_streams(n, T):
    """Lanes of one context advance in lockstep with grouped launches (the
    SYRK, the factorisation and the trace GEMM of all lanes in one launch
    each); the per-lane arithmetic is unchanged, so the weights equal those
    of lanes on separate streams bit for bit, in waves, with graph replay or
    eager, with and without return targets."""
    print(f"[case] grouped lanes n={n} T={T}", flush=True)
    R = synth.factor_returns(n, T, 3, 0, 5.0, 0.0, 11)
    C4, tg = _frontier_instances(R, 3)
    ctx = yb.Context(torch.from_numpy(R).cuda())
    for targets in (tg, None):
        Wsep, isep = yb.batch_solve([ctx] * len(C4), C4, targets, max_lanes=4,
                                    grouped=False)
        for use_graph in (True, False):
            Wg, ig = yb.batch_solve([ctx] * len(C4), C4, targets, max_lanes=4,
                                    use_graph=use_graph, grouped=True)
            for b in range(len(C4)):
                assert ig[b].status == 0 and ig[b].iterations == isep[b].iterations
                assert np.array_equal(Wg[b].cpu().numpy(), Wsep[b].cpu().numpy())
    ctx.close()


def test_ragged_universes_batch():
    sizes = [17, 130, 257, 90]
    ctxs, Rs = [], []
    for i, n in enumerate(sizes):
        R = synth.factor_returns(n, 600, 4, 0, 4.0, 0.0, 1001 + i)
        Rs.append(R)
        ctxs.append(yb.Context(torch.from_numpy(R).cuda()))
    C4 = np.tile(np.array([1.0, 5.0, 2.0, 10.0]), (len(sizes), 1))
    outs, infos = yb.batch_solve(ctxs, C4)
    for i, R in enumerate(Rs):
        assert infos[i].status == 0, infos[i]
        xr, _ = O.solve(R, C4[i])
        w = outs[i].cpu().numpy()
        assert w.shape == (sizes[i],)
        assert np.abs(w - xr).max() <= _kappa_w(R, C4[i], xr, None)
    for cx in ctxs:
        cx.close()


def test_frontier_from_given_starts():
    R = synth.factor_returns(60, 500, 3, 0, 5.0, 0.0, 21)
    mu, _ = O.center(R)
    C4 = np.array([synth.crra_coefficients(g) for g in (2.0, 4.0, 8.0)])
    tg = np.quantile(mu, [0.4, 0.6, 0.8])
    ctx = yb.Context(torch.from_numpy(R).cuda())
    W, infos = ctx.frontier(C4, tg)
    # restarting from the solutions stops at the first stationarity test
    W2, infos2 = ctx.frontier(C4, tg, W0=W)
    for b in range(3):
        assert infos2[b].status == 0 and infos2[b].iterations == 0, infos2[b]
        assert np.abs(W2[b].cpu().numpy() - W[b].cpu().numpy()).max() <= 1e-14
    # an infeasible start is moved onto the constraints first
    rng = np.random.default_rng(0)
    Wr = torch.from_numpy(rng.standard_normal((3, 60)) * 0.01 + 1.0 / 60).cuda()
    W3, infos3 = ctx.frontier(C4, tg, W0=Wr)
    for b in range(3):
        assert infos3[b].status == 0
        xr, _ = O.solve(R, C4[b], target=tg[b])
        assert np.abs(W3[b].cpu().numpy() - xr).max() <= _kappa_w(R, C4[b], xr, tg[b])
        assert abs(mu @ W3[b].cpu().numpy() - tg[b]) <= 1e-14
    ctx.close()


@pytest.mark.parametrize("n", [40, 200])
def test_simplex_frontier_matches_single_solves(n):
    """Batched lanes on the simplex: the boundary block (segment trial,
    face-solver holds, projected-KKT stop) runs inside the graph-replayed
    iterations and must reproduce each instance's single solve and the
    oracle's outcome."""
    print(f"[case] simplex frontier n={n}", flush=True)
    R = synth.uniform_returns(n, 252, seed=n)
    mu, A = O.center(R)
    C4 = np.array([[1.0, 10.0, 1.0, 10.0], [10.0, 10.0, 10.0, 10.0],
                   [1.0, 5.0, 2.0, 10.0], [2.0, 1.0, 0.5, 4.0],
                   [1.0, 10.0, 1.0, 10.0]])
    opts = yb.default_opts(feasible_set="simplex")
    ctx = yb.Context(torch.from_numpy(R).cuda())
    W, infos = ctx.frontier(C4, opts=opts)
    W = W.cpu().numpy()
    for b, c in enumerate(C4):
        w1, i1 = ctx.solve(c, opts=opts)
        xr, ir = O.solve(R, c, opts=O.Options(feasible_set="simplex"))
        print(f"b={b} batch {infos[b].status} {infos[b].iterations} it kkt "
              f"{infos[b].kkt:.1e}; single {i1.iterations} it; oracle "
              f"{ir.iterations} it", flush=True)
        assert infos[b].iterations == i1.iterations
        assert infos[b].projected_steps == i1.projected_steps
        assert np.abs(W[b] - w1.cpu().numpy()).max() <= 1e-12
        assert infos[b].kkt <= 1e-6
        assert O.objective(A, mu, c, W[b]) == pytest.approx(
            O.objective(A, mu, c, xr), rel=1e-9, abs=1e-12)
    # instances 0 and 4 are the same problem
    assert np.abs(W[0] - W[4]).max() == 0.0
    ctx.close()


def _close(got, ref, rtol):
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err <= rtol, f"relative error {err:.3e} > {rtol:.1e}"


@pytest.mark.parametrize("grouped", [True, False])
@pytest.mark.parametrize("iters", [1, 4])
def test_frontier_pcg_iterates_match_single_and_oracle(grouped, iters):
    """PCG configuration in a batch.  On separate streams each lane runs the
    single solve's kernels in the same order: weights equal to the single
    solve's bit for bit.  In lockstep every CG step is one pair of block
    products for all lanes, which sum in another order: the same CG step
    counts as the single solve, and iterates as close to the oracle's as the
    single solve's within a factor 10 (the truncated inner solves amplify
    rounding differently per instance; the single solve's own iterate test
    holds c = (1, 5, 2, 10) to 1e-8, checked here too).  Budget hull: with a
    return target the truncation test of some inner solve falls within
    rounding of its tolerance for single solves as well."""
    print(f"[case] frontier PCG iterates grouped={grouped} iters={iters}",
          flush=True)
    R = synth.factor_returns(300, 1000, 5, 0, 5.0, 0.0, 7)
    C4 = np.array([[1.0, 5.0, 2.0, 10.0]] +
                  [synth.crra_coefficients(g) for g in (2.0, 4.0, 6.0, 10.0)])
    kw = dict(large=True, max_iter=iters, eps=0.0, stall_recovery=0)
    ctx = yb.Context(torch.from_numpy(R).cuda())
    W, infos = yb.batch_solve([ctx] * len(C4), C4,
                              opts=yb.default_opts(**kw), grouped=grouped)
    for b in range(len(C4)):
        w1, i1 = ctx.solve(C4[b], opts=yb.default_opts(**kw))
        w1 = w1.cpu().numpy()
        wb = W[b].cpu().numpy()
        oo = O.Options.large()
        oo.max_iter, oo.eps, oo.stall_recovery = iters, 0.0, False
        xr, ir = O.solve(R, C4[b], opts=oo)
        e1 = np.abs(w1 - xr).max() / np.abs(xr).max()
        eb = np.abs(wb - xr).max() / np.abs(xr).max()
        print(f"b={b}: cg {infos[b].cg_iters} single {i1.cg_iters} oracle "
              f"{ir.cg_iters}; error batch {eb:.2e} single {e1:.2e}",
              flush=True)
        assert infos[b].iterations == i1.iterations == iters
        assert infos[b].cg_iters == i1.cg_iters
        if grouped:
            assert eb <= 10.0 * e1 + 1e-9
        else:
            assert np.array_equal(wb, w1)
        if b == 0:
            assert infos[b].cg_iters == ir.cg_iters and eb <= 1e-8
    ctx.close()


def test_frontier_pcg_solves_match_oracle():
    """Full frontier solves in the PCG configuration (lockstep, graph
    replay), return targets: every instance converges to the oracle's
    minimiser (within kappa_w) in the oracle's number of outer iterations."""
    print("[case] frontier PCG solves n=300 T=1000", flush=True)
    R = synth.factor_returns(300, 1000, 5, 0, 5.0, 0.0, 7)
    C4, tg = _frontier_instances(R, 3)
    ctx = yb.Context(torch.from_numpy(R).cuda())
    W, infos = ctx.frontier(C4, tg, opts=yb.default_opts(large=True))
    W = W.cpu().numpy()
    for b in range(len(C4)):
        xr, ir = O.solve(R, C4[b], target=tg[b], opts=O.Options.large())
        print(f"b={b}: batch {infos[b].status} {infos[b].iterations} it "
              f"{infos[b].cg_iters} cg; oracle {ir.status} {ir.iterations} it "
              f"{ir.cg_iters} cg", flush=True)
        assert infos[b].status == ir.status == 0
        assert infos[b].iterations == ir.iterations
        assert np.abs(W[b] - xr).max() <= _kappa_w(R, C4[b], xr, tg[b])
    ctx.close()


@pytest.mark.parametrize("restart_max_iter", [1, 120])
def test_frontier_pcg_restarts_match_oracle(restart_max_iter):
    """Stall recovery inside a batch (krylov_maxit = 1, max_iter = 2): the
    instances that end the baseline phase above eps continue with twice the
    Krylov budget, then with the direct solve, like the oracle's solve;
    restarts, the iterations of every phase, status, CG steps and iterates
    match it per instance."""
    print(f"[case] frontier PCG restarts restart_max_iter={restart_max_iter}",
          flush=True)
    R = synth.workload_returns("n12_T500")
    C4 = np.array([synth.WORKLOADS["n12_T500"]["c"],
                   synth.crra_coefficients(4.0), synth.crra_coefficients(8.0)])
    ctx = yb.Context(torch.from_numpy(R).cuda())
    W, infos = ctx.frontier(C4, opts=yb.default_opts(
        large=True, krylov_maxit=1, max_iter=2,
        restart_max_iter=restart_max_iter))
    for b in range(len(C4)):
        oo = O.Options.large()
        oo.krylov_maxit, oo.max_iter, oo.restart_max_iter = 1, 2, restart_max_iter
        xr, ir = O.solve(R, C4[b], opts=oo)
        its = [p[4] for p in ir.phases]
        its = tuple(its + [0] * (3 - len(its)))
        print(f"b={b}: batch restarts {infos[b].restarts} phases "
              f"{infos[b].phase_iterations}; oracle {ir.restarts} {its}",
              flush=True)
        assert infos[b].restarts == ir.restarts
        assert infos[b].phase_iterations == its
        assert infos[b].iterations == ir.iterations
        assert infos[b].status == ir.status
        assert infos[b].cg_iters == ir.cg_iters
        assert np.abs(W[b].cpu().numpy() - xr).max() <= 1e-9
    assert any(i.restarts >= 1 for i in infos)
    ctx.close()


def test_frontier_rejects_probe_trace():
    R = synth.factor_returns(40, 400, 2, 0, 5.0, 0.0, 3)
    ctx = yb.Context(torch.from_numpy(R).cuda())
    with pytest.raises(yb.YandError) as e:
        ctx.frontier(np.array([[1.0, 5.0, 2.0, 10.0]]),
                     opts=yb.default_opts(large=True, trace_mode="probe"))
    assert e.value.code == -1
    ctx.close()


@pytest.mark.parametrize("restart_max_iter", [2, 120])
def test_frontier_pcg_simplex_restarts_match_oracle(restart_max_iter):
    """Simplex with the boundary block in a batch (no targets, so the face
    solver runs), PCG configuration, max_iter = 2: the instances continue
    with the projected trial steps 0.045 and then 0.02 like the oracle's
    solve; restarts, phase iterations, projected steps, status and iterates
    match it per instance."""
    print(f"[case] frontier PCG simplex restarts restart_max_iter="
          f"{restart_max_iter}", flush=True)
    R = synth.workload_returns("n12_T500")
    C4 = np.array([synth.WORKLOADS["n12_T500"]["c"],
                   synth.crra_coefficients(3.0), synth.crra_coefficients(7.0)])
    ctx = yb.Context(torch.from_numpy(R).cuda())
    W, infos = ctx.frontier(C4, opts=yb.default_opts(
        large=True, feasible_set="simplex", max_iter=2,
        restart_max_iter=restart_max_iter))
    for b in range(len(C4)):
        oo = O.Options.large()
        oo.feasible_set = "simplex"
        oo.max_iter, oo.restart_max_iter = 2, restart_max_iter
        xr, ir = O.solve(R, C4[b], opts=oo)
        its = [p[4] for p in ir.phases]
        its = tuple(its + [0] * (3 - len(its)))
        print(f"b={b}: batch {infos[b].status} restarts {infos[b].restarts} "
              f"{infos[b].phase_iterations}; oracle {ir.status} "
              f"{ir.restarts} {its}", flush=True)
        assert infos[b].restarts == ir.restarts
        assert infos[b].phase_iterations == its
        assert infos[b].projected_steps == ir.projected_steps
        assert infos[b].status == ir.status
        assert np.abs(W[b].cpu().numpy() - xr).max() <= 1e-9
    assert any(i.restarts >= 1 for i in infos)
    ctx.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_frontier_pcg_reduced_storage(prec):
    """FP32/BF16 storage: the lanes run on separate streams (their trace
    products are on the storage precision's matrix cores) with the single
    solve's kernels, so each instance equals its single solve, and converges
    to a stationary point of the rounded problem judged by the oracle."""
    from storage import round_storage
    print(f"[case] frontier PCG {prec} n=300 T=1000", flush=True)
    R = synth.factor_returns(300, 1000, 5, 0, 5.0, 0.0, 7)
    mu, A = O.center(R)
    Ar = round_storage(A, prec)
    C4, tg = _frontier_instances(R, 2)
    ctx = yb.Context(torch.from_numpy(R).cuda(), prec)
    opts = yb.default_opts(large=True)
    W, infos = ctx.frontier(C4, tg, opts=opts)
    for b in range(len(C4)):
        w1, i1 = ctx.solve(C4[b], target=tg[b], opts=opts)
        wb = W[b].cpu().numpy()
        assert infos[b].status == 0 and infos[b].iterations == i1.iterations
        assert infos[b].cg_iters == i1.cg_iters
        assert np.abs(wb - w1.cpu().numpy()).max() <= 1e-12
        Cm, _ = O.constraints(mu, tg[b])
        U = O.tangent_basis(Cm)
        assert np.linalg.norm(U.T @ O.gradient(Ar, mu, C4[b], wb)) <= 2e-8
    ctx.close()
