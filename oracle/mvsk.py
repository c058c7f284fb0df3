"""FP64 CPU oracle of YAND-MVSK (test infrastructure only; see package doc).

Every function cites the passage of the paper it follows.  Section numbers
follow the paper: Section 2 (problem setting), Section 4 (solver, with
Algorithm 1 "YAND-MVSK algorithm"), Section 5 (Proposition "Exact operator
representation", Proposition "Quartic exact line search from sample power
sums", Proposition "Affine-subspace reduction"), Appendix B (Lemma
"Interior-safe steplength cap", Proposition "A sufficient condition for the
imported bounded-direction hypothesis"), Appendix D (Table "YAND-MVSK parameter
settings").

Readings of passages the paper leaves open are listed in the design notes of
the repository (exact log-det correction, 1/(m+1) factor, relative
regularisation, PCG preconditioner, stall rule, tie rule).  The parity status
of each function:

* centering, objective, moments, gradient, HVP, third-order action,
  line-search coefficients, step selection, feasibility cap, reduced basis,
  affine-normal direction, solve loop: pinned (tests/test_oracle_pins.py).
* simplex projection, projected-KKT residual, boundary block with its face
  solver, Armijo rule: pinned (tests/test_oracle_simplex.py).
* stall test and the stall-recovery restarts: pinned
  (tests/test_oracle_stall.py).
* probe estimate of the trace (counter-based signs, block PCG): pinned
  (tests/test_oracle_probe.py).
* return-floor protocol: pinned (tests/test_oracle_floor.py).
* PCG inner iterates: parity unpinned per iteration (the paper does not name
  its preconditioner); pinned only at solve level through uniqueness of the
  minimiser under the convexity certificate.
"""

from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

__all__ = [
    "center", "psi", "dpsi", "d2psi", "d3psi", "objective", "moments",
    "gradient", "hvp", "third", "constraints", "feasible_start",
    "tangent_basis", "householder_frame", "Direction", "affine_normal",
    "linesearch_coeffs", "alpha_max", "quartic_value", "select_step",
    "Options", "SolveInfo", "solve", "certified_convex", "Unbounded",
    "Indefinite", "project_simplex", "kkt_residual", "face_free",
    "face_basis", "armijo_step", "return_floor", "splitmix64", "rademacher",
]


class Unbounded(ArithmeticError):
    """The quartic line model has no minimiser on [0, alpha_max)."""


class Indefinite(ArithmeticError):
    """The regularised tangent Hessian stayed indefinite after escalation."""


# ---------------------------------------------------------------------------
# Section 2: sample mean, centered returns, moments.
# ---------------------------------------------------------------------------

def center(R: np.ndarray):
    """mu = T^-1 R^T 1 and A = R - 1 mu^T (Section 2; Algorithm 1, setup)."""
    R = np.asarray(R, dtype=np.float64)
    T = R.shape[0]
    mu = R.sum(axis=0) / T
    A = R - mu[None, :]
    return mu, A


def psi(c, s):
    """psi(s) = c2 s^2 - c3 s^3 + c4 s^4 (Section 2, lifted form)."""
    return c[1] * s**2 - c[2] * s**3 + c[3] * s**4


def dpsi(c, s):
    return 2.0 * c[1] * s - 3.0 * c[2] * s**2 + 4.0 * c[3] * s**3


def d2psi(c, s):
    """psi''(s) = 2c2 - 6c3 s + 12c4 s^2 (Proposition 'Lifted separability')."""
    return 2.0 * c[1] - 6.0 * c[2] * s + 12.0 * c[3] * s**2


def d3psi(c, s):
    return -6.0 * c[2] + 24.0 * c[3] * s


def moments(A, mu, x):
    """m1 = mu^T x and m_p = T^-1 sum_t (a_t^T x)^p, p = 2,3,4 (Section 2)."""
    z = A @ x
    T = A.shape[0]
    return np.array([mu @ x, np.sum(z**2) / T, np.sum(z**3) / T,
                     np.sum(z**4) / T])


def objective(A, mu, c, x):
    """f(x) = -c1 mu^T x + (c2 |z|^2 - c3 sum z^3 + c4 sum z^4)/T, z = Ax.

    Proposition 'Exact operator representation', equation (operator-f).
    """
    T = A.shape[0]
    z = A @ x
    return (-c[0] * (mu @ x) + c[1] / T * np.sum(z**2)
            - c[2] / T * np.sum(z**3) + c[3] / T * np.sum(z**4))


def gradient(A, mu, c, x):
    """Equation (operator-grad): -c1 mu + A^T(2c2 z - 3c3 z^2 + 4c4 z^3)/T."""
    T = A.shape[0]
    z = A @ x
    return (-c[0] * mu + 2.0 * c[1] / T * (A.T @ z)
            - 3.0 * c[2] / T * (A.T @ z**2) + 4.0 * c[3] / T * (A.T @ z**3))


def hvp(A, c, x, v):
    """Equation (operator-hvp): Hessian of f at x applied to v."""
    T = A.shape[0]
    z = A @ x
    Av = A @ v
    return (2.0 * c[1] / T * (A.T @ Av) - 6.0 * c[2] / T * (A.T @ (z * Av))
            + 12.0 * c[3] / T * (A.T @ (z**2 * Av)))


def third(A, c, x, u, v):
    """Equation (operator-third): D^3 f(x)[u, v, .]."""
    T = A.shape[0]
    z = A @ x
    Au = A @ u
    Av = A @ v
    return (-6.0 * c[2] / T * (A.T @ (Au * Av))
            + 24.0 * c[3] / T * (A.T @ (z * Au * Av)))


def certified_convex(c) -> bool:
    """Corollary 'coefficient-only convexity certificate': c4 > 0, 8c2c4 > 3c3^2."""
    return bool(c[3] > 0.0 and 8.0 * c[1] * c[3] > 3.0 * c[2] ** 2)


# ---------------------------------------------------------------------------
# Section 4.2 / Proposition 'Affine-subspace reduction': reduced coordinates.
# ---------------------------------------------------------------------------

def constraints(mu, target=None):
    """Equality constraints C^T x = b.

    Budget only: C = [1], b = [1] (the simplex tangent space of Section 4.2).
    With a return target r: C = [1, mu], b = [1, r]; the affine-subspace
    reduction applies unchanged with the smaller tangent space null(C^T).
    """
    n = mu.shape[0]
    if target is None:
        return np.ones((n, 1)), np.array([1.0])
    return np.stack([np.ones(n), mu], axis=1), np.array([1.0, float(target)])


def feasible_start(C, b, x=None):
    """Equal weights (Algorithm 1 input; Section 6.1), moved by the
    minimum-norm correction onto C^T x = b when a target is present."""
    n = C.shape[0]
    x = np.full(n, 1.0 / n) if x is None else np.array(x, dtype=np.float64)
    r = C.T @ x - b
    return x - C @ np.linalg.solve(C.T @ C, r)


def tangent_basis(C):
    """Orthonormal U spanning null(C^T) (Section 4.2), from a complete QR."""
    p = C.shape[1]
    Qc, _ = np.linalg.qr(C, mode="complete")
    return np.ascontiguousarray(Qc[:, p:])


def householder_frame(nu):
    """Householder frame Q with Q^T Q = I and Q^T nu = 0 (Section 4.2).

    The reflector I - 2 v v^T / v^T v with v = nu + sign(nu_1) e_1 maps e_1 to
    a multiple of nu; its remaining columns span the orthogonal complement.
    """
    m = nu.shape[0]
    v = nu.copy()
    s = 1.0 if nu[0] >= 0.0 else -1.0
    v[0] += s * np.linalg.norm(nu)
    Hh = np.eye(m) - 2.0 * np.outer(v, v) / (v @ v)
    return np.ascontiguousarray(Hh[:, 1:])


# ---------------------------------------------------------------------------
# Section 4.2 / 4.4: the affine-normal direction with the exact trace.
# ---------------------------------------------------------------------------

@dataclass
class Direction:
    d: np.ndarray            # ambient direction d = U d_y
    gnorm: float             # ||gbar||
    lam: float               # regularisation used in H_{T,lambda}
    a: np.ndarray            # log-det correction (reduced, length m-1)
    u: np.ndarray            # tangential coefficients
    cg_iters: int = 0
    q: np.ndarray | None = None   # q_t (exact, or the probe estimate)
    probe_iters: int = 0          # CG iterations of the probe solves


# ---------------------------------------------------------------------------
# Counter-based random signs for the probe estimate of the trace.
# ---------------------------------------------------------------------------

_SM_GAMMA = 0x9E3779B97F4A7C15
_SM_M1 = 0xBF58476D1CE4E5B9
_SM_M2 = 0x94D049BB133111EB


def splitmix64(state):
    """Output of the SplitMix64 generator (Steele, Lea and Flood, 2014) for
    Weyl states ``state`` (uint64 array): the state advanced by the golden
    gamma and passed through the variant-13 finaliser."""
    z = np.asarray(state, dtype=np.uint64) + np.uint64(_SM_GAMMA)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(_SM_M1)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(_SM_M2)
    return z ^ (z >> np.uint64(31))


def rademacher(seed, draw, T, k):
    """T x k matrix of independent signs xi_tj = +-1 for the draw-th probe
    block of a solve: the sign bit of SplitMix64 at the counter
    seed + gamma * (draw 2^42 + t 2^10 + j), t < 2^32, j < 2^10."""
    if not (0 < k <= 1024 and T < (1 << 32) and 0 <= draw < (1 << 22)):
        raise ValueError("probe counter out of range")
    t = np.arange(T, dtype=np.uint64)[:, None]
    j = np.arange(k, dtype=np.uint64)[None, :]
    ctr = (np.uint64(draw) << np.uint64(42)) | (t << np.uint64(10)) | j
    with np.errstate(over="ignore"):
        st = np.uint64(seed) + ctr * np.uint64(_SM_GAMMA)
        bits = splitmix64(st) >> np.uint64(63)
    return 1.0 - 2.0 * bits.astype(np.float64)


def _pcg(Bmat, rhs, tol, maxit, precond):
    """Preconditioned CG on the reduced tangent system, start 0.

    Reading of the 'pcg reduced solve' of Table 'YAND-MVSK parameter
    settings' (the paper names no preconditioner): stop when
    ||r_k|| <= tol ||r_0|| or after maxit iterations.  precond(r) applies
    the preconditioner's inverse.
    """
    u = np.zeros_like(rhs)
    r = rhs.copy()
    r0 = np.linalg.norm(r)
    if r0 == 0.0:
        return u, 0
    zv = precond(r)
    p = zv.copy()
    rz = r @ zv
    it = 0
    while it < maxit:
        Bp = Bmat @ p
        pBp = p @ Bp
        it += 1
        if not pBp > 0.0:
            # a direction of non-positive curvature ends the iteration
            # without a step along it (truncated CG, Steihaug 1983)
            break
        alpha = rz / pBp
        u += alpha * p
        r -= alpha * Bp
        if np.linalg.norm(r) <= tol * r0:
            break
        zv = precond(r)
        rz_new = r @ zv
        p = zv + (rz_new / rz) * p
        rz = rz_new
    return u, it


def affine_normal(A, mu, c, x, U, *, solver="direct", reg=0.0,
                  krylov_tol=1e-3, krylov_maxit=15, max_escalations=16,
                  trace="exact", probes=64, seed=0, draw=0):
    """Exact-trace affine-normal direction in reduced coordinates.

    Section 4.2 and Section 4.4: with gbar = U^T g, nu = gbar/|gbar|, the
    Householder frame Q, H_red = U^T H U,
        h = Q^T H_red nu,   H_{T,lam} = Q^T H_red Q + lam I,
        u = H_{T,lam}^{-1} (h - |gbar|/(m+1) a),   d_y = Q u - nu,  d = U d_y,
    with m = dim of the reduced space (the form of Appendix B, Proposition
    'A sufficient condition for the imported bounded-direction hypothesis').

    The exact log-det correction is
        a_l = sum_ij (H_{T,lam}^{-1})_ij D^3 phi[Q e_i, Q e_j, Q e_l],
    the derivative of log det Q^T H_red(y + Q eta) Q at eta = 0; with P = A U Q
    and q_t = p_t^T H_{T,lam}^{-1} p_t it equals P^T (psi'''(z) * q) / T.

    ``reg`` is relative: lam = reg * trace(Q^T H_red Q) / (m - 1).  The direct
    solver starts at reg (0 by default) and escalates lam on a failed Cholesky
    factorisation; the PCG solver keeps the factorisation only for the exact
    trace and solves for u by ``_pcg``, preconditioned by the Jacobi inverse
    of the ambient Hessian diagonal (plus lam) restricted to the reduced
    space.

    trace = "probe" (PCG solver only) replaces the exact q by Hutchinson's
    estimate of the diagonal of P H_{T,lam}^{-1} P^T (Appendix C, the
    Krylov reduced solve): with the T x k sign matrix Xi = rademacher(seed,
    draw, T, k), y_j solves H_{T,lam} y_j = P^T xi_j by the same PCG
    (tolerance, budget, preconditioner) and q_t = k^-1 sum_j xi_tj (P y_j)_t.
    No factorisation is formed.
    """
    T = A.shape[0]
    m = U.shape[1]
    z = A @ x
    g = gradient(A, mu, c, x)
    gbar = U.T @ g
    gn = float(np.linalg.norm(gbar))
    nu = gbar / gn
    if m == 1:
        d = U @ (-nu)
        return Direction(d=d, gnorm=gn, lam=0.0, a=np.zeros(0), u=np.zeros(0))
    Q = householder_frame(nu)
    V = U @ Q
    P = A @ V
    D2 = d2psi(c, z)
    B0 = P.T @ (D2[:, None] * P) / T
    scale = np.trace(B0) / (m - 1)
    lam = reg * scale
    if trace == "probe":
        if solver != "pcg":
            raise ValueError("the probe trace needs the PCG solver")
        Bm = B0 + lam * np.eye(m - 1)
        dj = np.sum(A * A * (D2 / T)[:, None], axis=0) + lam
        dj = np.where(dj > 0.0, dj, 1.0)
        prec = lambda r: V.T @ ((V @ r) / dj)  # noqa: E731
        Xi = rademacher(seed, draw, T, probes)
        Yp = np.empty((m - 1, probes))
        pit = 0
        for j in range(probes):
            Yp[:, j], it_j = _pcg(Bm, P.T @ Xi[:, j], krylov_tol,
                                  krylov_maxit, prec)
            pit += it_j
        q = np.mean(Xi * (P @ Yp), axis=1)
        a = P.T @ (d3psi(c, z) * q) / T
        h = V.T @ hvp(A, c, x, U @ nu)
        rhs = h - gn / (m + 1) * a
        u, cg_iters = _pcg(Bm, rhs, krylov_tol, krylov_maxit, prec)
        dy = Q @ u - nu
        return Direction(d=U @ dy, gnorm=gn, lam=lam, a=a, u=u,
                         cg_iters=cg_iters, q=q, probe_iters=pit)
    elif trace != "exact":
        raise ValueError(trace)
    for _ in range(max_escalations + 1):
        Bm = B0 + lam * np.eye(m - 1)
        try:
            L = np.linalg.cholesky(Bm)
            break
        except np.linalg.LinAlgError:
            lam = max(10.0 * lam, 1e-12 * scale)
    else:
        raise Indefinite("tangent Hessian indefinite after escalation")
    h = V.T @ hvp(A, c, x, U @ nu)
    Y = sla.solve_triangular(L, P.T, lower=True)       # (m-1) x T
    q = np.sum(Y * Y, axis=0)
    a = P.T @ (d3psi(c, z) * q) / T
    rhs = h - gn / (m + 1) * a
    cg_iters = 0
    if solver == "direct":
        u = sla.cho_solve((L, True), rhs)
    elif solver == "pcg":
        # Jacobi on the ambient Hessian diagonal, restricted to the reduced
        # space: V^T diag(A^T diag(psi''/T) A + lam)^-1 V
        dj = np.sum(A * A * (D2 / T)[:, None], axis=0) + lam
        dj = np.where(dj > 0.0, dj, 1.0)
        u, cg_iters = _pcg(Bm, rhs, krylov_tol, krylov_maxit,
                           lambda r: V.T @ ((V @ r) / dj))
    else:
        raise ValueError(solver)
    dy = Q @ u - nu
    return Direction(d=U @ dy, gnorm=gn, lam=lam, a=a, u=u, cg_iters=cg_iters,
                     q=q)


# ---------------------------------------------------------------------------
# Proposition 'Quartic exact line search from sample power sums'.
# ---------------------------------------------------------------------------

def linesearch_coeffs(A, mu, c, x, d):
    """A0..A4 of f(x + alpha d) from s_rs = T^-1 sum_t z_t^r w_t^s."""
    T = A.shape[0]
    z = A @ x
    w = A @ d

    def s(r, k):
        return np.sum(z**r * w**k) / T

    A0 = objective(A, mu, c, x)
    A1 = (-c[0] * (mu @ d) + 2.0 * c[1] * s(1, 1) - 3.0 * c[2] * s(2, 1)
          + 4.0 * c[3] * s(3, 1))
    A2 = c[1] * s(0, 2) - 3.0 * c[2] * s(1, 2) + 6.0 * c[3] * s(2, 2)
    A3 = -c[2] * s(0, 3) + 4.0 * c[3] * s(1, 3)
    A4 = c[3] * s(0, 4)
    return np.array([A0, A1, A2, A3, A4])


def alpha_max(x, d, tau):
    """Lemma 'Interior-safe steplength cap': min over d_i < 0 of (x_i-tau)/(-d_i)."""
    neg = d < 0.0
    if not np.any(neg):
        return math.inf
    return float(np.min((x[neg] - tau) / (-d[neg])))


def project_simplex(y, tau=0.0):
    """Euclidean projection onto Delta(tau) = {x : x_i >= tau, 1^T x = 1},
    the projection of the projected trial step (reduced-simplex wrapper of
    the implementation appendix).  Shifted by tau it is the projection onto
    the simplex of mass s = 1 - n tau, done by the sorting method (Held,
    Wolfe and Crowder 1974; Duchi et al. 2008): with u = y - tau sorted
    decreasingly, rho is the last j with u_(j) > (sum_{i<=j} u_(i) - s) / j,
    theta = (sum_{i<=rho} u_(i) - s) / rho and x = max(u - theta, 0) + tau.
    """
    y = np.asarray(y, dtype=np.float64)
    n = y.size
    s = 1.0 - n * tau
    if not s > 0.0:
        raise ValueError("tau must be below 1/n")
    u = y - tau
    v = np.sort(u)[::-1]
    cs = np.cumsum(v)
    j = np.arange(1, n + 1)
    rho = int(j[v - (cs - s) / j > 0.0][-1])
    # theta from a correctly rounded sum over the support (the running sum
    # above only locates rho)
    theta = (math.fsum(v[:rho]) - s) / rho
    return np.maximum(u - theta, 0.0) + tau


def kkt_residual(A, mu, c, x, tau=0.0):
    """Projected-simplex KKT residual |x - Pi_Delta(tau)(x - grad f(x))|_2.

    The computational study evaluates solutions by a projected-simplex KKT
    residual against a 1e-6 target without stating its formula; this is the
    standard projected-gradient residual on the slice Delta(tau) the solver
    works on.  It vanishes exactly at the KKT points of min f over
    Delta(tau) and equals the tangent-gradient norm |P_1 grad f| at interior
    points where the unit projected-gradient step stays inside.  (Against
    Delta(0) a KKT point of Delta(tau) with n_b coordinates on the bound
    keeps the floor tau sqrt(n_b^2 / (n - n_b) + n_b): the bound coordinates
    drop to 0 and their mass n_b tau spreads over the free ones.)
    """
    g = gradient(A, mu, c, x)
    return float(np.linalg.norm(x - project_simplex(x - g, tau)))


def face_free(x, g, tau, hold=None):
    """Free coordinates of the current face of Delta(tau) (boundary block of
    Algorithm 1: continuation on the exposed active face).  Coordinates
    above the slice bound, x_i > tau (1 + 1e-6), are free; a bound
    coordinate is released when its multiplier g_i - nu is negative, with nu
    the mean of g over the coordinates above the bound (the budget
    multiplier of the face problem), unless the face solver holds it at the
    bound (hold, see _iterate)."""
    strict = x > tau * (1.0 + 1e-6)
    nu = float(np.sum(g[strict])) / int(np.count_nonzero(strict))
    release = g < nu
    if hold is not None:
        release &= ~hold
    return strict | release


def face_basis(free):
    """Orthonormal basis of the face's tangent space {d : d_i = 0 off the
    free set, sum_i d_i = 0}: the budget tangent basis of the free
    coordinates, zero on the bound ones."""
    n, k = free.size, int(np.count_nonzero(free))
    U = np.zeros((n, k - 1))
    if k > 1:
        U[free] = tangent_basis(np.ones((k, 1)))
    return U


def quartic_value(coef, alpha):
    return (coef[0] + coef[1] * alpha + coef[2] * alpha**2
            + coef[3] * alpha**3 + coef[4] * alpha**4)


def select_step(coef, amax=math.inf):
    """Exact step: argmin of the quartic over {0, amax} and the real roots of
    its derivative inside (0, amax) (Proposition 'Quartic exact line search').

    Roots come from the companion-matrix eigenvalues (numpy.roots).  The
    candidates are compared on phi(alpha) - A0 = A1 a + A2 a^2 + A3 a^3 + A4 a^4
    so that decreases far below the rounding of A0 still count.  Ties are
    broken toward the smallest step among candidates within
    1e-15 * sum_{i>=1} |A_i| alpha^i of the minimum.  A constant model (A1..A4
    all zero: a zero direction) gives 0.  On an unbounded interval the quartic
    must grow at infinity (leading nonzero coefficient positive), otherwise
    ``Unbounded`` is raised.
    """
    coef = np.asarray(coef, dtype=np.float64)
    if not np.any(coef[1:] != 0.0):
        return 0.0          # a constant model (zero direction): stay put
    if not math.isfinite(amax):
        lead = next((coef[i] for i in (4, 3, 2, 1) if coef[i] != 0.0), 0.0)
        if lead <= 0.0:
            raise Unbounded("line model unbounded below on [0, inf)")
    dcoef = [4.0 * coef[4], 3.0 * coef[3], 2.0 * coef[2], coef[1]]
    cands = [0.0]
    if math.isfinite(amax):
        cands.append(float(amax))
    nz = np.trim_zeros(np.array(dcoef), "f")
    if nz.size > 1:
        for r in np.roots(nz):
            if abs(r.imag) <= 1e-8 * max(1.0, abs(r.real)):
                a = float(r.real)
                if 0.0 < a < amax:
                    cands.append(a)
    cands = np.array(sorted(set(cands)))
    pw = cands[:, None] ** np.arange(1, 5)[None, :]
    vals = pw @ coef[1:]
    scale = pw @ np.abs(coef[1:])
    ok = vals <= vals.min() + 1e-15 * scale
    return float(cands[np.argmax(ok)])


def armijo_step(coef, amax=math.inf, sigma=1e-4, rho=0.5, max_halvings=60):
    """Armijo backtracking on the quartic line model (the line-search rule of
    the convergence theory and of the Armijo diagnostic of Table 'YAND-MVSK
    parameter settings'): from alpha = min(1, amax), halve until
    phi(alpha) - phi(0) <= sigma alpha phi'(0), phi'(0) = A1.  The model is
    exact, so each trial costs no pass over A.  The paper fixes only
    sigma in (0, 1); sigma = 1e-4, rho = 1/2 and 60 halvings (then 0) are
    readings."""
    A1, A2, A3, A4 = (float(v) for v in coef[1:5])
    a = min(1.0, amax)
    for _ in range(max_halvings):
        dec = a * (A1 + a * (A2 + a * (A3 + a * A4)))
        if dec <= sigma * a * A1:
            return a
        a *= rho
    return 0.0


# ---------------------------------------------------------------------------
# Algorithm 1: the outer loop.
# ---------------------------------------------------------------------------

@dataclass
class Options:
    """Parameters of Table 'YAND-MVSK parameter settings' plus readings.

    solver: 'direct' (YAND-MVSK small) or 'pcg' (YAND-MVSK large).
    feasible_set: 'budget' (affine hull, no cap) or 'simplex' (cap on
    Delta(tau), Lemma 'Interior-safe steplength cap').
    eta: nominal projected trial step of the boundary block (0.05 in Table
    'YAND-MVSK parameter settings'); 0 keeps the capped raw step only.
    linesearch: 'exact' (quartic exact rule) or 'armijo' (armijo_step).
    trace: 'exact' or 'probe' (PCG phases only: Hutchinson's estimate of q
    from ``probes`` random sign vectors per direction, drawn from
    rademacher(probe_seed, direction index of the solve, ...)).
    """
    solver: str = "direct"
    feasible_set: str = "budget"
    eps: float = 1e-8
    max_iter: int = 300
    max_elapsed: float = math.inf
    reg: float = 0.0
    krylov_tol: float = 1e-3
    krylov_maxit: int = 15
    tau: float = 1e-8
    eta: float = 0.05
    linesearch: str = "exact"
    stall_recovery: bool = True
    restart_max_iter: int = 120
    trace: str = "exact"
    probes: int = 64
    probe_seed: int = 0

    @staticmethod
    def large():
        """YAND-MVSK (large): PCG, 40 iterations, 60 s, reg 1e-4."""
        return Options(solver="pcg", max_iter=40, max_elapsed=60.0, reg=1e-4)


@dataclass
class SolveInfo:
    iterations: int = 0
    restarts: int = 0
    f: float = math.nan
    gnorm: float = math.nan
    status: int = 0
    cg_iters: int = 0
    oracle_passes: int = 0
    ls_passes: int = 0
    kkt: float = math.nan
    projected_steps: int = 0
    history: list = field(default_factory=list)
    phases: list = field(default_factory=list)
    directions: int = 0
    probe_iters: int = 0


# A projected segment whose line search moves less than this fraction of it
# is no usable descent step (reading of the reduced-simplex wrapper).
SEGMENT_USABLE = 0.1


def _iterate(A, mu, c, x, U, opts: Options, solver, krylov_maxit, max_iter,
             info: SolveInfo, t0, eta=None):
    """Run outer iterations from x; return (x, converged, reason).

    reason: 'converged'; 'stall' when the objective decreased by less than
    1e-14 of its magnitude on 3 iterations in a row; 'budget' when max_iter
    iterations ran; 'time' when max_elapsed (seconds, > 0) ran out.

    Simplex with eta > 0 runs the boundary block of Algorithm 1 and the
    reduced-simplex wrapper of the implementation appendix:
      * the direction lives on the current face (face_free, face_basis), so
        coordinates at the slice bound stay there unless released;
      * when the cap alpha_max(x, d; tau) is below the nominal step eta, the
        trial x + eta d is projected onto Delta(tau) and the line search runs
        on the corrected segment x + a (xbar - x), a in [0, 1], provided
        that segment is a descent direction and not numerically zero;
        otherwise the capped raw step is taken, which exposes the next face;
      * the corrected segment is used only when it gives a usable step: its
        own line search (same rule, over [0, 1]) must reach at least
        SEGMENT_USABLE of the segment;
      * otherwise (no descent along the segment, or no usable step on it)
        control passes to the face solver: the released coordinates at the
        bound that the direction drives further down, and the coordinates
        that stop the raw step at alpha_max, are held at the bound, and the
        capped raw step is taken; the following iterations run on that
        lower-dimensional face; the holds are dropped once the held face is
        stationary (|reduced gradient| <= eps), which then counts as
        convergence only without holds; an iteration that adds holds does
        not count toward the stall test;
      * the stopping test also accepts a projected-KKT residual
        (kkt_residual on Delta(tau)) at or below eps.
    With eta = 0 the simplex set only caps the raw step.
    """
    eta = opts.eta if eta is None else eta
    simplex = opts.feasible_set == "simplex"
    faces = simplex and eta > 0.0
    small = 0
    reason = "budget"
    f_prev = objective(A, mu, c, x)
    hold = np.zeros(x.size, dtype=bool)
    release = False
    thr = opts.tau * (1.0 + 1e-6)
    for _ in range(max_iter):
        g = gradient(A, mu, c, x)
        info.oracle_passes += 1
        if release:
            hold[:] = False
            release = False
        free = face_free(x, g, opts.tau, hold) if faces else None
        Ui = face_basis(free) if faces else U
        gn = float(np.linalg.norm(Ui.T @ g))
        info.gnorm = gn
        if simplex:
            info.kkt = float(np.linalg.norm(
                x - project_simplex(x - g, opts.tau)))
        if simplex and info.kkt <= opts.eps:
            return x, True, "converged"
        if gn <= opts.eps:
            if not hold.any():
                return x, True, "converged"
            release = True
        if opts.max_elapsed > 0.0 and time.perf_counter() - t0 > opts.max_elapsed:
            return x, False, "time"
        reg = opts.reg if solver == "pcg" else 0.0
        dr = affine_normal(A, mu, c, x, Ui, solver=solver, reg=reg,
                           krylov_tol=opts.krylov_tol,
                           krylov_maxit=krylov_maxit,
                           trace=opts.trace if solver == "pcg" else "exact",
                           probes=opts.probes, seed=opts.probe_seed,
                           draw=info.directions)
        info.directions += 1
        info.cg_iters += dr.cg_iters
        info.probe_iters += dr.probe_iters
        d = dr.d
        amax = alpha_max(x, d, opts.tau) if simplex else math.inf
        rule = armijo_step if opts.linesearch == "armijo" else select_step
        held = int(np.count_nonzero(hold))
        coef = None
        if faces and amax < eta:
            dbar = project_simplex(x + eta * d, opts.tau) - x
            if (np.max(np.abs(dbar)) > 1e-15 * np.max(np.abs(x))
                    and float(g @ dbar) < 0.0):
                cs = linesearch_coeffs(A, mu, c, x, dbar)
                info.ls_passes += 1
                a_s = rule(cs, 1.0)
                if a_s >= SEGMENT_USABLE:
                    d, amax, coef, alpha = dbar, 1.0, cs, a_s
                    info.projected_steps += 1
            if coef is None:
                # face solver: released bound coordinates that d drives
                # further down, and the coordinates that stop the raw step
                # (they reach the bound at alpha_max), are held at the bound
                neg = d < 0.0
                cap = np.full(x.size, np.inf)
                cap[neg] = (x[neg] - opts.tau) / (-d[neg])
                hold |= free & neg & ((x <= thr) | (cap <= amax * (1.0 + 1e-12)))
        if coef is None:
            coef = linesearch_coeffs(A, mu, c, x, d)
            info.ls_passes += 1
            alpha = rule(coef, amax)
        x = x + alpha * d
        info.iterations += 1
        f_new = quartic_value(coef, alpha)
        info.history.append((gn, alpha, f_new))
        # a step that changes the face (new holds) is progress of the face
        # solver even when it moves no weight
        if (f_prev - f_new < 1e-14 * abs(f_prev)
                and int(np.count_nonzero(hold)) == held):
            small += 1
            if small >= 3:
                reason = "stall"
                break
        else:
            small = 0
        f_prev = f_new
    # budget spent or stalled: the reported state is that of the returned x
    g = gradient(A, mu, c, x)
    Ui = face_basis(face_free(x, g, opts.tau)) if faces else U
    info.gnorm = float(np.linalg.norm(Ui.T @ g))
    conv = info.gnorm <= opts.eps
    if simplex:
        info.kkt = float(np.linalg.norm(x - project_simplex(x - g, opts.tau)))
        conv = conv or info.kkt <= opts.eps
    return x, conv, "converged" if conv else reason


def solve(R, c, target=None, x0=None, opts: Options | None = None,
          centered=None):
    """Algorithm 1 (YAND-MVSK) in FP64 with explicit reduced bases.

    Stall recovery (reading of the 'stall-recovery restarts' of Table
    'YAND-MVSK parameter settings'): when the baseline budget ends above
    eps, or the objective stops decreasing for 3 iterations, restart from
    the current iterate with restart_max_iter iterations.  Budget set: first
    with twice the Krylov budget, then with the direct solve.  Simplex: with
    the projected trial steps 0.045, then 0.02, of the same table.  The
    boundary block needs the budget hull alone; with a return target it is
    off (capped steps only).  max_elapsed <= 0 means no time limit.
    Status: 0 converged; 2 stalled (the last phase ended at the stall test,
    or restarts ran and the solve is still above eps); 1 the iteration or
    time budget ended above eps without a restart.
    info.phases lists each phase as (solver, krylov_maxit, max_iter, eta,
    iterations, reason).
    centered: an optional (mu, A) used in place of center(R), for instance A
    rounded to a storage precision (the problem such a store defines).
    """
    opts = opts or Options()
    c = np.asarray(c, dtype=np.float64)
    mu, A = center(R) if centered is None else centered
    C, b = constraints(mu, target)
    x = feasible_start(C, b, x0)
    if opts.feasible_set == "simplex" and np.any(x < opts.tau):
        raise ValueError("start outside the interior slice")
    U = tangent_basis(C)
    info = SolveInfo()
    eta = opts.eta if target is None else 0.0
    t0 = time.perf_counter()
    it0 = info.iterations
    x, conv, reason = _iterate(A, mu, c, x, U, opts, opts.solver,
                               opts.krylov_maxit, opts.max_iter, info, t0,
                               eta)
    info.phases.append((opts.solver, opts.krylov_maxit, opts.max_iter, eta,
                        info.iterations - it0, reason))
    if not conv and opts.stall_recovery and opts.solver == "pcg":
        if opts.feasible_set == "simplex" and eta > 0.0:
            plan = [("pcg", opts.krylov_maxit, 0.045),
                    ("pcg", opts.krylov_maxit, 0.02)]
        else:
            plan = [("pcg", 2 * opts.krylov_maxit, eta), ("direct", 0, eta)]
        for solver, kmax, e in plan:
            info.restarts += 1
            t0 = time.perf_counter()
            it0 = info.iterations
            x, conv, reason = _iterate(A, mu, c, x, U, opts, solver, kmax,
                                       opts.restart_max_iter, info, t0, e)
            info.phases.append((solver, kmax, opts.restart_max_iter, e,
                                info.iterations - it0, reason))
            if conv:
                break
    info.f = objective(A, mu, c, x)
    if conv:
        info.status = 0
    elif info.restarts > 0 or reason == "stall":
        info.status = 2
    else:
        info.status = 1
    return x, info


# ---------------------------------------------------------------------------
# Section 7: the return-floor protocol of the economic comparison.
# ---------------------------------------------------------------------------

@dataclass
class FloorResult:
    c: np.ndarray
    x: np.ndarray
    ret: float
    floor: float
    solves: int
    info: SolveInfo


def return_floor(R, profile, q, opts: Options | None = None, max_rounds=40):
    """The return-floor protocol of the real-data comparison (Section
    'Computational Study', real-data experiment): the moment coefficients are
    normalised by the equal-weight portfolio's moment magnitudes,
    c_k = p_k / |m_k(1/n)| for k = 2, 3, 4 with profile = (p2, p3, p4), and
    the mean coefficient c1 is calibrated so that the long-only MVSK
    portfolio's in-sample mean return mu^T x lies as close as possible to the
    floor, the q-th percentile of the asset means (linear interpolation
    between order statistics).

    The root-find over solves is a reading (the paper gives none).  It leans
    on the mean return of the minimiser being nondecreasing in c1 (true when
    f is convex: compare the optimality of the two minimisers).  c1 = 0 first
    (kept when it already meets the floor, or when all asset means are
    equal; negative c1 would reward a lower mean); then
    c1 = 1 / (max mu - min mu), growing by factors of 4 until the floor is
    met; then geometric bisection of the bracket (its midpoint is
    c_hi / 2 while the lower end is 0), at most max_rounds rounds each,
    stopping once |mu^T x - floor| <= 1e-9 (max mu - min mu).  Every solve
    starts from equal weights.  The closest solve is returned (ties to the
    larger c1).  A solve's error (an indefinite tangent Hessian outside the
    convexity certificate) ends the protocol with that error."""
    opts = opts or Options(feasible_set="simplex")
    p2, p3, p4 = (float(v) for v in profile)
    mu, A = center(R)
    n = mu.size
    m = moments(A, mu, np.full(n, 1.0 / n))
    base = np.zeros(4)
    for k, p in ((1, p2), (2, p3), (3, p4)):
        if p != 0.0:
            if m[k] == 0.0:
                raise ValueError("profile weight on a vanishing moment")
            base[k] = p / abs(m[k])
    floor = float(np.quantile(mu, q))
    spread = float(mu.max() - mu.min())
    tol = 1e-9 * spread
    solves = 0

    def run(c1):
        nonlocal solves
        c = base.copy()
        c[0] = c1
        x, info = solve(R, c, opts=opts)
        solves += 1
        return float(mu @ x), x, info, c

    best = None

    def keep(r):
        nonlocal best
        if best is None or abs(r[0] - floor) < abs(best[0] - floor) or (
                abs(r[0] - floor) == abs(best[0] - floor) and r[3][0] > best[3][0]):
            best = r

    lo = run(0.0)
    keep(lo)
    if lo[0] < floor and spread > 0.0:
        hi = run(1.0 / spread)
        keep(hi)
        k = 0
        while hi[0] < floor and k < max_rounds:
            lo = hi
            hi = run(4.0 * hi[3][0])
            keep(hi)
            k += 1
        k = 0
        while hi[0] >= floor and abs(best[0] - floor) > tol and k < max_rounds:
            c_lo, c_hi = lo[3][0], hi[3][0]
            mid = run(0.5 * c_hi if c_lo == 0.0 else math.sqrt(c_lo * c_hi))
            keep(mid)
            if mid[0] >= floor:
                hi = mid
            else:
                lo = mid
            k += 1
    r, x, info, c = best
    return FloorResult(c=c, x=x, ret=r, floor=floor, solves=solves, info=info)

