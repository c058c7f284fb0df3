"""The push-through identity behind the T < n exact trace of the PCG
configuration, checked numerically on the CPU (host-side mathematics of the
GPU path; the oracle keeps the explicit (m-1) x (m-1) factorisation).

With P = A V (V orthonormal, V V^T = P_S), S = diag(s) > 0 and lambda > 0:
    q_t = p_t^T (P^T S P + lambda I)^-1 p_t
        = (1 - lambda [(S^1/2 G S^1/2 + lambda I)^-1]_tt) / s_t,
    G = P P^T = A P_S A^T.
"""

import numpy as np
import pytest


@pytest.mark.parametrize("T,n,p", [(7, 30, 1), (40, 200, 2), (65, 131, 2)])
def test_push_through_trace_matches_reduced_factorisation(T, n, p):
    rng = np.random.default_rng(T * n)
    A = rng.standard_normal((T, n))
    A -= A.mean(axis=0)                       # centred like the sample matrix
    E = np.linalg.qr(rng.standard_normal((n, p + 1)))[0]   # frame + normal
    V = np.linalg.qr(np.eye(n) - E @ E.T)[0][:, : n - p - 1]
    P = A @ V
    s = rng.uniform(0.5, 2.0, T) / T
    lam = 1e-4 * np.trace(P.T @ (s[:, None] * P)) / (n - p - 1)
    Bm = P.T @ (s[:, None] * P) + lam * np.eye(n - p - 1)
    q_ref = np.einsum("ti,ij,tj->t", P, np.linalg.inv(Bm), P)
    # thin form: G from the ambient projector, the T x T system only
    G = A @ A.T - (A @ E) @ (A @ E).T
    assert np.allclose(G, P @ P.T, rtol=0, atol=1e-12 * np.abs(G).max())
    C = np.sqrt(s)[:, None] * G * np.sqrt(s)[None, :] + lam * np.eye(T)
    Linv = np.linalg.inv(np.linalg.cholesky(C))
    q = (1.0 - lam * np.sum(Linv * Linv, axis=0)) / s
    assert np.max(np.abs(q - q_ref)) <= 1e-9 * np.max(np.abs(q_ref))
    # and the same trace term as the oracle's a = P^T (psi''' q) / T
    w3 = rng.standard_normal(T)
    assert np.allclose(P.T @ (w3 * q), P.T @ (w3 * q_ref), rtol=1e-8,
                       atol=1e-10 * np.abs(P.T @ (w3 * q_ref)).max())


def test_trace_scale_matches_reduced_trace():
    # lambda's scale sum_t s_t G_tt is the trace of the reduced P^T S P
    rng = np.random.default_rng(3)
    T, n = 30, 90
    A = rng.standard_normal((T, n))
    A -= A.mean(axis=0)
    E = np.linalg.qr(rng.standard_normal((n, 2)))[0]
    V = np.linalg.qr(np.eye(n) - E @ E.T)[0][:, : n - 2]
    s = rng.uniform(0.5, 2.0, T)
    G = A @ A.T - (A @ E) @ (A @ E).T
    P = A @ V
    assert np.sum(s * np.diag(G)) == pytest.approx(
        np.trace(P.T @ (s[:, None] * P)), rel=1e-12)
