"""Return panels with a prescribed conditioning of the reduced data map AU.

The controlled CRRA conditioning benchmark (computational study and its
appendix table) fixes the positive singular spectrum of AU, U an
orthonormal basis of the simplex tangent space {1}^perp, and keeps the
equal-weight start in the null space of A.  The construction
A = Q diag(s) W^T does both: Q (T x r) has orthonormal columns orthogonal to
1_T, so A is centred; W (n x r) has orthonormal columns orthogonal to 1_n,
so A 1 = 0 and W^T U has orthonormal rows, making the nonzero singular
values of AU exactly s.  r = min(n, T) - 1, and s runs geometrically from
s0 to s0 * kappa, so kappa_+(AU) = kappa.

Recipe ``conditioned_returns(n, T, kappa, seed)``: with
``rng = numpy.random.default_rng(seed)`` draw, in this order, a T x r and an
n x r standard normal block (orthonormalised together with the all-ones
vector by a reduced QR), and the asset means ``mu ~ N(5e-4, 1e-3^2)``; s0
makes the root-mean-square entry of A equal to 1%; R = A + 1 mu^T.
"""

from __future__ import annotations

import numpy as np


def _orth_to_ones(G: np.ndarray) -> np.ndarray:
    """Orthonormal columns spanning the part of range(G) orthogonal to 1."""
    m = G.shape[0]
    Qf, _ = np.linalg.qr(np.column_stack([np.ones(m), G]))
    return Qf[:, 1:]


def conditioned_returns(n: int, T: int, kappa: float, seed: int,
                        rms: float = 0.01) -> np.ndarray:
    """Returns R (T x n) whose centred map A has kappa_+(AU) = kappa and A 1 = 0."""
    rng = np.random.default_rng(seed)
    r = min(n, T) - 1
    Q = _orth_to_ones(rng.standard_normal((T, r)))
    W = _orth_to_ones(rng.standard_normal((n, r)))
    mu = 5e-4 + 1e-3 * rng.standard_normal(n)
    s = kappa ** (np.arange(r) / max(r - 1, 1))
    s *= rms * np.sqrt(T * n / np.sum(s * s))
    A = (Q * s) @ W.T
    return np.ascontiguousarray(A + mu[None, :])


def conditioning_spectrum(n: int, T: int, kappa: float, rms: float = 0.01):
    """The positive singular values s of AU used by conditioned_returns."""
    r = min(n, T) - 1
    s = kappa ** (np.arange(r) / max(r - 1, 1))
    return s * rms * np.sqrt(T * n / np.sum(s * s))
