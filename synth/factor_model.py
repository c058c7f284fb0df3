"""Heavy-tailed factor-model return panels and the paper's uniform panel.

The factor generator stands in for the licensed 5-minute A-share panel of the
economic study (Section 7: n = 5440 assets, 48 bars a day), which is not
available.  Every draw comes from ``numpy.random.default_rng(seed)`` in a fixed
order, so a (shape, seed) pair names one return matrix exactly.

Recipe ``G(n, T, K, S, nu, p_jump, seed)`` (all returns per bar, zero drift):

* loadings ``beta ~ N(1, 0.3^2)``, shape n x K;
* unit-variance Student-t innovations ``t_nu * sqrt((nu - 2) / nu)``;
* factor returns ``F = 0.002 * t`` (T x K), idiosyncratic noise
  ``E = 0.002 * t`` (T x n);
* sectors (S > 0): asset i belongs to sector ``i mod S`` with unit loading on
  a sector return ``0.002 * t`` (T x S);
* jumps (p_jump > 0): each bar is a jump bar with probability p_jump; on such
  a bar every asset moves by ``J_t * beta[i, 0]`` with ``J_t ~ N(0, 0.02^2)``;
* ``R = F beta^T + E (+ sector block) (+ jumps)`` in float64.

Draw order: beta, F, E, sector returns, jump mask, jump sizes.
"""

from __future__ import annotations

import numpy as np

BAR_VOL = 0.002


def _unit_t(rng: np.random.Generator, nu: float, size) -> np.ndarray:
    """Student-t draws rescaled to unit variance (requires nu > 2)."""
    if nu <= 2.0:
        raise ValueError("nu must exceed 2 for a finite variance")
    return rng.standard_t(nu, size=size) * np.sqrt((nu - 2.0) / nu)


def factor_returns(n: int, T: int, K: int, S: int, nu: float, p_jump: float,
                   seed: int) -> np.ndarray:
    """Return a float64 T x n matrix drawn from the recipe ``G`` above."""
    if n < 1 or T < 1 or K < 0 or S < 0:
        raise ValueError("bad shape")
    rng = np.random.default_rng(seed)
    beta = rng.normal(1.0, 0.3, size=(n, K))
    F = BAR_VOL * _unit_t(rng, nu, (T, K))
    E = BAR_VOL * _unit_t(rng, nu, (T, n))
    R = E
    if K > 0:
        R += F @ beta.T
    if S > 0:
        sec = BAR_VOL * _unit_t(rng, nu, (T, S))
        R += sec[:, np.arange(n) % S]
    if p_jump > 0.0:
        mask = rng.random(T) < p_jump
        sizes = rng.normal(0.0, 10.0 * BAR_VOL, size=T)
        lead = beta[:, 0] if K > 0 else np.ones(n)
        jump = np.where(mask, sizes, 0.0)
        R += jump[:, None] * lead[None, :]
    return np.ascontiguousarray(R, dtype=np.float64)


def priced_factor_returns(n: int, T: int, K: int, nu: float, seed: int,
                          premium: float = 5e-4,
                          p_crash: float = 0.01) -> np.ndarray:
    """A panel whose riskier assets carry higher means and whose market
    falls in rare crashes, as a return floor and a skew preference need.

    ``G(n, T, K, 0, nu, 0, seed)`` plus two terms on the first loading
    ``beta[:, 0]`` (the draws of ``G`` recomputed from the same seed):
    a drift ``premium * beta[i, 0]`` per bar, and crash bars (probability
    p_crash each) on which asset i moves by ``-|J_t| beta[i, 0]`` with
    ``J_t ~ N(0, (10 * 0.002)^2)``.  The crash mask and sizes come from
    ``numpy.random.default_rng((seed, 1))``, mask first."""
    R = factor_returns(n, T, K, 0, nu, 0.0, seed)
    lead = np.random.default_rng(seed).normal(1.0, 0.3, size=(n, K))[:, 0]
    rng = np.random.default_rng((seed, 1))
    mask = rng.random(T) < p_crash
    sizes = -np.abs(rng.normal(0.0, 10.0 * BAR_VOL, size=T))
    R += np.where(mask, sizes, 0.0)[:, None] * lead[None, :]
    return np.ascontiguousarray(R + premium * lead[None, :])


def uniform_returns(n: int, T: int, seed: int, lo: float = -0.1,
                    hi: float = 0.4) -> np.ndarray:
    """Independent returns on [lo, hi]: the synthetic benchmark of Section 6.1."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(T, n))


def crra_coefficients(gamma: float) -> np.ndarray:
    """CRRA preference vector (c1..c4) of Remark 'Standard CRRA calibration'."""
    g = float(gamma)
    return np.array([1.0, g / 2.0, g * (g + 1.0) / 6.0,
                     g * (g + 1.0) * (g + 2.0) / 24.0])


# Named workloads: generator arguments, preference vector and seed.
WORKLOADS = {
    "n12_T500": dict(n=12, T=500, K=3, S=0, nu=5.0, p_jump=0.0, seed=0,
                     c=(1.0, 1.0, 1.0, 1.0)),
    "n400_T4800": dict(n=400, T=4800, K=10, S=0, nu=4.0, p_jump=0.0, seed=1,
                       c=(1.0, 5.0, 2.0, 10.0)),
    "n2000_T12000": dict(n=2000, T=12000, K=20, S=20, nu=4.0, p_jump=0.0,
                         seed=2, c=(1.0, 5.0, 2.0, 10.0)),
    "n1000_T12000_frontier": dict(n=1000, T=12000, K=10, S=0, nu=4.0,
                                  p_jump=0.0, seed=3, c=(1.0, 5.0, 2.0, 10.0)),
    "n5440_T12000": dict(n=5440, T=12000, K=30, S=30, nu=3.5, p_jump=0.01,
                         seed=4, c=(1.0, 5.0, 2.0, 10.0)),
}


def workload_returns(name: str, T: int | None = None) -> np.ndarray:
    """Draw the return matrix of a named workload (optionally fewer bars)."""
    w = WORKLOADS[name]
    return factor_returns(w["n"], w["T"] if T is None else T, w["K"], w["S"],
                          w["nu"], w["p_jump"], w["seed"])


def frontier_targets(R: np.ndarray, count: int) -> np.ndarray:
    """Return targets evenly spaced from the minimum-variance mean to max mean.

    Input construction only: the sample mean and covariance are taken with
    NumPy library routines; the minimum-variance mean is mu^T S^-1 1 / 1^T S^-1 1.
    Under the budget constraint alone every target is attainable.
    """
    mu = R.mean(axis=0)
    S = np.cov(R, rowvar=False, bias=True)
    ones = np.ones(R.shape[1])
    si1 = np.linalg.solve(S, ones)
    r_mv = float(mu @ si1 / (ones @ si1))
    return np.linspace(r_mv, float(mu.max()), count)


def ragged_universe_sizes(count: int = 32, lo: int = 100, hi: int = 1500,
                          seed: int = 1000) -> np.ndarray:
    """Universe sizes n_i ~ U{lo..hi} for the ragged batched workload."""
    rng = np.random.default_rng(seed)
    return rng.integers(lo, hi + 1, size=count)
