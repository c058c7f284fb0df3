"""The controlled-conditioning generator: centred map, equal weights in the
null space of A, and the prescribed positive spectrum of AU (checked with an
SVD of AU for an orthonormal basis U of the simplex tangent space)."""

import numpy as np
import pytest

import oracle as O
import synth


@pytest.mark.parametrize("n,T", [(40, 80), (60, 25)])
@pytest.mark.parametrize("kappa", [1.0, 10.0, 1e3])
def test_conditioned_returns_spectrum(n, T, kappa):
    R = synth.conditioned_returns(n, T, kappa, seed=7)
    mu, A = O.center(R)
    assert np.abs(A @ np.full(n, 1.0 / n)).max() <= 1e-15
    U = O.tangent_basis(np.ones((n, 1)))
    sv = np.linalg.svd(A @ U, compute_uv=False)
    r = min(n, T) - 1
    s = np.sort(synth.conditioning_spectrum(n, T, kappa))[::-1]
    assert np.abs(sv[:r] - s).max() <= 1e-12 * s.max()
    assert sv[r:].max(initial=0.0) <= 1e-12 * s.max()
    assert sv[0] / sv[r - 1] == pytest.approx(kappa, rel=1e-10)
    assert np.sqrt(np.mean(A * A)) == pytest.approx(0.01, rel=1e-12)
