"""CPU pins of the oracle's principal components of the bands (moments, the
Jacobi eigen-decomposition, projection and inverse).

What pins it, none of it derived from the oracle itself:
- moments: numpy's mean and population covariance, and exact rational
  arithmetic (fractions) rounded once, on random u16 samples;
- eigen-decomposition: numpy.linalg.eigh (LAPACK) eigenvalues and
  eigenvectors up to sign; the closed form of a 2 x 2 covariance
  [[a, b], [b, a]]; orthonormality; A v = lambda v; the sign and order
  conventions;
- projection: numpy's (x - m) V in binary64 then binary32, within one f32
  rounding; the variance of each PC equals its eigenvalue; all PCs invert
  back to the integer input exactly after rounding;
- a band that is a copy of another gives a zero eigenvalue.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O


def _samples(n, Bn, seed, correlated=True):
    rng = np.random.default_rng(seed)
    z = rng.normal(0, 1, (n, Bn))
    if correlated:
        mix = rng.normal(0, 1, (Bn, Bn))
        z = z @ mix
    x = 3000 + 600 * z + rng.integers(0, 50, (n, Bn))
    return np.clip(np.round(x), 0, 65535).astype(np.uint16)


@pytest.mark.parametrize("Bn", [1, 3, 4, 10])
def test_moments_against_numpy_and_exact_rationals(Bn):
    x = _samples(700, Bn, seed=Bn)
    mean, cov = O.pca_moments(x)
    xf = x.astype(np.float64)
    assert np.allclose(mean, xf.mean(0), rtol=0, atol=1e-9)
    ref = np.cov(xf.T, bias=True).reshape(Bn, Bn)
    assert np.allclose(cov, ref, rtol=1e-12, atol=1e-9)
    # exact: the rational (n Q - S S) / n^2 and S / n, correctly rounded
    n = x.shape[0]
    xi = x.astype(object)
    for b in range(Bn):
        S_b = int(xi[:, b].sum())
        assert mean[b] == float(Fraction(S_b, n))
        for c in range(Bn):
            S_c = int(xi[:, c].sum())
            Q = int((xi[:, b] * xi[:, c]).sum())
            exact = Fraction(n * Q - S_b * S_c, n * n)
            assert abs(cov[b, c] - float(exact)) <= 4e-16 * abs(float(exact)) + 1e-300


@pytest.mark.parametrize("Bn", [2, 3, 6, 10, 16])
def test_eigen_against_lapack(Bn):
    x = _samples(900, Bn, seed=100 + Bn)
    _, cov = O.pca_moments(x)
    ev, V = O.pca_eigen(cov)
    w, U = np.linalg.eigh(cov)
    w, U = w[::-1], U[:, ::-1]
    assert np.allclose(ev, w, rtol=1e-10, atol=1e-8 * w[0])
    assert np.all(np.diff(ev) <= 0)
    for j in range(Bn):
        u = U[:, j] * np.sign(U[np.argmax(np.abs(U[:, j])), j])
        assert np.allclose(V[:, j], u, atol=1e-8), j
        assert V[np.argmax(np.abs(V[:, j])), j] > 0
        assert np.allclose(cov @ V[:, j], ev[j] * V[:, j], atol=1e-7 * ev[0])
    assert np.allclose(V.T @ V, np.eye(Bn), atol=1e-13)


def test_two_by_two_closed_form():
    a, b = 5.0, 2.0
    cov = np.array([[a, b], [b, a]])
    ev, V = O.pca_eigen(cov)
    assert np.allclose(ev, [a + b, a - b], rtol=1e-15)
    r = 1 / np.sqrt(2)
    assert np.allclose(V[:, 0], [r, r], atol=1e-15)
    assert np.allclose(np.abs(V[:, 1]), [r, r], atol=1e-15)
    # the larger-magnitude component (the first of equals) is positive
    assert V[0, 1] > 0 and V[1, 1] < 0
    # diagonal input: no rotation, order by size
    ev, V = O.pca_eigen(np.diag([1.0, 7.0, 3.0]))
    assert list(ev) == [7.0, 3.0, 1.0]
    assert np.array_equal(V, np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0]], float))


@pytest.mark.parametrize("Bn", [3, 4, 10])
def test_projection_variance_and_round_trip(Bn):
    x = _samples(600, Bn, seed=200 + Bn).reshape(6, 10, 10, Bn)
    mean, cov = O.pca_moments(x)
    ev, V = O.pca_eigen(cov)
    y = O.pca_project(x, mean, V, 0, Bn)
    ref = ((x.reshape(-1, Bn).astype(np.float64) - mean) @ V).astype(np.float32)
    assert np.allclose(y.reshape(-1, Bn), ref, rtol=2 ** -22, atol=1e-3)
    # PC variances are the eigenvalues
    yv = y.reshape(-1, Bn).astype(np.float64)
    assert np.allclose(yv.var(0), ev, rtol=1e-5, atol=1e-3 * ev[0])
    assert np.allclose(yv.mean(0), 0, atol=1e-3 * np.sqrt(ev[0]))
    # a sub-range of PCs is the matching columns
    assert np.array_equal(O.pca_project(x, mean, V, 1, 3), y[..., 1:3])
    # every PC kept: the integer input comes back after rounding
    back = O.pca_inverse(y, mean, V, O.U16)
    assert np.array_equal(back, x)
    backf = O.pca_inverse(y, mean, V, O.F32)
    assert np.allclose(backf, x, atol=0.01)
    # fewer PCs: the least-squares reconstruction, error = dropped variance
    k = Bn - 1
    part = O.pca_inverse(y[..., :k], mean, V, O.F32).astype(np.float64)
    err = ((part - x) ** 2).sum(-1).mean()
    assert abs(err - ev[k:].sum()) <= 1e-3 * ev[0] + 1e-4 * ev[k:].sum()


def test_duplicated_band_has_zero_variance_direction():
    x = _samples(400, 3, seed=9)
    x = np.concatenate([x, x[:, :1]], 1)  # band 3 copies band 0
    _, cov = O.pca_moments(x)
    ev, V = O.pca_eigen(cov)
    assert abs(ev[-1]) <= 1e-9 * ev[0]
    r = 1 / np.sqrt(2)
    assert np.allclose(np.abs(V[:, -1]), [r, 0, 0, r], atol=1e-7)
