"""The host 1-D decomposition behind the fast-diagonalisation solve
(lasto_fdm_axis; no device work): A = S diag(lam) Sinv for the interior
three-point operator of a graded axis, S Sinv = I, the eigenvalues against
numpy's, and the uniform-mesh closed form -4/h^2 sin^2(k pi / (2 (n-1)))."""
import math

import numpy as np
import pytest


@pytest.fixture(scope="module")
def L():
    from paper_0806_1723_amd import lasto
    lasto.load()
    return lasto


def interior_operator(x):
    n = len(x)
    m = n - 2
    A = np.zeros((m, m))
    for t in range(m):
        i = t + 1
        hm, hp = x[i] - x[i - 1], x[i + 1] - x[i]
        w = 0.5 * (hm + hp)
        A[t, t] = -1.0 / (hm * w) - 1.0 / (hp * w)
        if t > 0:
            A[t, t - 1] = 1.0 / (hm * w)
        if t + 1 < m:
            A[t, t + 1] = 1.0 / (hp * w)
    return A


@pytest.mark.parametrize("n", [3, 4, 17, 66, 257])
def test_decomposition_reproduces_the_operator(L, n):
    rng = np.random.default_rng(n)
    x = np.concatenate([[0.0], np.cumsum(rng.uniform(0.2, 1.8, n - 1))])
    lam, S, Si = L.fdm_axis(x)
    A = interior_operator(x)
    scale = np.abs(A).max()
    assert np.abs(S @ np.diag(lam) @ Si - A).max() <= 1e-12 * scale * n
    assert np.abs(S @ Si - np.eye(n - 2)).max() <= 1e-12 * n
    want = np.sort(np.linalg.eigvals(A).real)
    assert np.abs(np.sort(lam) - want).max() <= 1e-11 * scale
    assert (lam < 0).all()


def test_uniform_mesh_closed_form(L):
    n, h = 65, 0.25
    x = np.arange(n) * h
    lam, _, _ = L.fdm_axis(x)
    k = np.arange(1, n - 1)
    want = -4.0 / h ** 2 * np.sin(k * math.pi / (2 * (n - 1))) ** 2
    assert np.abs(np.sort(lam) - np.sort(want)).max() <= 1e-12 * abs(want).max()


def test_bad_coordinates_rejected(L):
    with pytest.raises(L.LastoError):
        L.fdm_axis(np.array([0.0, 1.0, 1.0, 2.0]))
