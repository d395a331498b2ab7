"""Pins of the FP64 smoothed-gradient oracle (paper Sec. 5.2, the shape
step's (I + lambda L)^{-2} filter) against closed forms and brute force."""
import numpy as np
import pytest

from oracle import smoothing as S
from workloads import meshes


def _dense_laplacian(F, n):
    """Independent dense construction by a loop over the face edges."""
    A = np.zeros((n, n))
    for f in np.asarray(F):
        for p in range(3):
            i, j = int(f[p]), int(f[(p + 1) % 3])
            if i != j:
                A[i, j] = A[j, i] = 1.0
    return np.diag(A.sum(1)) - A


def test_tetrahedron_closed_form():
    # K4: L = 4 I - J, eigenvalues 0 (constants) and 4 (zero-mean vectors)
    V, F = meshes.tetrahedron()
    rng = np.random.default_rng(0)
    g = rng.standard_normal((4, 3))
    lam = 50.0
    mean = g.mean(0, keepdims=True)
    want = mean + (g - mean) / (1.0 + 4.0 * lam) ** 2
    assert np.allclose(S.laplace_smooth(F, 4, g, lam), want, rtol=0, atol=1e-14)


def test_octahedron_closed_form():
    # K_{2,2,2}: L = 5 I - J + P (P swaps opposite vertices); eigenvalue 4 on
    # vectors odd under P, 6 on zero-mean vectors even under P, 0 on constants
    V = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    F = np.array([[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4], [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]])
    assert meshes.check_closed_oriented(F)
    opp = np.array([1, 0, 3, 2, 5, 4])
    rng = np.random.default_rng(1)
    g = rng.standard_normal((6, 3))
    lam = 3.0
    mean = g.mean(0, keepdims=True)
    odd = 0.5 * (g - g[opp])
    even = 0.5 * (g + g[opp]) - mean
    want = mean + odd / (1 + 4 * lam) ** 2 + even / (1 + 6 * lam) ** 2
    assert np.allclose(S.laplace_smooth(F, 6, g, lam), want, rtol=0, atol=1e-13)


@pytest.mark.parametrize("lam", [0.0, 0.5, 50.0])
def test_icosphere_against_dense_inverse(lam):
    V, F = meshes.icosphere(1)
    n = len(V)
    rng = np.random.default_rng(2)
    g = rng.standard_normal((n, 3))
    M = np.eye(n) + lam * _dense_laplacian(F, n)
    Minv = np.linalg.inv(M)
    want = Minv @ (Minv @ g)
    got = S.laplace_smooth(F, n, g, lam)
    assert np.abs(got - want).max() <= 1e-12 * max(1.0, np.abs(want).max())
    if lam == 0.0:
        assert np.array_equal(got, g)


def test_invariants_constants_symmetry_isolated_vertex():
    V, F = meshes.icosphere(2)
    n = len(V) + 1            # one vertex on no edge
    lam = 50.0
    c = np.ones((n, 3)) * np.array([1.0, -2.0, 0.5])
    assert np.allclose(S.laplace_smooth(F, n, c, lam), c, rtol=0, atol=1e-12)
    rng = np.random.default_rng(3)
    a, b = rng.standard_normal((n, 3)), rng.standard_normal((n, 3))
    Sa, Sb = S.laplace_smooth(F, n, a, lam), S.laplace_smooth(F, n, b, lam)
    assert abs((Sa * b).sum() - (a * Sb).sum()) < 1e-12 * np.abs(a).sum()
    assert np.allclose(Sa[-1], a[-1], rtol=0, atol=1e-15)     # isolated: identity row
    # smoothing damps: the filtered field is no larger than the input
    assert np.linalg.norm(Sa) <= np.linalg.norm(a)
