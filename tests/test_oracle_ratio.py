"""Pins of the oracle's acceptance ratio (the Slater part of Eq.
(11.12.23.1)) by the determinant itself: numpy.linalg.det of the Slater
matrix before and after one electron moves, and finite differences of that
ratio for its gradient and Laplacian."""
import numpy as np

import oracle

SKEW = np.array([[5.0, 0.3, 0.1], [0.2, 4.5, 0.4], [0.1, -0.3, 6.0]])


def slater(A, n, c, R):
    return oracle.evaluate(A, n, c, R, want=("val",))["val"]      # D[j, l] = psi_l(r_j)


def test_ratio_is_the_determinant_ratio():
    rng = np.random.default_rng(0)
    n = (7, 8, 6)
    L = 12
    c = rng.uniform(-1, 1, n + (L,))
    R = rng.uniform(0, 5, (L, 3))                  # the old configuration
    D = slater(SKEW, n, c, R)
    Dinv = np.linalg.inv(D)
    moves = R + rng.normal(0, 0.4, R.shape)        # one trial move per electron
    cols = np.arange(L)
    r = oracle.ratio(SKEW, n, c, moves, Dinv.T.copy(), cols)
    d0 = np.linalg.det(D)
    for j in range(L):
        Dj = D.copy()
        Dj[j] = slater(SKEW, n, c, moves[j:j + 1])[0]
        np.testing.assert_allclose(r["ratio"][j], np.linalg.det(Dj) / d0, rtol=1e-9)


def test_ratio_gradient_and_laplacian_by_finite_differences():
    rng = np.random.default_rng(1)
    n = (9, 8, 10)
    L = 10
    c = rng.uniform(-1, 1, n + (L,))
    R = rng.uniform(0, 5, (L, 3))
    D = slater(SKEW, n, c, R)
    Dinv = np.linalg.inv(D)
    d0 = np.linalg.det(D)
    j = 3
    rp = R[j] + np.array([0.21, -0.13, 0.07])
    h = 1e-4

    def det_ratio(x):
        Dj = D.copy()
        Dj[j] = slater(SKEW, n, c, x[None, :])[0]
        return np.linalg.det(Dj) / d0

    r = oracle.ratio(SKEW, n, c, rp[None, :], Dinv.T.copy(), [j])
    g_fd = np.zeros(3)
    lap_fd = 0.0
    f0 = det_ratio(rp)
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        fp, fm = det_ratio(rp + e), det_ratio(rp - e)
        g_fd[d] = (fp - fm) / (2 * h)
        lap_fd += (fp - 2 * f0 + fm) / (h * h)
    np.testing.assert_allclose(r["ratio"][0], f0, rtol=1e-10)
    np.testing.assert_allclose(r["grad"][0], g_fd, rtol=1e-6, atol=1e-8 * abs(f0))
    np.testing.assert_allclose(r["lap"][0], lap_fd, rtol=1e-4, atol=1e-5 * abs(f0))


def test_unmoved_electron_has_ratio_one():
    rng = np.random.default_rng(2)
    n = (6, 6, 6)
    L = 8
    c = rng.uniform(-1, 1, n + (L,))
    R = rng.uniform(0, 4, (L, 3))
    Dinv = np.linalg.inv(slater(np.diag([4.0, 4.0, 4.0]), n, c, R))
    r = oracle.ratio(np.diag([4.0, 4.0, 4.0]), n, c, R, Dinv.T.copy(), np.arange(L))
    np.testing.assert_allclose(r["ratio"], 1.0, rtol=1e-10)
