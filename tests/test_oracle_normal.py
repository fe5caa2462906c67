"""Pins of the oracle's regularised merging (section II-C, Eq. (2)): the
dense NUDFT matrix against the pinned direct sums, the Toeplitz identity of
the normal matrix, the convolution against the dense product, the dense
solve and CG against each other, and the L-curve corner on a curve with a
known bend."""
import numpy as np
import pytest

import synth
from oracle import nudft, normal


def points(n=300, seed=2):
    return synth.random_points(seed, n)


@pytest.mark.parametrize("real", [False, True])
def test_matrix_matches_direct_sums(real):
    N = 5
    g = np.random.default_rng(1)
    m = g.standard_normal((N,) * 3) + (0 if real else 1j * g.standard_normal((N,) * 3))
    x = points(200)
    np.testing.assert_allclose(normal.nudft_matrix(x, N, real) @ m.reshape(-1),
                               nudft.nudft2(m, x, real=real), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("real", [False, True])
def test_toeplitz_identity_of_the_normal_matrix(real):
    N = 5
    x = points(250)
    d = np.random.default_rng(3).uniform(0.5, 1.0, 250)
    H = normal.normal_matrix(x, d, N, real)
    T = normal.toeplitz_kernel(x, d, N, real)
    h, c = (N - 1) // 2, N - 1
    K = [(a, b, e) for a in range(N) for b in range(N) for e in range(N)]
    for i, (a, b, e) in enumerate(K[::7]):
        for j, (a2, b2, e2) in enumerate(K[::5]):
            row, col = K.index((a, b, e)), K.index((a2, b2, e2))
            if real:
                ref = 0.5 * (T[c + a - a2, c + b - b2, c + e - e2] +
                             T[a + a2 - 2 * h + c, b + b2 - 2 * h + c, e + e2 - 2 * h + c])
            else:
                ref = T[c + a - a2, c + b - b2, c + e - e2]
            assert abs(H[row, col] - ref) <= 1e-10 * np.abs(H).max()


@pytest.mark.parametrize("real", [False, True])
def test_convolution_equals_dense_product(real):
    N = 5
    x = points(300)
    d = np.random.default_rng(4).uniform(0.5, 1.0, 300)
    g = np.random.default_rng(5)
    v = g.standard_normal((N,) * 3) + (0 if real else 1j * g.standard_normal((N,) * 3))
    H = normal.normal_matrix(x, d, N, real)
    T = normal.toeplitz_kernel(x, d, N, real)
    np.testing.assert_allclose(normal.toeplitz_apply(T, v, real).reshape(-1), H @ v.reshape(-1),
                               rtol=1e-11, atol=1e-11 * np.abs(H).max())


@pytest.mark.parametrize("real", [False, True])
def test_cg_converges_to_the_dense_solution(real):
    N = 5
    x = points(400)
    g = np.random.default_rng(6)
    d = g.uniform(0.5, 1.0, 400)
    b = g.standard_normal(400) + (0 if real else 1j * g.standard_normal(400))
    x0 = g.standard_normal((N,) * 3)
    lam = 20.0
    xs = normal.solve_dense(x, d, b, N, lam, x0, real)
    A = normal.nudft_matrix(x, N, real)
    # normal equations hold
    lhs = A.conj().T @ (d * (A @ xs.reshape(-1))) + lam * xs.reshape(-1)
    rhs = A.conj().T @ (d * b) + lam * x0.reshape(-1)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-10, atol=1e-10 * np.abs(rhs).max())
    T = normal.toeplitz_kernel(x, d, N, real)
    xc, hist = normal.cg(lambda v: normal.toeplitz_apply(T, v, real) + lam * v,
                         rhs.reshape(N, N, N), x0, 60)
    assert hist[-1] <= 1e-10 * hist[0]
    np.testing.assert_allclose(xc, xs, rtol=1e-8, atol=1e-8 * np.abs(xs).max())


def test_cg_stops_at_an_exact_solution():
    # identity operator: one step reaches the solution exactly; a start at
    # the solution has a zero residual from the outset
    g = np.random.default_rng(8)
    rhs = g.standard_normal((3, 3, 3))
    x, hist = normal.cg(lambda v: v, rhs, np.zeros((3, 3, 3)), 5)
    np.testing.assert_allclose(x, rhs, rtol=1e-15)
    assert np.all(np.isfinite(hist)) and np.all(hist[2:] == 0.0)
    x, hist = normal.cg(lambda v: 2.0 * v, rhs, rhs / 2.0, 3)
    np.testing.assert_array_equal(x, rhs / 2.0)
    assert np.all(hist == 0.0)


def test_lcurve_corner_on_a_known_bend():
    # (log rho, log eta) along a vertical then a horizontal segment: the
    # only bend is at index 6
    t = np.linspace(0, 1, 12)
    lam = np.exp(t)
    u = np.where(np.arange(12) < 6, 0.0, np.arange(12) - 6.0)
    v = np.where(np.arange(12) < 6, 6.0 - np.arange(12), 0.0)
    assert normal.lcurve_corner(lam, np.exp(u), np.exp(v)) in (5, 6)
    # a smooth L: rho rises steeply only past lambda = 1, eta falls
    lam = np.logspace(-3, 3, 25)
    rho = 1.0 + lam ** 2
    eta = 1.0 + 1.0 / lam ** 2
    k = normal.lcurve_corner(lam, rho, eta)
    assert abs(np.log10(lam[k])) <= 0.75
