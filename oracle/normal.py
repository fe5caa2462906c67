"""Regularised merging: the normal equations of Eq. (2) and the L-curve.

Section II-C: merging solves min_x |A x - b| for the autocorrelation x on
the uniform grid (A the type-2 operator, b the oriented intensities), made
well posed by Tikhonov regularisation:

    (A* D A + lambda I) x = A* D b + lambda x0,

D the per-point weights, x0 the initial guess.  A* D A is applied as a
convolution on the Cartesian grid (the Toeplitz method): its entries depend
only on k - k', through the type-1 transform of the weights on modes of
twice the range.  The system is solved by conjugate gradients, once per
regularisation parameter, and the L-curve picks the parameter.

Plain definitions here (tiny N): the dense NUDFT matrix, the dense normal
matrix, the Toeplitz kernel by direct sums, the convolution by explicit
shifts, plain CG, a dense solve and the discrete L-curve curvature.

Readings (listed in the design doc):
* COMPLEX domain: A[j, k] = exp(+i k.x_j), A* D A = T[k - k'] with
  T[m] = sum_j d_j exp(-i m.x_j), m in {-2h..2h}^3.
* REAL domain: A[j, k] = cos(k.x_j); A^T D A x = C * even(x) with
  C[m] = sum_j d_j cos(m.x_j) (the Hankel part C[k + k'] acts on the
  reflected x), so the solve keeps the odd part of x at that of x0.
* L-curve: rho = |D^{1/2}(A x - b)|^2 and eta = |x - x0|^2 per lambda; the
  corner is the largest curvature of (log rho, log eta) as functions of
  log lambda, by central differences on a uniform log-lambda grid.

TEST INFRASTRUCTURE ONLY (see package docstring).
"""
from __future__ import annotations

import numpy as np

from .nudft import _modes


def nudft_matrix(x, N: int, real: bool = False) -> np.ndarray:
    """A[j, k] (J x N^3): exp(+i k.x_j), or cos(k.x_j) in the REAL domain."""
    ph = np.asarray(x, dtype=np.float64).reshape(-1, 3) @ _modes(N).T
    return np.cos(ph) if real else np.exp(1j * ph)


def normal_matrix(x, d, N: int, real: bool = False) -> np.ndarray:
    """Dense A^H diag(d) A."""
    A = nudft_matrix(x, N, real)
    return A.conj().T @ (np.asarray(d, dtype=np.float64)[:, None] * A)


def toeplitz_kernel(x, d, N: int, real: bool = False) -> np.ndarray:
    """T[m] = sum_j d_j exp(-i m.x_j) (REAL: cos) on (2N - 1)^3 modes,
    m in {-(N-1)..N-1}^3, by direct sums."""
    M = 2 * N - 1
    ph = _modes(M) @ np.asarray(x, dtype=np.float64).reshape(-1, 3).T
    d = np.asarray(d, dtype=np.float64)
    T = (np.cos(ph) @ d) if real else (np.exp(-1j * ph) @ d)
    return T.reshape(M, M, M)


def even_part(x) -> np.ndarray:
    """(x[k] + x[-k]) / 2 on the centred grid."""
    x = np.asarray(x)
    return 0.5 * (x + x[::-1, ::-1, ::-1])


def toeplitz_apply(T, x, real: bool = False) -> np.ndarray:
    """y[k] = sum_k' T[k - k'] x[k'] (REAL: of even(x)), k, k' in {-h..h}^3,
    by explicit shifts of the kernel."""
    x = np.asarray(x)
    if real:
        x = even_part(x)
    N = x.shape[0]
    c = N - 1                       # kernel index of m = 0
    y = np.zeros(x.shape, dtype=np.result_type(T, x))
    for a in range(N):
        for b in range(N):
            for e in range(N):
                v = x[a, b, e]
                if v == 0:
                    continue
                # y[k] += T[k - k'] v for k' = (a, b, e) - h: window of T
                y += v * T[c - a:c - a + N, c - b:c - b + N, c - e:c - e + N]
    return y


def solve_dense(x, d, b, N: int, lam: float, x0, real: bool = False) -> np.ndarray:
    """Exact solution of (A^H D A + lam I) x = A^H D b + lam x0 (dense)."""
    A = nudft_matrix(x, N, real)
    d = np.asarray(d, dtype=np.float64)
    H = A.conj().T @ (d[:, None] * A) + lam * np.eye(N ** 3)
    rhs = A.conj().T @ (d * np.asarray(b)) + lam * np.asarray(x0).reshape(-1)
    return np.linalg.solve(H, rhs).reshape(N, N, N)


def cg(apply_op, rhs, x0, iters: int):
    """Conjugate gradients for a Hermitian positive definite operator,
    started at x0; returns (x, residual norms |r_i| for i = 0..iters).
    A residual that reaches exactly zero ends the iteration (x is then the
    solution; later norms are recorded as 0)."""
    x = np.array(x0, dtype=np.result_type(rhs, x0, np.float64))
    r = rhs - apply_op(x)
    p = r.copy()
    rr = np.vdot(r, r).real
    hist = [np.sqrt(rr)]
    for _ in range(iters):
        if rr == 0.0:
            hist.append(0.0)
            continue
        Ap = apply_op(p)
        alpha = rr / np.vdot(p, Ap).real
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = np.vdot(r, r).real
        hist.append(np.sqrt(rr_new))
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, np.array(hist)


def lcurve_corner(lambdas, rho, eta) -> int:
    """Index of the largest curvature of the L-curve (log rho, log eta) over
    a uniform grid in log lambda (central differences; end points
    excluded)."""
    t = np.log(np.asarray(lambdas, dtype=np.float64))
    u = np.log(np.asarray(rho, dtype=np.float64))
    v = np.log(np.asarray(eta, dtype=np.float64))
    dt = t[1] - t[0]
    best, arg = -np.inf, 1
    for i in range(1, len(t) - 1):
        du = (u[i + 1] - u[i - 1]) / (2 * dt)
        dv = (v[i + 1] - v[i - 1]) / (2 * dt)
        ddu = (u[i + 1] - 2 * u[i] + u[i - 1]) / dt ** 2
        ddv = (v[i + 1] - 2 * v[i] + v[i - 1]) / dt ** 2
        kappa = (du * ddv - ddu * dv) / (du * du + dv * dv) ** 1.5
        if kappa > best:
            best, arg = kappa, i
    return arg
