"""FP64 ES-kernel NUFFT, type 2 (slicing) and type 1 (merging adjoint).

Slicing (section II-A) is a type-2 NUFFT of the model; merging (section
II-C, Eq. (1)-(2)) needs the type-1 NUFFT A* of the oriented data.  The paper
uses the ES-kernel NUFFT library of its reference [barnett2019parallel]; the
steps below follow that method in its usual order:

type 2, modes m (N^3, N odd) -> values at points x (J, 3):
  1. deconvolve:  b_k = m_k / (psi_hat(k0) psi_hat(k1) psi_hat(k2))
  2. zero-pad:    B (nf^3, nf = 2N) with B[k mod nf] = b_k
  3. transform:   u_l = sum_k B_k exp(+2 pi i k.l / nf)
  4. interpolate: s(x) = sum_{a,b,c in 0..w-1} u_{l0+(a,b,c) mod nf}
                          psi(t0-l0_0-a) psi(t1-l0_1-b) psi(t2-l0_2-c)
     with t = x nf / (2 pi) and l0 = ceil(t - w/2): the w cells
     t - w/2 <= l < t + w/2 (half-open support).
type 1, values y at points x -> modes (N^3): the transposes in reverse:
  1. spread:      v_l = sum_j y_j psi psi psi (t_j - l)   (same support rule)
  2. transform:   V = sum_l v_l exp(-2 pi i k.l / nf)
  3. truncate + deconvolve: f_k = V[k mod nf] / (psi_hat psi_hat psi_hat)

so type 1 is the exact adjoint of this (approximate) type 2.  Real mode:
type 2 uses the even part of m and returns Re(s) (= sum m_k cos(k.x));
type 1 returns Re(f) (= the adjoint of real-mode type 2 for real y).

TEST INFRASTRUCTURE ONLY (see package docstring).
"""
from __future__ import annotations

import numpy as np

from .es import es_kernel, es_hat


def _params(N: int, w: int, beta_over_w: float):
    if N % 2 != 1:
        raise ValueError("N must be odd")
    nf = 2 * N
    beta = beta_over_w * w
    h = (N - 1) // 2
    k = np.arange(-h, h + 1)
    ph = es_hat(k, w, beta, nf)
    return nf, beta, k, ph


def _support(x, nf: int, w: int, beta: float):
    """Fine-grid coordinates t, first support cell l0 and the w weights per
    axis, for points x (J, 3)."""
    t = np.asarray(x, dtype=np.float64).reshape(-1, 3) * (nf / (2.0 * np.pi))
    l0 = np.ceil(t - 0.5 * w).astype(np.int64)
    a = np.arange(w)
    wts = es_kernel(t[:, :, None] - (l0[:, :, None] + a), w, beta)  # (J,3,w)
    return t, l0, wts


def fine_grid(m, w: int = 6, beta_over_w: float = 2.30, real: bool = False):
    """Steps 1-3 of type 2: the oversampled uniform grid u (nf^3, complex)."""
    m = np.asarray(m)
    N = m.shape[0]
    nf, beta, k, ph = _params(N, w, beta_over_w)
    if real:
        m = 0.5 * (m + m[::-1, ::-1, ::-1])
    b = m / (ph[:, None, None] * ph[None, :, None] * ph[None, None, :])
    B = np.zeros((nf, nf, nf), dtype=np.complex128)
    kk = k % nf
    B[np.ix_(kk, kk, kk)] = b
    return nf ** 3 * np.fft.ifftn(B)


def nufft2(m, x, w: int = 6, beta_over_w: float = 2.30, real: bool = False,
           chunk: int = 1 << 20) -> np.ndarray:
    """Type-2 NUFFT of modes m (N,N,N) at points x (J,3)."""
    m = np.asarray(m)
    N = m.shape[0]
    nf, beta, _, _ = _params(N, w, beta_over_w)
    u = fine_grid(m, w, beta_over_w, real)
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    out = np.empty(x.shape[0], dtype=np.complex128)
    for s0 in range(0, x.shape[0], chunk):
        t, l0, wts = _support(x[s0:s0 + chunk], nf, w, beta)
        acc = np.zeros(t.shape[0], dtype=np.complex128)
        for a in range(w):
            i0 = (l0[:, 0] + a) % nf
            for b in range(w):
                i1 = (l0[:, 1] + b) % nf
                wab = wts[:, 0, a] * wts[:, 1, b]
                for c in range(w):
                    i2 = (l0[:, 2] + c) % nf
                    acc += u[i0, i1, i2] * (wab * wts[:, 2, c])
        out[s0:s0 + chunk] = acc
    return out.real.copy() if real else out


def spread(y, x, nf: int, w: int, beta: float) -> np.ndarray:
    """Type-1 step 1: v_l = sum_j y_j psi psi psi(t_j - l), (nf,nf,nf)."""
    y = np.asarray(y).reshape(-1)
    t, l0, wts = _support(x, nf, w, beta)
    v = np.zeros(nf ** 3, dtype=np.complex128)
    yr, yi = y.real.astype(np.float64), np.imag(y).astype(np.float64)
    for a in range(w):
        i0 = (l0[:, 0] + a) % nf
        for b in range(w):
            i1 = (l0[:, 1] + b) % nf
            wab = wts[:, 0, a] * wts[:, 1, b]
            for c in range(w):
                i2 = (l0[:, 2] + c) % nf
                flat = (i0 * nf + i1) * nf + i2
                wt = wab * wts[:, 2, c]
                v.real += np.bincount(flat, weights=yr * wt, minlength=nf ** 3)
                if np.iscomplexobj(y):
                    v.imag += np.bincount(flat, weights=yi * wt, minlength=nf ** 3)
    return v.reshape(nf, nf, nf)


def nufft1(y, x, N: int, w: int = 6, beta_over_w: float = 2.30,
           real: bool = False) -> np.ndarray:
    """Type-1 NUFFT of values y (J,) at points x (J,3) onto N^3 modes."""
    nf, beta, k, ph = _params(N, w, beta_over_w)
    v = spread(y, x, nf, w, beta)
    V = np.fft.fftn(v)
    kk = k % nf
    f = V[np.ix_(kk, kk, kk)] / (ph[:, None, None] * ph[None, :, None] * ph[None, None, :])
    return f.real.copy() if real else f
