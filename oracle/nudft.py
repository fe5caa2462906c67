"""Exact nonuniform DFTs by direct summation (tiny inputs only).

These are the plain definitions the NUFFT approximates.  Modes are centred,
k in {-h..h}^3 with N = 2h + 1 odd, array index i <-> mode i - h (C order,
axis 0 <-> x_0); points x are in radians per voxel.

* type 2 (slicing, section II-A):   s_j = sum_k m_k exp(+i k.x_j)
  real mode:                         s_j = sum_k m_k cos(k.x_j)
* type 1 (merging A*, Eq. (2)):     f_k = sum_j y_j exp(-i k.x_j)
  real mode:                         f_k = sum_j y_j cos(k.x_j)

Each type-1 form is the exact adjoint of the type-2 form of the same mode.

TEST INFRASTRUCTURE ONLY (see package docstring).
"""
from __future__ import annotations

import numpy as np


def _modes(N: int) -> np.ndarray:
    h = (N - 1) // 2
    k = np.arange(-h, h + 1, dtype=np.float64)
    K = np.stack(np.meshgrid(k, k, k, indexing="ij"), axis=-1)
    return K.reshape(-1, 3)


def nudft2(m, x, real: bool = False, chunk: int = 512) -> np.ndarray:
    """Type-2 direct sum at points x (J, 3) of coefficients m (N, N, N)."""
    m = np.asarray(m)
    N = m.shape[0]
    K = _modes(N)
    mf = m.reshape(-1)
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    out = np.empty(x.shape[0], dtype=np.float64 if real else np.complex128)
    for s in range(0, x.shape[0], chunk):
        ph = x[s:s + chunk] @ K.T
        if real:
            out[s:s + chunk] = np.cos(ph) @ mf
        else:
            out[s:s + chunk] = np.exp(1j * ph) @ mf
    return out


def nudft1(y, x, N: int, real: bool = False, chunk: int = 512) -> np.ndarray:
    """Type-1 direct sum of values y (J,) at points x (J, 3) onto N^3 modes."""
    K = _modes(N)
    y = np.asarray(y)
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(K.shape[0], dtype=np.float64 if real else np.complex128)
    for s in range(0, x.shape[0], chunk):
        ph = K @ x[s:s + chunk].T
        if real:
            out += np.cos(ph) @ y[s:s + chunk]
        else:
            out += np.exp(-1j * ph) @ y[s:s + chunk]
    return out.reshape(N, N, N)
