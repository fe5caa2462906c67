"""Gradient of the weighted slice-to-image loss with respect to the model.

The loss L(m) = sum_{n,p} w_np |s_np(m) - d_np|^2 with s = A m the type-2
slices at each image's orientation is the weighted least-squares objective
of merging (section II-C, Eq. (1) with the weights D of Eq. (2)); its
gradient is 2 A^H (W (A m - d)), the type-1 NUFFT of the weighted residual
(the right-hand side A* D b of Eq. (2) minus A* D A m).  For complex m this
is the convention dL/dRe(m) + i dL/dIm(m).

TEST INFRASTRUCTURE ONLY (see package docstring).
"""
from __future__ import annotations

import numpy as np

from .nufft import nufft1, nufft2


def loss(m, x, d, wts, w: int = 6, beta_over_w: float = 2.30) -> float:
    s = nufft2(m, x, w, beta_over_w)
    r = s - np.asarray(d).reshape(-1)
    return float(np.sum(np.asarray(wts).reshape(-1) * (r.real ** 2 + r.imag ** 2)))


def grad(m, x, d, wts, w: int = 6, beta_over_w: float = 2.30) -> np.ndarray:
    m = np.asarray(m)
    s = nufft2(m, x, w, beta_over_w)
    r = np.asarray(wts).reshape(-1) * (s - np.asarray(d).reshape(-1))
    return 2.0 * nufft1(r, x, m.shape[0], w, beta_over_w)


def fd_grad(m, x, d, wts, voxels, h: float, w: int = 6,
            beta_over_w: float = 2.30) -> np.ndarray:
    """Central differences of the loss at flat voxel indices, real and
    imaginary directions: returns complex dL/dRe + i dL/dIm."""
    m = np.asarray(m, dtype=np.complex128)
    out = np.empty(len(voxels), dtype=np.complex128)
    for i, v in enumerate(voxels):
        parts = []
        for dirn in (1.0, 1j):
            mp = m.copy().reshape(-1)
            mm = m.copy().reshape(-1)
            mp[v] += h * dirn
            mm[v] -= h * dirn
            lp = loss(mp.reshape(m.shape), x, d, wts, w, beta_over_w)
            lm = loss(mm.reshape(m.shape), x, d, wts, w, beta_over_w)
            parts.append((lp - lm) / (2.0 * h))
        out[i] = parts[0] + 1j * parts[1]
    return out
