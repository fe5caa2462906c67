"""Exponential-of-semicircle (ES) spreading kernel and its Fourier transform.

The paper computes slicing and merging with the ES-kernel NUFFT of its
reference [barnett2019parallel] (section III-A).  Reading used here: kernel

    psi(tau) = exp(beta * (sqrt(1 - (2 tau / w)^2) - 1))   for |tau| <= w/2,

zero outside, with tau measured in fine-grid cells, width w and shape
beta = 2.30 w at upsampling factor 2.

TEST INFRASTRUCTURE ONLY (see package docstring).
"""
from __future__ import annotations

import numpy as np


def es_kernel(tau, w: int, beta: float) -> np.ndarray:
    """psi(tau) for an array of offsets ``tau`` (cells); 0 for |tau| > w/2."""
    tau = np.asarray(tau, dtype=np.float64)
    z = 2.0 * tau / w
    inside = np.abs(z) <= 1.0
    out = np.zeros_like(tau)
    out[inside] = np.exp(beta * (np.sqrt(1.0 - z[inside] ** 2) - 1.0))
    return out


def es_hat(k, w: int, beta: float, nf: int, nodes: int = 400) -> np.ndarray:
    """psi_hat(k) = integral_{-w/2}^{w/2} psi(tau) cos(2 pi k tau / nf) dtau.

    This is the Fourier coefficient of the kernel at mode k on a fine grid of
    nf cells, the factor the NUFFT divides out (the deconvolution).  Computed
    by Gauss-Legendre quadrature in tau with ``nodes`` nodes.
    """
    k = np.asarray(k, dtype=np.float64)
    z, wt = np.polynomial.legendre.leggauss(nodes)
    tau = 0.5 * w * z
    vals = es_kernel(tau, w, beta)
    ph = np.cos(2.0 * np.pi * np.multiply.outer(k, tau) / nf)
    return 0.5 * w * (ph * (vals * wt)).sum(axis=-1)
