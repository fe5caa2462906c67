"""Phasing: from the merged volume's Fourier amplitudes to a density.

Section II-D: starting from a random seed state, real-space constraints on
the density rho and reciprocal-space constraints on its transform are applied
in turn through the FFT and its inverse, combining error reduction (ER),
hybrid input-output (HIO) and shrinkwrap.  The paper names the three methods
(its citations: Gerchberg-Saxton, Fienup 1978, Marchesini et al. 2003) and
gives no formulas; their standard definitions are used, in the paper's
terms:

* transform: F = FFT(rho), numpy's convention (e^{-2 pi i k.r / N},
  standard index order), rho real on an N^3 grid;
* reciprocal-space projection P_M: where the amplitude A[k] is measured
  (mask M), F[k] <- A[k] F[k] / |F[k]| (phase 0 where F[k] = 0); elsewhere
  F[k] is kept; rho' = Re IFFT(F);
* real-space projection P_S: rho' on the support S (and, with positivity,
  only where rho' >= 0), 0 elsewhere;
* ER: rho <- P_S(P_M(rho));
* HIO: rho' = P_M(rho); rho <- rho' where the real-space constraint holds
  (r in S, and rho' >= 0 with positivity), rho - beta rho' elsewhere;
* error of an iteration: sum over measured k of (|F[k]| - A[k])^2 divided by
  sum over measured k of A[k]^2, from the F of the iterate it starts with;
* shrinkwrap: S <- { r : (g * |rho|)(r) >= tau max (g * |rho|) }, g the
  periodic Gaussian of standard deviation sigma cells, normalised to unit
  sum, separable, applied by direct circular convolution along each axis.

TEST INFRASTRUCTURE ONLY (see package docstring).
"""
from __future__ import annotations

import numpy as np


def fourier_projection(rho, amp, measured=None):
    """P_M: impose the measured amplitudes, keep the phases; returns
    (rho', F) with F the transform of the input."""
    F = np.fft.fftn(np.asarray(rho, dtype=np.float64))
    mag = np.abs(F)
    unit = np.where(mag > 0, F / np.where(mag > 0, mag, 1.0), 1.0)
    G = np.asarray(amp, dtype=np.float64) * unit
    if measured is not None:
        G = np.where(measured, G, F)
    return np.fft.ifftn(G).real, F


def fourier_error(F, amp, measured=None):
    """sum_M (|F| - A)^2 / sum_M A^2."""
    amp = np.asarray(amp, dtype=np.float64)
    m = np.ones(amp.shape, bool) if measured is None else np.asarray(measured, bool)
    return float(np.sum((np.abs(F) - amp)[m] ** 2) / np.sum(amp[m] ** 2))


def _holds(rho_p, support, positivity):
    ok = np.asarray(support, bool)
    return ok & (rho_p >= 0) if positivity else ok


def er_step(rho, amp, support, measured=None, positivity=True):
    """One error-reduction iteration; returns (rho_next, error)."""
    rp, F = fourier_projection(rho, amp, measured)
    return np.where(_holds(rp, support, positivity), rp, 0.0), fourier_error(F, amp, measured)


def hio_step(rho, amp, support, beta=0.9, measured=None, positivity=True):
    """One hybrid input-output iteration; returns (rho_next, error)."""
    rho = np.asarray(rho, dtype=np.float64)
    rp, F = fourier_projection(rho, amp, measured)
    return (np.where(_holds(rp, support, positivity), rp, rho - beta * rp),
            fourier_error(F, amp, measured))


def gaussian_kernel_1d(n: int, sigma: float) -> np.ndarray:
    """Periodic 1-D Gaussian g[d] ~ exp(-d^2 / (2 sigma^2)), d the signed
    periodic offset (d = j for j <= n / 2, j - n above), unit sum."""
    j = np.arange(n)
    d = np.where(j <= n // 2, j, j - n).astype(np.float64)
    g = np.exp(-d * d / (2.0 * sigma * sigma))
    return g / g.sum()


def blur(x, sigma: float) -> np.ndarray:
    """Circular convolution with the separable periodic Gaussian, one axis
    at a time, by direct sums: y[i] = sum_j g[(i - j) mod n] x[j]."""
    y = np.asarray(x, dtype=np.float64)
    for ax in range(y.ndim):
        n = y.shape[ax]
        g = gaussian_kernel_1d(n, sigma)
        out = np.zeros_like(y)
        for s in range(n):
            out += g[s] * np.roll(y, s, axis=ax)   # roll by s: out[i] += g[s] y[i - s]
        y = out
    return y


def shrinkwrap(rho, sigma: float, tau: float) -> np.ndarray:
    """New support: cells where the blurred |rho| reaches tau times its
    maximum."""
    b = blur(np.abs(np.asarray(rho, dtype=np.float64)), sigma)
    return b >= tau * b.max()
