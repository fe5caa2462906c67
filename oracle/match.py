"""Orientation matching: distances, argmin, top-2 gap, error bounds, BF16.

Section II-B: each of the N experimental images is compared with all M model
images and takes the orientation of the closest one in Euclidean distance
(O(MN) work).  Readings: D[m, n] = sum_p (s_mp - d_np)^2; ties go to the
lowest model index m (first occurrence).

The GPU computes D as |s|^2 + |d|^2 - 2 s.d in FP32 (and optionally with BF16
products); the bounds here state how far such a value can sit from the
exact one, so that tests can demand identical argmins exactly where the
exact top-2 gap exceeds them.

TEST INFRASTRUCTURE ONLY (see package docstring).
"""
from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24   # unit roundoff of IEEE binary32
UBF = 2.0 ** -8    # unit roundoff of bfloat16 (8-bit significand)


def distances_direct(S, D) -> np.ndarray:
    """D[m, n] = sum_p (S[m,p] - D[n,p])^2 summed directly, FP64 (tiny)."""
    S = np.asarray(S, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    out = np.empty((S.shape[0], D.shape[0]))
    for n in range(D.shape[0]):
        diff = S - D[n][None, :]
        out[:, n] = (diff * diff).sum(axis=1)
    return out


def distances_expanded(S, D) -> np.ndarray:
    """|s_m|^2 + |d_n|^2 - 2 s_m.d_n in FP64 (same value as the direct sum
    up to FP64 rounding)."""
    S = np.asarray(S, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    sn = (S * S).sum(axis=1)
    dn = (D * D).sum(axis=1)
    return sn[:, None] + dn[None, :] - 2.0 * (S @ D.T)


def distances_weighted(S, D, w) -> np.ndarray:
    """D_w[m, n] = sum_p w_p (S[m,p] - D[n,p])^2 with per-pixel weights
    w_p >= 0 (the weights D of Eq. (2); a beam-stop mask is w_p in {0, 1}),
    summed directly in FP64."""
    S = np.asarray(S, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    out = np.empty((S.shape[0], D.shape[0]))
    for n in range(D.shape[0]):
        diff = S - D[n][None, :]
        out[:, n] = (diff * diff * w[None, :]).sum(axis=1)
    return out


def argmin_first(Dmat) -> np.ndarray:
    """Per image (column), the lowest m attaining the minimum distance."""
    return np.argmin(np.asarray(Dmat), axis=0).astype(np.int64)


def top2(Dmat):
    """Per column: (smallest value, second smallest value)."""
    part = np.partition(np.asarray(Dmat), 1, axis=0)
    return part[0], part[1]


def gamma(L: int, u: float = U32) -> float:
    """gamma_L = L u / (1 - L u): the standard bound on the relative error
    of L chained floating-point additions/multiplications."""
    return L * u / (1.0 - L * u)


def fp32_distance_bound(snorm2, dnorm2, absdot, L: int) -> np.ndarray:
    """Bound on |fl32(D) - D| for D = |s|^2 + |d|^2 - 2 s.d evaluated in
    FP32 when every sum in it is a chain of at most L roundings:
    gamma_L (|s|^2 + |d|^2 + 2 sum_p |s_p d_p|)."""
    return gamma(L) * (np.asarray(snorm2) + np.asarray(dnorm2) + 2.0 * np.asarray(absdot))


def bf16_round(x) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest, ties to even) and
    return them as float32."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32)


def topk(Dmat, k: int):
    """Per column, the k smallest values' row indices, ordered by (value,
    index); shape (k, n_cols)."""
    Dm = np.asarray(Dmat)
    order = np.lexsort((np.broadcast_to(np.arange(Dm.shape[0])[:, None], Dm.shape), Dm), axis=0)
    return order[:k]


# ---------------------------------------------------------------------------
# Centred BF16 proxy (the precision form of section II-B: BF16 products with
# FP32 accumulation nominate candidates, an FP32 rescore decides).
#
# Reading: subtracting one vector c from every model image and every image
# leaves each distance unchanged, |(s - c) - (d - c)| = |s - d|, and removes
# the bright low-q intensity all slices and images share, so BF16 rounding
# acts on the small centred values.  With s^ = bf16(s - c) and d^ = bf16(d
# - c), the proxy b = |s^ - d^|^2 is a true squared distance, and the
# triangle inequality gives |sqrt(D) - sqrt(b)| <= e_m + f_n with the
# per-row rounding-error norms e_m = |s^ - (s - c)|, f_n = |d^ - (d - c)|.


def centre_rounded_mean(D) -> np.ndarray:
    """Per-pixel centre: the mean of the images' values at each pixel,
    rounded to the nearest integer (ties to even), so centred photon counts
    stay integers.  Returned as float32."""
    D = np.asarray(D, dtype=np.float64)
    return np.round(D.mean(axis=0)).astype(np.float32)


def bf16_centred(X, c):
    """(values, squared norms, rounding-error norms) of bf16(x - c) per row.

    x - c is formed in float32 (one IEEE subtraction per element), then
    rounded to BF16 (nearest, ties to even).  norm2 = sum_p v_p^2 of the BF16
    values v; err = |v - (x - c)| with x - c exact (float64)."""
    X32 = np.asarray(X, dtype=np.float32)
    c32 = np.asarray(c, dtype=np.float32)
    xc = X32 - c32[None, :]                      # float32 subtraction
    v = bf16_round(xc).astype(np.float64)
    exact = X32.astype(np.float64) - c32.astype(np.float64)[None, :]
    norm2 = (v * v).sum(axis=1)
    err = np.sqrt(((v - exact) ** 2).sum(axis=1))
    return v, norm2, err


def centred_proxy(Sv, Dv) -> np.ndarray:
    """Exact squared distances between the BF16 rows: b[m, n] = |s^_m - d^_n|^2."""
    return distances_expanded(Sv, Dv)


def centred_certificate(b, e, f, D_exact, k: int = 8) -> np.ndarray:
    """Per image n, whether the k smallest proxies contain every minimiser of
    the exact distance: each row m outside the k has sqrt(D_mn) >=
    sqrt(b_mn) - e_m - f_n, so the top-k is certified when that lower bound
    exceeds sqrt(min over the top-k of D) for every m outside it."""
    b = np.asarray(b)
    top = topk(b, k)
    out = np.empty(b.shape[1], dtype=bool)
    M = b.shape[0]
    for n in range(b.shape[1]):
        inside = np.zeros(M, dtype=bool)
        inside[top[:, n]] = True
        if inside.all():
            out[n] = True
            continue
        lb = np.sqrt(np.maximum(b[~inside, n], 0.0)) - np.asarray(e)[~inside] - f[n]
        out[n] = lb.min() > np.sqrt(np.asarray(D_exact)[top[:, n], n].min())
    return out
