"""Pins of the oracle's centred BF16 proxy (section II-B precision form):
centring invariance, the per-row rounding-error bound by brute force, BF16
values against torch's rounding, and the top-8 certificate's soundness on
random and adversarial instances."""
import numpy as np
import torch

from oracle import match


def test_centre_rounded_mean_by_hand():
    D = np.array([[1.0, 2.0, 0.0], [2.0, 2.0, 5.0], [2.0, 5.0, 0.0], [3.0, 1.0, 5.0]])
    # means 2.0, 2.5, 2.5 -> 2, 2, 2 (ties to even)
    np.testing.assert_array_equal(match.centre_rounded_mean(D), [2.0, 2.0, 2.0])
    np.testing.assert_array_equal(match.centre_rounded_mean(D[:3]), [2.0, 3.0, 2.0])


def test_centring_leaves_distances_unchanged():
    g = np.random.default_rng(0)
    S = g.gamma(2.0, 30.0, (25, 300))
    D = g.poisson(S[[1, 4, 4, 20]])
    c = match.centre_rounded_mean(D).astype(np.float64)
    a = match.distances_direct(S, D)
    b = match.distances_direct(S - c, D - c)
    np.testing.assert_allclose(b, a, rtol=1e-12)


def test_bf16_centred_against_torch_and_direct_sums():
    g = np.random.default_rng(1)
    X = g.gamma(1.5, 40.0, (12, 777)).astype(np.float32)
    c = np.round(X.mean(0)).astype(np.float32)
    v, n2, err = match.bf16_centred(X, c)
    xc = torch.from_numpy(X) - torch.from_numpy(c)[None, :]          # float32 subtraction
    tv = xc.to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(v, tv)
    for r in range(X.shape[0]):
        ref_n2 = sum(float(t) * float(t) for t in tv[r])
        ref_e = np.sqrt(sum((float(tv[r, p]) - (float(X[r, p]) - float(c[p]))) ** 2 for p in range(X.shape[1])))
        assert abs(n2[r] - ref_n2) <= 1e-12 * ref_n2
        assert abs(err[r] - ref_e) <= 1e-12 * ref_e
    # integers within +-256 are exact in BF16: no rounding error
    Ci = g.integers(-256, 257, (3, 500)).astype(np.float32)
    _, _, e0 = match.bf16_centred(Ci, np.zeros(500, np.float32))
    np.testing.assert_array_equal(e0, 0.0)


def test_triangle_bound_brute_force():
    """|sqrt(D) - sqrt(b)| <= e_m + f_n for every pair (non-integer images,
    so both rows carry rounding error), and the bound is not vacuous."""
    g = np.random.default_rng(2)
    S = g.gamma(2.0, 25.0, (40, 513)).astype(np.float32)
    D = (S[g.integers(0, 40, 30)] * g.uniform(0.9, 1.1, (30, 513))).astype(np.float32)
    c = match.centre_rounded_mean(D)
    Sv, _, e = match.bf16_centred(S, c)
    Dv, _, f = match.bf16_centred(D, c)
    ex = match.distances_direct(S, D)
    b = match.centred_proxy(Sv, Dv)
    dev = np.abs(np.sqrt(ex) - np.sqrt(np.maximum(b, 0)))
    bound = e[:, None] + f[None, :]
    assert np.all(dev <= bound * (1 + 1e-12))
    assert dev.max() > 0.05 * bound.max()


def _argmin_in_topk(b, ex, k):
    top = match.topk(b, k)
    am = match.argmin_first(ex)
    return np.array([am[n] in top[:, n] for n in range(b.shape[1])])


def test_certificate_is_sound_on_random_instances():
    """Whenever the certificate holds, the exact minimiser is among the k
    smallest proxies (brute force over every row)."""
    g = np.random.default_rng(3)
    for trial in range(6):
        M, P = 150, 256
        S = g.gamma(2.0, 20.0, (M, P)).astype(np.float32)
        # near-duplicates around a few rows make close competitors
        for r in range(0, 30, 3):
            S[r + 1] = S[r] * (1 + 1e-3 * g.standard_normal(P)).astype(np.float32)
            S[r + 2] = S[r] * (1 + 1e-3 * g.standard_normal(P)).astype(np.float32)
        D = g.poisson(S[g.integers(0, M, 40)]).astype(np.float32)
        c = match.centre_rounded_mean(D)
        Sv, _, e = match.bf16_centred(S, c)
        Dv, _, f = match.bf16_centred(D, c)
        ex = match.distances_direct(S, D)
        b = match.centred_proxy(Sv, Dv)
        cert = match.centred_certificate(b, e, f, ex, k=8)
        ok = _argmin_in_topk(b, ex, 8)
        assert np.all(ok[cert])
        assert cert.mean() > 0.5


def test_certificate_fails_where_bf16_cannot_separate():
    """Twelve rows that differ only below BF16 resolution: the proxy cannot
    rank them, so an image matching one of them is not certified; images far
    from them are."""
    g = np.random.default_rng(4)
    P = 512
    base = g.gamma(2.0, 100.0, P)
    S = np.stack([base * (1 + 2e-4 * g.standard_normal(P)) for _ in range(12)]
                 + [g.gamma(2.0, 100.0, P) for _ in range(20)]).astype(np.float32)
    D = np.stack([S[5] + 1e-3, S[20]]).astype(np.float32)
    c = np.zeros(P, np.float32)
    Sv, _, e = match.bf16_centred(S, c)
    Dv, _, f = match.bf16_centred(D, c)
    ex = match.distances_direct(S, D)
    cert = match.centred_certificate(match.centred_proxy(Sv, Dv), e, f, ex, k=8)
    np.testing.assert_array_equal(cert, [False, True])


def test_weighted_distances_pins():
    """Per-pixel weights (Eq. (2)'s D; a beam-stop mask is 0/1): unit weights
    give the plain distances; a brute-force double loop agrees; values at
    masked pixels do not matter; scaling one pixel's weight by t scales its
    contribution by t."""
    g = np.random.default_rng(7)
    S = g.gamma(2.0, 10.0, (9, 40))
    D = g.poisson(S[[1, 4, 7]]).astype(np.float64)
    np.testing.assert_allclose(match.distances_weighted(S, D, np.ones(40)),
                               match.distances_direct(S, D), rtol=1e-14)
    w = g.uniform(0.0, 2.0, 40)
    ref = np.zeros((9, 3))
    for m in range(9):
        for n in range(3):
            for p in range(40):
                ref[m, n] += w[p] * (S[m, p] - D[n, p]) ** 2
    np.testing.assert_allclose(match.distances_weighted(S, D, w), ref, rtol=1e-13)
    mask = np.ones(40)
    mask[10:20] = 0.0
    D2 = D.copy()
    D2[:, 10:20] = 1e6
    np.testing.assert_array_equal(match.distances_weighted(S, D, mask),
                                  match.distances_weighted(S, D2, mask))
    w2 = w.copy()
    w2[3] *= 5.0
    delta = match.distances_weighted(S, D, w2) - match.distances_weighted(S, D, w)
    np.testing.assert_allclose(delta, 4.0 * w[3] * (S[:, 3:4] - D[:, 3][None, :]) ** 2, rtol=1e-10)
