"""Pins of the oracle's matching (brute force, ties, bounds, BF16 rounding,
top-k certificate), the gradient (finite differences) and the synthetic
image generator."""
import numpy as np
import pytest
import torch

import synth
from oracle import match, grad, nufft, geometry


def test_expanded_equals_direct_and_brute_force_argmin():
    g = np.random.default_rng(0)
    S = g.standard_normal((40, 64))
    D = g.standard_normal((15, 64))
    Dd = match.distances_direct(S, D)
    De = match.distances_expanded(S, D)
    np.testing.assert_allclose(De, Dd, rtol=1e-12, atol=1e-10)
    am = match.argmin_first(Dd)
    for n in range(D.shape[0]):
        best = min(range(S.shape[0]), key=lambda m: (np.sum((S[m] - D[n]) ** 2), m))
        assert am[n] == best


def test_argmin_ties_go_to_lowest_index_and_self_match():
    g = np.random.default_rng(1)
    S = g.standard_normal((10, 32))
    S[7] = S[3]               # duplicate model image: tie between 3 and 7
    D = np.stack([S[3], S[5], S[9]])
    Dd = match.distances_direct(S, D)
    np.testing.assert_array_equal(match.argmin_first(Dd), [3, 5, 9])
    b1, b2 = match.top2(Dd)
    np.testing.assert_array_equal(b1, 0.0)
    assert b2[0] == 0.0 and b2[1] > 0 and b2[2] > 0


def test_topk_order_and_ties():
    Dm = np.array([[3.0, 1.0], [1.0, 1.0], [2.0, 0.5], [1.0, 7.0]])
    np.testing.assert_array_equal(match.topk(Dm, 3), [[1, 2], [3, 0], [2, 1]])


def test_bf16_round_matches_torch():
    g = np.random.default_rng(2)
    x = np.concatenate([g.standard_normal(20000).astype(np.float32) * 100,
                        np.array([1.0, 1.00390625, 1.005859375, 1.001953125, -2.998046875, 0.0, 65504.0], np.float32)])
    # add exact ties: values halfway between two bf16 numbers
    base = (g.integers(0, 2 ** 15, 1000).astype(np.uint32) << 16) | 0x8000
    x = np.concatenate([x, base.view(np.float32)[np.isfinite(base.view(np.float32))]])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(match.bf16_round(x), ref)


def test_fp32_distance_bound_holds_and_is_not_vacuous():
    g = np.random.default_rng(3)
    P = 4096
    S = (50 + 10 * g.standard_normal((30, P))).astype(np.float32)
    D = (50 + 10 * g.standard_normal((20, P))).astype(np.float32)
    exact = match.distances_expanded(S, D)
    s32 = (S * S).sum(axis=1, dtype=np.float32)
    d32 = (D * D).sum(axis=1, dtype=np.float32)
    dot32 = np.empty((30, 20), np.float32)
    for m in range(30):          # FP32 dot products: chains of at most P
        dot32[m] = (S[m][None, :] * D).sum(axis=1, dtype=np.float32)
    fl = (s32[:, None] + d32[None, :]) - np.float32(2) * dot32
    absdot = np.abs(S.astype(np.float64)) @ np.abs(D.astype(np.float64)).T
    bnd = match.fp32_distance_bound((S.astype(np.float64) ** 2).sum(1)[:, None], (D.astype(np.float64) ** 2).sum(1)[None, :], absdot, P + 3)
    assert np.all(np.abs(fl - exact) <= bnd)
    assert np.median(bnd / np.abs(exact)) < 0.5


def test_gradient_matches_central_differences():
    """The loss is quadratic in m, so central differences equal the analytic
    gradient up to rounding."""
    N = 7
    g = np.random.default_rng(5)
    m = g.standard_normal((N,) * 3) + 1j * g.standard_normal((N,) * 3)
    q = synth.quaternions(synth.config(4), "image_quats", 3)
    x = geometry.slice_points(q, synth.detector_q(10)).reshape(-1, 3)
    d = g.standard_normal(len(x)) + 1j * g.standard_normal(len(x))
    wts = 0.5 + 0.5 * g.random(len(x))
    gr = grad.grad(m, x, d, wts)
    vox = np.array([0, 17, 100, 171, 342])
    fd = grad.fd_grad(m, x, d, wts, vox, h=1e-3)
    np.testing.assert_allclose(fd, gr.reshape(-1)[vox], rtol=1e-9, atol=1e-9 * np.abs(gr).max())


def test_gradient_is_zero_at_exact_fit():
    N = 7
    g = np.random.default_rng(6)
    m = g.standard_normal((N,) * 3) + 1j * g.standard_normal((N,) * 3)
    x = synth.random_points(6, 300)
    d = nufft.nufft2(m, x)
    assert grad.loss(m, x, d, np.ones(len(x))) <= 1e-20
    assert np.abs(grad.grad(m, x, d, np.ones(len(x)))).max() <= 1e-10


def test_synthetic_images_have_target_photon_mean():
    cfg = synth.config(1)
    m, _ = synth.intensity_model(cfg)
    q = synth.quaternions(cfg, "image_quats", 8)
    det = synth.detector_q(cfg.n_det)
    x = geometry.slice_points(q, det).reshape(-1, 3)
    lam0 = np.maximum(nufft.nufft2(m, x, real=True), 0)
    alpha = synth.photon_scale(lam0, cfg.photons)
    lam = alpha * lam0
    assert lam.mean() == pytest.approx(cfg.photons, rel=1e-12)
    d = synth.poisson_counts(cfg, lam)
    assert d.mean() == pytest.approx(cfg.photons, rel=0.01)
    np.testing.assert_array_equal(d, np.round(d))


def test_prefix_stability_of_streams():
    cfg = synth.config(1)
    a = synth.quaternions(cfg, "ref_quats", 100)
    b = synth.quaternions(synth.config(3), "ref_quats", 500)
    np.testing.assert_array_equal(a, b[:100])
    lam = np.full(4000, 20.0)
    np.testing.assert_array_equal(synth.poisson_counts(cfg, lam[:1000]), synth.poisson_counts(cfg, lam)[:1000])
