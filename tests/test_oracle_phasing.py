"""CPU pins of the phasing oracle (section II-D: ER, HIO, shrinkwrap)."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import phasing as ph


def blob_object(seed: int, N: int = 16):
    """A smooth positive density on a compact irregular support (the cells
    above 5% of its maximum), its amplitudes and support."""
    g = np.random.default_rng(seed)
    raw = np.zeros((N, N, N))
    raw[4:11, 5:12, 4:10] = g.random((7, 7, 6))
    rho = ph.blur(raw, 0.7)
    sup = rho > 0.05 * rho.max()
    rho = np.where(sup, rho, 0.0)
    return rho, np.abs(np.fft.fftn(rho)), sup


def aligned_error(r, t):
    """Relative error of r against t up to the trivial ambiguities of
    phasing (circular translation and centro-inversion)."""
    best = np.inf
    Ft = np.fft.fftn(t)
    for cand in (r, np.roll(r[::-1, ::-1, ::-1], 1, axis=(0, 1, 2))):
        cc = np.fft.ifftn(np.fft.fftn(cand) * np.conj(Ft)).real
        s = np.unravel_index(np.argmax(cc), cc.shape)
        al = np.roll(cand, [-s[0], -s[1], -s[2]], axis=(0, 1, 2))
        best = min(best, np.linalg.norm(al - t) / np.linalg.norm(t))
    return best


def test_projection_keeps_a_consistent_object_and_imposes_amplitudes():
    rho, A, sup = blob_object(0)
    rp, F = ph.fourier_projection(rho, A)
    np.testing.assert_allclose(rp, rho, atol=1e-12 * rho.max())
    assert ph.fourier_error(F, A) < 1e-28
    # any real input: the output carries the amplitudes A, and a second
    # projection changes nothing (A is Friedel-symmetric)
    x = np.random.default_rng(1).standard_normal(rho.shape)
    p1, _ = ph.fourier_projection(x, A)
    np.testing.assert_allclose(np.abs(np.fft.fftn(p1)), A, atol=1e-10 * A.max())
    p2, _ = ph.fourier_projection(p1, A)
    np.testing.assert_allclose(p2, p1, atol=1e-10 * np.abs(p1).max())


def test_unmeasured_coefficients_are_kept():
    rho, A, _ = blob_object(1)
    N = rho.shape[0]
    k = np.fft.fftfreq(N) * N
    K = np.sqrt(k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2)
    measured = K > 1.5                        # a beam stop: low |k| unmeasured (Friedel-symmetric)
    x = np.random.default_rng(2).standard_normal(rho.shape)
    p, _ = ph.fourier_projection(x, A, measured)
    Fx, Fp = np.fft.fftn(x), np.fft.fftn(p)
    np.testing.assert_allclose(Fp[~measured], Fx[~measured], atol=1e-10 * np.abs(Fx).max())
    np.testing.assert_allclose(np.abs(Fp[measured]), A[measured], atol=1e-10 * A.max())


def test_true_object_is_a_fixed_point():
    rho, A, sup = blob_object(2)
    for step in (lambda r: ph.er_step(r, A, sup), lambda r: ph.hio_step(r, A, sup, 0.9)):
        r, e = step(rho)
        np.testing.assert_allclose(r, rho, atol=1e-12 * rho.max())
        assert e < 1e-28


def test_error_reduction_never_increases_the_error():
    rho, A, sup = blob_object(3)
    r = np.random.default_rng(4).random(rho.shape) * sup
    errs = []
    for _ in range(40):
        r, e = ph.er_step(r, A, sup)
        errs.append(e)
    errs = np.array(errs)
    assert np.all(errs[1:] <= errs[:-1] * (1 + 1e-12))
    assert errs[-1] < errs[0]


@pytest.mark.parametrize("seed", [0, 3])
def test_hio_then_er_recovers_the_object(seed):
    """From a random start inside the support, HIO then ER reach amplitudes
    and support both satisfied and the object itself up to translation and
    inversion (a sign or index slip in either step stalls this)."""
    rho, A, sup = blob_object(seed)
    r = np.random.default_rng(seed + 10).random(rho.shape) * sup
    for _ in range(300):
        r, e = ph.hio_step(r, A, sup, 0.9)
    for _ in range(100):
        r, e = ph.er_step(r, A, sup)
    assert e < 1e-6
    assert aligned_error(r, rho) < 5e-3


def test_gaussian_kernel_and_blur():
    N, sigma = 9, 1.3
    g = ph.gaussian_kernel_1d(N, sigma)
    assert abs(g.sum() - 1) < 1e-15 and np.all(g[1:] == g[1:][::-1])
    # blur of a unit impulse at the origin is the separable kernel
    d = np.zeros((N, N, N))
    d[0, 0, 0] = 1.0
    np.testing.assert_allclose(ph.blur(d, sigma), np.einsum("i,j,k->ijk", g, g, g), atol=1e-16)
    # scipy's wrapped Gaussian filter with the kernel reaching every offset
    # once (odd N) is the same periodic convolution
    x = np.random.default_rng(5).random((N, N, N))
    ref = ndimage.gaussian_filter(x, sigma, mode="wrap", truncate=(N // 2) / sigma)
    np.testing.assert_allclose(ph.blur(x, sigma), ref, rtol=1e-12, atol=1e-14)
    assert abs(ph.blur(x, sigma).sum() - x.sum()) < 1e-10


def test_shrinkwrap_of_a_ball_is_the_ball():
    N = 16
    c = np.arange(N) - 8
    R2 = c[:, None, None] ** 2 + c[None, :, None] ** 2 + c[None, None, :] ** 2
    ball = R2 <= 16
    s = ph.shrinkwrap(ball.astype(float), 0.3, 0.5)
    np.testing.assert_array_equal(s, ball)
    # a wider blur grows the support
    assert ph.shrinkwrap(ball.astype(float), 1.5, 0.1).sum() > ball.sum()
