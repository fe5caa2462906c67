"""Pins of the oracle's ES kernel, its Fourier transform and the geometry."""
import numpy as np
import pytest
from scipy import integrate
from scipy.spatial.transform import Rotation

import synth
from oracle import es, geometry


def test_es_kernel_values():
    w, beta = 6, 2.30 * 6
    assert es.es_kernel(0.0, w, beta) == pytest.approx(1.0, abs=0)
    # edge of the support: sqrt(0) -> exp(-beta); outside: 0
    assert es.es_kernel(3.0, w, beta) == pytest.approx(np.exp(-beta), rel=1e-15)
    assert es.es_kernel(-3.0, w, beta) == pytest.approx(np.exp(-beta), rel=1e-15)
    assert es.es_kernel(3.0 + 1e-12, w, beta) == 0.0
    t = np.linspace(-3, 3, 101)
    np.testing.assert_array_equal(es.es_kernel(t, w, beta), es.es_kernel(-t, w, beta))
    # a hand value: tau = 1.5 -> z = 0.5 -> exp(beta (sqrt(0.75) - 1))
    assert es.es_kernel(1.5, w, beta) == pytest.approx(np.exp(beta * (np.sqrt(0.75) - 1)), rel=1e-15)


@pytest.mark.parametrize("w,nf", [(6, 66), (6, 130), (7, 258), (14, 34)])
def test_es_hat_against_adaptive_quadrature(w, nf):
    """psi_hat by Gauss-Legendre vs scipy's adaptive quadrature of the same
    integral in the substituted variable tau = (w/2) sin(theta), which
    removes the square-root endpoint behaviour."""
    beta = 2.30 * w
    ks = np.array([0, 1, 5, nf // 4, nf // 2 - 1])
    got = es.es_hat(ks, w, beta, nf)

    def integrand(th, k):
        tau = 0.5 * w * np.sin(th)
        return np.exp(beta * (np.cos(th) - 1.0)) * np.cos(2 * np.pi * k * tau / nf) * 0.5 * w * np.cos(th)

    ref = np.array([integrate.quad(integrand, -np.pi / 2, np.pi / 2, args=(k,), epsabs=1e-16, epsrel=1e-13, limit=200)[0] for k in ks])
    np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-14)


def test_quat_to_R_matches_scipy_and_is_a_rotation():
    q = synth.quaternions(synth.config(1), "ref_quats", 50)
    R = geometry.quat_to_R(q)
    ref = Rotation.from_quat(np.c_[q[:, 1:], q[:, :1]]).as_matrix()  # scipy is scalar-last
    np.testing.assert_allclose(R, ref, atol=1e-14)
    I = np.einsum("mij,mkj->mik", R, R)
    np.testing.assert_allclose(I, np.broadcast_to(np.eye(3), I.shape), atol=1e-14)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-13)


def test_quat_known_rotation_double_cover_and_normalisation():
    c = np.cos(np.pi / 4)
    qz = np.array([[c, 0.0, 0.0, c]])        # 90 degrees about z
    R = geometry.quat_to_R(qz)[0]
    np.testing.assert_allclose(R @ [1, 0, 0], [0, 1, 0], atol=1e-15)
    np.testing.assert_allclose(R @ [0, 1, 0], [-1, 0, 0], atol=1e-15)
    q = synth.quaternions(synth.config(2), "image_quats", 20)
    np.testing.assert_array_equal(geometry.quat_to_R(q), geometry.quat_to_R(-q))
    np.testing.assert_allclose(geometry.quat_to_R(3.7 * q), geometry.quat_to_R(q), atol=1e-15)


def test_quaternion_product_composes_rotations():
    """Hamilton product: R(a (x) b) = R(a) R(b)."""
    a, b = synth.quaternions(synth.config(1), "image_quats", 2)
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    ab = np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                   w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                   w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                   w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])
    Ra, Rb, Rab = geometry.quat_to_R(np.stack([a, b, ab]))
    np.testing.assert_allclose(Rab, Ra @ Rb, atol=1e-14)


def test_slice_points_is_rotation_of_template():
    q = synth.quaternions(synth.config(1), "ref_quats", 3)
    det = synth.detector_q(8)
    x = geometry.slice_points(q, det)
    R = geometry.quat_to_R(q)
    for m in range(3):
        np.testing.assert_allclose(x[m], det @ R[m].T, atol=1e-15)
        np.testing.assert_allclose(np.linalg.norm(x[m], axis=1), np.linalg.norm(det, axis=1), atol=1e-14)


def test_detector_on_ewald_sphere():
    n = 64
    q = synth.detector_q(n)
    assert q.shape == (n * n, 3)
    r = np.linalg.norm(q, axis=1)
    assert r.max() == pytest.approx(0.9 * np.pi, rel=1e-15)
    # the four corners are the farthest pixels
    corners = [0, n - 1, n * (n - 1), n * n - 1]
    np.testing.assert_allclose(r[corners], 0.9 * np.pi, rtol=1e-14)
    # q = k (s_hat - z_hat) lies on the sphere |q + k z_hat| = k
    k = 0.9 * np.pi / np.linalg.norm(np.array([(n - 1) / 2, (n - 1) / 2, 2 * n]) / np.linalg.norm([(n - 1) / 2, (n - 1) / 2, 2 * n]) - [0, 0, 1])
    np.testing.assert_allclose(np.linalg.norm(q + [0, 0, k], axis=1), k, rtol=1e-13)
    assert np.all(q[:, 2] <= 0)
    # pixel (r, c) -> p = r n + c with c along x
    assert q[1, 0] > q[0, 0] and q[n, 1] > q[0, 1]
