"""GPU type-1 adjoint (merging A*, section II-C Eq. (2)) against the FP64
oracle with identical parameters, plus the adjointness identity on the GPU."""
import numpy as np
import pytest
import torch

import synth
import paper_2109_05339_amd as spfel
from oracle import geometry, nufft
from tests._common import DEV, rel, gpu, host, model, detector, f32

pytestmark = pytest.mark.gpu
TOL = 1e-5


def oracle_merge(y, quats, det, N, real, weights=None):
    x = geometry.slice_points(f32(quats), f32(det)).reshape(-1, 3)
    yy = np.asarray(y).reshape(-1)
    if weights is not None:
        yy = yy * np.asarray(weights, dtype=np.float64).reshape(-1)
    return nufft.nufft1(yy, x, N, real=real)


def test_real_merge_c1_shape():
    cfg = synth.config(1)
    det = detector(cfg.n_det)
    q = synth.quaternions(cfg, "image_quats", 24)
    g = np.random.default_rng(1)
    y = (g.poisson(20.0, (24, det.shape[0]))).astype(np.float32)
    plan = spfel.Plan(cfg.n_model, device=DEV)
    out = host(plan.merge_adjoint(gpu(q), gpu(det), gpu(y)))
    assert rel(out, oracle_merge(y, q, det, cfg.n_model, True)) <= TOL


def test_complex_merge_with_weights_ragged():
    N = 13
    det = np.concatenate([synth.detector_q(9), synth.random_points(3, 20)])
    q = synth.quaternions(synth.config(4), "image_quats", 5)
    g = np.random.default_rng(2)
    y = (g.standard_normal((5, len(det))) + 1j * g.standard_normal((5, len(det)))).astype(np.complex64)
    w = synth.pixel_weights(synth.config(4), 5, len(det))
    plan = spfel.Plan(N, domain=spfel.COMPLEX, device=DEV)
    out = host(plan.merge_adjoint(gpu(q), gpu(det), gpu(y, torch.complex64), gpu(w)))
    assert rel(out, oracle_merge(y.astype(np.complex128), q, det, N, False, w)) <= TOL


def test_c4_shape_complex():
    cfg = synth.config(4)
    det = detector(cfg.n_det)
    q = synth.quaternions(cfg, "image_quats", 16)
    g = np.random.default_rng(3)
    y = (g.standard_normal((16, det.shape[0])) + 1j * g.standard_normal((16, det.shape[0]))).astype(np.complex64)
    plan = spfel.Plan(cfg.n_model, domain=spfel.COMPLEX, device=DEV)
    out = host(plan.merge_adjoint(gpu(q), gpu(det), gpu(y, torch.complex64)))
    assert rel(out, oracle_merge(y.astype(np.complex128), q, det, cfg.n_model, False)) <= TOL


@pytest.mark.parametrize("domain", [spfel.REAL, spfel.COMPLEX])
def test_gpu_adjointness(domain):
    N = 33
    det = detector(64)
    q = synth.quaternions(synth.config(1), "image_quats", 12)
    g = np.random.default_rng(4)
    plan = spfel.Plan(N, domain=domain, device=DEV)
    if domain == spfel.REAL:
        m = g.standard_normal((N,) * 3).astype(np.float32)
        y = g.standard_normal((12, det.shape[0])).astype(np.float32)
        dt = torch.float32
    else:
        m = (g.standard_normal((N,) * 3) + 1j * g.standard_normal((N,) * 3)).astype(np.complex64)
        y = (g.standard_normal((12, det.shape[0])) + 1j * g.standard_normal((12, det.shape[0]))).astype(np.complex64)
        dt = torch.complex64
    plan.set_model(gpu(m, dt))
    s = host(plan.slice(gpu(q), gpu(det))[0]).astype(np.complex128)
    f = host(plan.merge_adjoint(gpu(q), gpu(det), gpu(y, dt))).astype(np.complex128)
    lhs = np.vdot(y.astype(np.complex128).ravel(), s.ravel())
    rhs = np.vdot(f.ravel(), m.astype(np.complex128).ravel())
    assert abs(lhs - rhs) <= TOL * np.linalg.norm(s) * np.linalg.norm(y)


def test_defer_and_accumulate_flags():
    N = 13
    det = detector(12)
    q = synth.quaternions(synth.config(1), "image_quats", 10)
    g = np.random.default_rng(5)
    y = g.standard_normal((10, det.shape[0])).astype(np.float32)
    plan = spfel.Plan(N, device=DEV)
    one = host(plan.merge_adjoint(gpu(q), gpu(det), gpu(y)))
    plan.merge_adjoint(gpu(q[:4]), gpu(det), gpu(y[:4]), flags=spfel.MERGE_DEFER)
    two = host(plan.merge_adjoint(gpu(q[4:]), gpu(det), gpu(y[4:])))
    assert rel(two, one) <= TOL
    base = gpu(np.ones((N,) * 3, np.float32))
    plan.merge_adjoint(gpu(q), gpu(det), gpu(y), out=base, flags=spfel.MERGE_ACCUMULATE)
    assert rel(host(base) - 1.0, one) <= TOL
    empty = host(plan.merge_adjoint(torch.zeros((0, 4), device=DEV), gpu(det),
                                    torch.zeros((0, det.shape[0]), device=DEV)))
    assert np.all(empty == 0)


@pytest.mark.parametrize("domain", [spfel.REAL, spfel.COMPLEX])
def test_registered_detector_spread_against_oracle(domain):
    cfg = synth.config(1)
    det = detector(cfg.n_det)
    q = synth.quaternions(cfg, "image_quats", 30)
    g = np.random.default_rng(6)
    plan = spfel.Plan(cfg.n_model, domain=domain, device=DEV)
    plan.set_detector(gpu(det))
    w = synth.pixel_weights(cfg, 30, det.shape[0])
    if domain == spfel.REAL:
        y = g.poisson(20.0, (30, det.shape[0])).astype(np.float32)
        yt = gpu(y)
    else:
        y = (g.standard_normal((30, det.shape[0])) + 1j * g.standard_normal((30, det.shape[0]))).astype(np.complex64)
        yt = gpu(y, torch.complex64)
    out = host(plan.merge_adjoint(gpu(q), None, yt, gpu(w)))
    ref = oracle_merge(y.astype(np.complex128) if domain else y, q, det, cfg.n_model, domain == spfel.REAL, w)
    assert rel(out, ref) <= TOL
    gen = host(plan.merge_adjoint(gpu(q), gpu(det), yt, gpu(w)))
    assert rel(out, gen) <= 1e-6


def test_registered_detector_spread_c4_shape_and_fallback():
    cfg = synth.config(4)
    det = detector(cfg.n_det)
    q = synth.quaternions(cfg, "image_quats", 12)
    g = np.random.default_rng(8)
    y = (g.standard_normal((12, det.shape[0])) + 1j * g.standard_normal((12, det.shape[0]))).astype(np.complex64)
    plan = spfel.Plan(cfg.n_model, domain=spfel.COMPLEX, device=DEV)
    plan.set_detector(gpu(det))
    out = host(plan.merge_adjoint(gpu(q), None, gpu(y, torch.complex64)))
    assert rel(out, oracle_merge(y.astype(np.complex128), q, det, cfg.n_model, False)) <= TOL
    scat = synth.random_points(22, 600)
    plan2 = spfel.Plan(13, device=DEV)
    plan2.set_detector(gpu(scat))
    yr = g.standard_normal((3, 600)).astype(np.float32)
    q3 = synth.quaternions(cfg, "ref_quats", 3)
    out2 = host(plan2.merge_adjoint(gpu(q3), None, gpu(yr)))
    assert rel(out2, oracle_merge(yr, q3, scat, 13, True)) <= TOL
