"""GPU slicing (type-2 NUFFT, section II-A) against the FP64 oracle with
identical kernel parameters: relative L2 error <= 1e-5 over each output."""
import numpy as np
import pytest
import torch

import synth
import paper_2109_05339_amd as spfel
from oracle import geometry, nufft
from oracle import match as omatch
from tests._common import DEV, rel, gpu, host, model, detector, f32, oracle_slices

pytestmark = pytest.mark.gpu
TOL = 1e-5


def make_plan(N, domain=spfel.REAL, w=6):
    return spfel.Plan(N, kernel_width=w, domain=domain, device=DEV)


def test_real_slices_c1_shape():
    cfg = synth.config(1)
    m = model(1)
    det = detector(cfg.n_det)
    q = synth.quaternions(cfg, "ref_quats", cfg.n_refs)
    plan = make_plan(cfg.n_model)
    plan.set_model(gpu(m))
    s, sn = plan.slice(gpu(q), gpu(det), norms=True)
    torch.cuda.synchronize()
    s, sn = host(s), host(sn)
    rows = np.r_[0:24, cfg.n_refs - 8:cfg.n_refs]        # first, last (ragged tail) rows
    ref = oracle_slices(m, q[rows], det, real=True)
    assert rel(s[rows], ref) <= TOL
    for r in rows:
        assert rel(s[r], ref[list(rows).index(r)]) <= 3 * TOL
    # norms: |s_m|^2 of the float32 output within the float32 sum bound
    exact = (s.astype(np.float64) ** 2).sum(1)
    L = det.shape[0] // 256 + 10
    assert np.all(np.abs(sn - exact) <= omatch.gamma(L) * exact)


def test_complex_slices_random_points_and_ragged_detector():
    N = 13
    m = synth.random_model(5, N, complex_model=True)
    det = np.concatenate([synth.detector_q(10), synth.random_points(5, 37)])  # P = 137
    q = synth.quaternions(synth.config(4), "image_quats", 7)
    plan = make_plan(N, spfel.COMPLEX)
    plan.set_model(gpu(m, torch.complex64))
    s, sn = plan.slice(gpu(q), gpu(det), norms=True)
    s = host(s)
    ref = oracle_slices(m.astype(np.complex64).astype(np.complex128), q, det, real=False)
    assert rel(s, ref) <= TOL
    np.testing.assert_allclose(host(sn), (np.abs(s.astype(np.complex128)) ** 2).sum(1), rtol=1e-5)


@pytest.mark.parametrize("cid,rows", [(2, 3), (5, 2)])
def test_large_grid_shapes(cid, rows):
    """C2 (65^3, 128x128) and C5 (129^3, 256x256) shapes: float64 point
    coordinates keep the high modes within tolerance."""
    cfg = synth.config(cid)
    m = model(cid)
    det = detector(cfg.n_det)
    q = synth.quaternions(cfg, "ref_quats", rows)
    plan = make_plan(cfg.n_model)
    plan.set_model(gpu(m))
    s = host(plan.slice(gpu(q), gpu(det))[0])
    assert rel(s, oracle_slices(m, q, det, real=True)) <= TOL


def test_double_cover_is_bitwise():
    cfg = synth.config(1)
    plan = make_plan(cfg.n_model)
    plan.set_model(gpu(model(1)))
    q = synth.quaternions(cfg, "image_quats", 16)
    det = gpu(detector(cfg.n_det))
    a = host(plan.slice(gpu(q), det)[0])
    b = host(plan.slice(gpu(-q), det)[0])
    np.testing.assert_array_equal(a, b)


def test_friedel_symmetry_and_periodicity():
    cfg = synth.config(1)
    plan = make_plan(cfg.n_model)
    plan.set_model(gpu(model(1)))
    q = synth.quaternions(cfg, "image_quats", 8)
    det = detector(cfg.n_det)
    a = host(plan.slice(gpu(q), gpu(det))[0])
    b = host(plan.slice(gpu(q), gpu(-det))[0])
    assert rel(b, a) <= 2 * TOL
    ident = np.array([[1.0, 0.0, 0.0, 0.0]])
    shift = np.array([2 * np.pi, -2 * np.pi, 4 * np.pi])
    c = host(plan.slice(gpu(ident), gpu(det))[0])
    d = host(plan.slice(gpu(ident), gpu(det + shift))[0])
    assert rel(d, c) <= 2 * TOL


def test_grid_points_reproduce_intensity_samples():
    cfg = synth.Config(99, 1, 11, 12, 8, 1, 1, 1.0)
    m, I = synth.intensity_model(cfg)
    N, h = 11, 5
    j = np.arange(-h, h + 1)
    Q = np.stack(np.meshgrid(j, j, j, indexing="ij"), -1).reshape(-1, 3) * (2 * np.pi / N)
    plan = make_plan(N)
    plan.set_model(gpu(m))
    s = host(plan.slice(gpu(np.array([[1.0, 0, 0, 0]])), gpu(Q))[0])[0]
    assert rel(s, oracle_slices(m, [[1.0, 0, 0, 0]], Q, real=True)[0]) <= TOL
    assert rel(s, I.ravel()) <= 2e-5     # plus the w = 6 algorithmic error


def test_zero_model_gives_exact_zeros():
    plan = make_plan(9)
    plan.set_model(torch.zeros((9, 9, 9), device=DEV))
    s = host(plan.slice(gpu(synth.quaternions(synth.config(1), "ref_quats", 5)), gpu(detector(8)))[0])
    assert np.all(s == 0)


def test_empty_and_nonfinite_inputs():
    plan = make_plan(9)
    plan.set_model(gpu(synth.random_model(1, 9)))
    det = gpu(detector(8))
    s, sn = plan.slice(torch.zeros((0, 4), device=DEV), det, norms=True)
    assert s.shape == (0, 64) and sn.shape == (0,)
    s, sn = plan.slice(gpu(synth.quaternions(synth.config(1), "ref_quats", 3)),
                          torch.zeros((0, 3), device=DEV), norms=True)
    assert s.shape == (3, 0) and np.all(host(sn) == 0)
    q = synth.quaternions(synth.config(1), "ref_quats", 3)
    q[1] = [np.nan, 0, 0, 0]
    q2 = q.copy()
    q2[1] = 0.0
    a = host(plan.slice(gpu(q), det)[0])
    b = host(plan.slice(gpu(q2), det)[0])
    assert np.all(np.isnan(a[1])) and np.all(np.isnan(b[1]))
    assert np.all(np.isfinite(a[[0, 2]]))
    ref = oracle_slices(synth.random_model(1, 9), q[[0, 2]], detector(8), real=True)
    assert rel(a[[0, 2]], ref) <= TOL


def test_state_and_argument_errors():
    plan = make_plan(9)
    det = gpu(detector(8))
    q = gpu(synth.quaternions(synth.config(1), "ref_quats", 2))
    with pytest.raises(spfel.SpfelStateError):
        plan.slice(q, det)
    plan.set_model(gpu(synth.random_model(1, 9)))
    with pytest.raises(TypeError):
        plan.slice(q.double(), det)
    cplan = make_plan(9, spfel.COMPLEX)
    with pytest.raises(TypeError):
        cplan.set_model(gpu(synth.random_model(1, 9), torch.float32))
    plan.close()
    with pytest.raises(spfel.SpfelStateError):
        plan.slice(q, det)


@pytest.mark.parametrize("domain", [spfel.REAL, spfel.COMPLEX])
def test_registered_detector_tiles_are_bitwise_equal_to_generic_path(domain):
    """The tiled LDS-brick kernel reads the same fine-grid values with the
    same weights in the same order as the per-point gather."""
    cfg = synth.config(1)
    det = detector(cfg.n_det)
    q = synth.quaternions(cfg, "ref_quats", 40)
    plan = make_plan(cfg.n_model, domain)
    if domain == spfel.REAL:
        plan.set_model(gpu(model(1)))
    else:
        plan.set_model(gpu(synth.complex_perturbation(synth.config(4), model(1)), torch.complex64))
    plan.set_detector(gpu(det))
    a, an = plan.slice(gpu(q), None, norms=True)
    b, bn = plan.slice(gpu(q), gpu(det), norms=True)
    np.testing.assert_array_equal(host(a), host(b))
    np.testing.assert_array_equal(host(an), host(bn))


@pytest.mark.parametrize("M", [1, 2, 33, 70])
def test_registered_detector_orientation_groups_ragged_and_nonfinite(M):
    """Orientations are walked in groups of 32 per block: group sizes 1, 2,
    32 + 1 and 2 x 32 + 6 over a ragged detector (400 points: one full and
    one partial tile), with a zero and a NaN quaternion inside a group, equal
    the per-point path bit for bit."""
    N = 33
    det = detector(20)
    q = synth.quaternions(synth.config(1), "ref_quats", M)
    if M > 2:
        q[M // 2] = 0.0
        q[M - 2] = [np.nan, 0, 0, 0]
    plan = make_plan(N)
    plan.set_model(gpu(model(1)))
    plan.set_detector(gpu(det))
    a = host(plan.slice(gpu(q))[0])
    b = host(plan.slice(gpu(q), gpu(det))[0])
    np.testing.assert_array_equal(a, b)
    bad = [M // 2, M - 2] if M > 2 else []
    assert np.all(np.isnan(a[bad]))
    good = np.setdiff1d(np.arange(M), bad)
    assert rel(a[good], oracle_slices(model(1), q[good], det, real=True)) <= TOL


@pytest.mark.parametrize("cid,rows", [(2, 4), (5, 2)])
def test_registered_detector_large_shapes_against_oracle(cid, rows):
    cfg = synth.config(cid)
    det = detector(cfg.n_det)
    q = synth.quaternions(cfg, "image_quats", rows)
    plan = make_plan(cfg.n_model)
    plan.set_model(gpu(model(cid)))
    plan.set_detector(gpu(det))
    s = host(plan.slice(gpu(q))[0])
    assert rel(s, oracle_slices(model(cid), q, det, real=True)) <= TOL


def test_registered_scattered_points_use_the_global_fallback():
    """Points spread over the whole cube make every tile's brick exceed the
    LDS budget; the block then gathers from global memory, same values."""
    N = 33
    det = np.concatenate([synth.random_points(21, 700), synth.detector_q(16)])
    q = synth.quaternions(synth.config(1), "ref_quats", 6)
    plan = make_plan(N)
    plan.set_model(gpu(model(1)))
    plan.set_detector(gpu(det))
    a = host(plan.slice(gpu(q))[0])
    b = host(plan.slice(gpu(q), gpu(det))[0])
    np.testing.assert_array_equal(a, b)
    assert rel(a, oracle_slices(model(1), q, det, real=True)) <= TOL
    with pytest.raises(ValueError):
        make_plan(N).slice(gpu(q))


@pytest.mark.parametrize("registered", [False, True])
def test_more_orientations_than_one_rotation_batch(registered):
    """Orientations are sliced in batches of 65,536 (one table of scaled
    rotations per batch): 65,536 + 300 orientations in one call equal the
    two batches sliced in separate calls, bit for bit, and rows on both
    sides of the batch boundary match the oracle."""
    N, cap = 17, 65536
    det = detector(8)                                  # 64 points
    q = synth.quaternions(synth.config(1), "ref_quats", cap + 300)
    m = synth.random_model(8, N)
    plan = make_plan(N)
    plan.set_model(gpu(m))
    if registered:
        plan.set_detector(gpu(det))
    dq = None if registered else gpu(det)
    qt = gpu(q)
    whole = host(plan.slice(qt, dq)[0])
    first = host(plan.slice(qt[:cap].contiguous(), dq)[0])
    second = host(plan.slice(qt[cap:].contiguous(), dq)[0])
    np.testing.assert_array_equal(whole, np.concatenate([first, second]))
    rows = np.r_[0:2, cap - 2:cap + 2, cap + 298:cap + 300]
    assert rel(whole[rows], oracle_slices(m, q[rows], det, real=True)) <= TOL


@pytest.mark.parametrize("w,bw", [(4, 2.30), (5, 2.30), (7, 2.30), (8, 2.30), (6, 1.80)])
def test_other_kernel_widths_and_shapes(w, bw):
    """Every compiled kernel width, and a different ES shape, on both the
    per-point and the tiled path, against the oracle with the same w, beta
    and n_f (slices) and for the adjoint (merge)."""
    N = 21
    m = synth.random_model(9, N)
    det = detector(16)
    q = synth.quaternions(synth.config(1), "ref_quats", 6)
    plan = spfel.Plan(N, kernel_width=w, beta_over_w=bw, device=DEV)
    plan.set_model(gpu(m))
    x = geometry.slice_points(f32(q), f32(det)).reshape(-1, 3)
    ref = nufft.nufft2(m, x, w=w, beta_over_w=bw, real=True).reshape(len(q), -1)
    a = host(plan.slice(gpu(q), gpu(det))[0])
    assert rel(a, ref) <= TOL
    plan.set_detector(gpu(det))
    np.testing.assert_array_equal(host(plan.slice(gpu(q))[0]), a)
    y = np.random.default_rng(w).standard_normal((len(q), len(det))).astype(np.float32)
    out = host(plan.merge_adjoint(gpu(q), gpu(det), gpu(y)))
    assert rel(out, nufft.nufft1(y.astype(np.float64).reshape(-1), x, N, w=w, beta_over_w=bw,
                                 real=True)) <= TOL
