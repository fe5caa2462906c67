"""The merge and the gradient at the image counts and grids the bench runs:
the type-1 adjoint (merging A*, section II-C Eq. (2)) of all 2,048 images of
workload 2 (every image adds to the q ~ 0 cells, so the float32 atomic sums
there are 2,048 deep) and of 256 images on the 129^3 / 258^3 grid of
workload 5; a merge of more images than one binning batch holds; and the
weighted-loss gradient of the 65^3 complex model of workload 4 against the
FP64 oracle and against central differences.  All
through the registered-detector (tiled matrix-core spread) path; inputs are
made without the library, expected values by the oracle only."""
import numpy as np
import pytest
import torch

import synth
import paper_2109_05339_amd as spfel
from oracle import geometry, grad as ograd, nufft
from tests._common import DEV, rel, gpu, host, model, detector, f32, molecule_slices

pytestmark = pytest.mark.gpu
TOL = 1e-5


def poisson_images(cid, n):
    """Poisson images of the workload's molecule at its first n image
    orientations (intensity evaluated directly, scaled to the photon mean)."""
    cfg = synth.config(cid)
    q = synth.quaternions(cfg, "image_quats", n)
    lam = host(molecule_slices(cid, q, detector(cfg.n_det)))
    lam *= synth.photon_scale(lam, cfg.photons)
    return q, synth.poisson_counts(cfg, lam)


def oracle_merge_chunked(y, q, det, N, chunk):
    """Type-1 oracle summed over image chunks (it is linear in the values)."""
    out = 0.0
    for c0 in range(0, len(q), chunk):
        x = geometry.slice_points(f32(q[c0:c0 + chunk]), f32(det)).reshape(-1, 3)
        out = out + nufft.nufft1(np.asarray(y[c0:c0 + chunk], np.float64).ravel(), x, N, real=True)
    return out


def test_merge_all_workload2_images():
    cfg = synth.config(2)
    det = detector(cfg.n_det)
    q, y = poisson_images(2, cfg.n_images)
    plan = spfel.Plan(cfg.n_model, device=DEV)
    plan.set_detector(gpu(det))
    out = host(plan.merge_adjoint(gpu(q), None, gpu(y)))
    ref = oracle_merge_chunked(y, q, det, cfg.n_model, 256)
    err = rel(out, ref)
    print(f"merge of {cfg.n_images} images at 65^3: rel L2 {err:.2e}")
    assert err <= TOL


def test_merge_workload5_grid():
    cfg = synth.config(5)
    det = detector(cfg.n_det)
    q, y = poisson_images(5, 256)
    plan = spfel.Plan(cfg.n_model, device=DEV)
    plan.set_detector(gpu(det))
    out = host(plan.merge_adjoint(gpu(q), None, gpu(y)))
    ref = oracle_merge_chunked(y, q, det, cfg.n_model, 256)
    err = rel(out, ref)
    print(f"merge of 256 images at 129^3: rel L2 {err:.2e}")
    assert err <= TOL


def workload4_inputs(n):
    """Complex 65^3 model (workload 2's intensity model plus the seeded
    complex perturbation), scaled to the photon level of images that are the
    molecule's intensity at the first n image orientations; per-pixel
    weights in [0.5, 1)."""
    cfg = synth.config(4)
    det = detector(cfg.n_det)
    q = synth.quaternions(cfg, "image_quats", n)
    lam = host(molecule_slices(4, q, det))
    alpha = synth.photon_scale(lam, cfg.photons)
    d = (alpha * lam).astype(np.complex64)
    m = (alpha * synth.complex_perturbation(cfg, model(2))).astype(np.complex64)
    w = synth.pixel_weights(cfg, n, cfg.n_pix)
    return cfg, det, q, d, m, w


def gpu_loss_and_grad(plan, m, q, d, w, chunk=1024):
    mt = gpu(m, torch.complex64).requires_grad_(True)
    L = spfel.slice_loss(mt, gpu(q), None, gpu(d, torch.complex64), gpu(w), plan, chunk=chunk)
    L.backward()
    return float(L.detach()), host(mt.grad)


def test_workload4_gradient_against_oracle():
    cfg, det, q, d, m, w = workload4_inputs(256)
    plan = spfel.Plan(cfg.n_model, domain=spfel.COMPLEX, device=DEV)
    plan.set_detector(gpu(det))
    L, g = gpu_loss_and_grad(plan, m, q, d, w, chunk=128)
    x = geometry.slice_points(f32(q), f32(det)).reshape(-1, 3)
    m64, d64, w64 = m.astype(np.complex128), d.astype(np.complex128).ravel(), f32(w).ravel()
    Lref = ograd.loss(m64, x, d64, w64)
    gref = ograd.grad(m64, x, d64, w64)
    err = rel(g, gref)
    print(f"workload-4 gradient over 256 images: loss rel err {abs(L - Lref) / Lref:.2e}, "
          f"gradient rel L2 {err:.2e}")
    assert abs(L - Lref) <= 1e-4 * Lref
    assert err <= 1e-4


def test_workload4_gradient_against_central_differences():
    """All 4,096 images: the loss is quadratic in the model, so central
    differences of the GPU loss equal its gradient for any step h up to
    rounding.  The 64 voxels are set to zero first, so that the perturbed
    values +-h and +-ih are exact in complex64; h is a power of two near 1%
    of the data scale, far above the loss's rounding."""
    n = synth.config(4).n_images
    cfg, det, q, d, m, w = workload4_inputs(n)
    vox = synth.fd_voxels(cfg, 64)
    m = m.copy()
    m.reshape(-1)[vox] = 0
    plan = spfel.Plan(cfg.n_model, domain=spfel.COMPLEX, device=DEV)
    plan.set_detector(gpu(det))
    _, g = gpu_loss_and_grad(plan, m, q, d, w)
    qt, dt, wt = gpu(q), gpu(d, torch.complex64), gpu(w)

    def loss_at(mm):
        plan.set_model(gpu(mm, torch.complex64))
        acc = torch.zeros((), dtype=torch.float64, device=DEV)
        for c0 in range(0, n, 1024):
            s, _ = plan.slice(qt[c0:c0 + 1024])
            plan.weighted_residual(s, dt[c0:c0 + 1024], wt[c0:c0 + 1024], residual=False, loss=acc)
        return float(acc)

    h = 2.0 ** round(np.log2(0.01 * float(np.sqrt(np.mean(np.abs(d) ** 2)))))
    flat = m.reshape(-1)
    fd = np.empty(len(vox), np.complex128)
    for i, v in enumerate(vox):
        parts = []
        for dirn in (1.0, 1j):
            mp, mm = flat.copy(), flat.copy()
            mp[v] = h * dirn
            mm[v] = -h * dirn
            parts.append((loss_at(mp.reshape(m.shape)) - loss_at(mm.reshape(m.shape))) / (2 * h))
        fd[i] = parts[0] + 1j * parts[1]
    gv = g.reshape(-1)[vox].astype(np.complex128)
    worst = np.max(np.abs(gv - fd)) / np.abs(g).max()
    print(f"central differences on 64 voxels over {n} images (h = {h:g}): "
          f"max |fd - grad| / max|grad| {worst:.2e}")
    assert worst <= 1e-3


@pytest.mark.parametrize("real", [True, False])
def test_merge_across_binning_batches(real):
    """66,536 images of a 2 x 2 detector: more images than one binning batch
    takes (at most 65,536), so the merge runs two batches.  Against the
    oracle over all images, and equal to the sum of the merges of its two
    single-batch parts up to float32 rounding (a batch that read another
    batch's images or values would break both).  Both domains: they stage
    their points in different layouts."""
    N, n = 13, 65536 + 1000
    det = detector(2)
    q = synth.quaternions(synth.config(1), "image_quats", n)
    g = np.random.default_rng(31)
    if real:
        y = g.random((n, len(det))).astype(np.float32)
        yt = gpu(y)
    else:
        y = (g.random((n, len(det))) + 1j * g.standard_normal((n, len(det)))).astype(np.complex64)
        yt = gpu(y, torch.complex64)
    plan = spfel.Plan(N, domain=spfel.REAL if real else spfel.COMPLEX, device=DEV)
    plan.set_detector(gpu(det))
    whole = host(plan.merge_adjoint(gpu(q), None, yt))
    a = host(plan.merge_adjoint(gpu(q[:65536]), None, yt[:65536].contiguous()))
    b = host(plan.merge_adjoint(gpu(q[65536:]), None, yt[65536:].contiguous()))
    assert rel(whole, a + b) <= TOL
    x = geometry.slice_points(f32(q), f32(det)).reshape(-1, 3)
    ref = nufft.nufft1(y.astype(np.float64 if real else np.complex128).ravel(), x, N, real=real)
    err = rel(whole, ref)
    print(f"merge of {n} images over two batches ({'real' if real else 'complex'}): rel L2 {err:.2e}")
    assert err <= TOL
