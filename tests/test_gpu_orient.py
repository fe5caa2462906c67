"""The two-stream slice->match pipeline (spfel_orient) gives exactly the
result of slicing each chunk (centring it, in BF16 mode) and matching it into
the running best."""
import functools

import numpy as np
import pytest
import torch

import synth
import paper_2109_05339_amd as spfel
from tests._common import DEV, gpu, host, model, detector, molecule_slices

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def inputs():
    cfg = synth.config(1)
    plan = spfel.Plan(cfg.n_model, device=DEV)
    plan.set_detector(gpu(detector(cfg.n_det)))
    lam = host(molecule_slices(1, synth.quaternions(cfg, "image_quats", 300), detector(cfg.n_det)))
    alpha = synth.photon_scale(lam, cfg.photons)
    images = gpu(synth.poisson_counts(cfg, alpha * lam))
    plan.set_model(gpu(alpha * model(1)))
    return plan, gpu(synth.quaternions(cfg, "ref_quats", 1000)), images


def prepared(images, mode):
    return spfel.ImagesF32(images) if mode == spfel.MATCH_FP32 else spfel.ImagesBF16(images)


def reference(plan, q, images, mode, chunk):
    im = prepared(images, mode)
    bi, bd = spfel.new_best(images.shape[0], DEV)
    fl = torch.zeros(images.shape[0], dtype=torch.int32, device=DEV)
    for c0 in range(0, q.shape[0], chunk):
        if mode == spfel.MATCH_FP32:
            S, sn = plan.slice(q[c0:c0 + chunk], norms=True)
            spfel.match(S, sn, im.x, im.norm2, bi, bd, m_offset=c0)
        else:
            S, _ = plan.slice(q[c0:c0 + chunk])
            spfel.match_bf16(S, im, bi, bd, m_offset=c0, flags=fl)
    return host(bi), host(bd), host(fl)


@pytest.mark.parametrize("mode", [spfel.MATCH_FP32, spfel.MATCH_BF16_RESCORE8])
@pytest.mark.parametrize("chunk,overlap", [(300, True), (1000, True), (256, False)])
def test_orient_equals_chunked_slice_and_match(mode, chunk, overlap):
    plan, q, images = inputs()
    ref = reference(plan, q, images, mode, chunk)
    bi, bd = spfel.new_best(images.shape[0], DEV)
    fl = torch.zeros(images.shape[0], dtype=torch.int32, device=DEV)
    plan.orient(q, prepared(images, mode), bi, bd, mode=mode, chunk=chunk, overlap=overlap,
                flags=fl)
    np.testing.assert_array_equal(host(bi), ref[0])
    np.testing.assert_array_equal(host(bd), ref[1])
    if mode != spfel.MATCH_FP32:
        np.testing.assert_array_equal(host(fl), ref[2])


def test_orient_fp32_equals_one_shot_match():
    plan, q, images = inputs()
    S, sn = plan.slice(q, norms=True)
    im = spfel.ImagesF32(images)
    b1 = spfel.new_best(images.shape[0], DEV)
    spfel.match(S, sn, im.x, im.norm2, *b1)
    b2 = spfel.new_best(images.shape[0], DEV)
    plan.orient(q, im, *b2, chunk=128)
    np.testing.assert_array_equal(host(b1[0]), host(b2[0]))
    np.testing.assert_array_equal(host(b1[1]), host(b2[1]))


def test_orient_validation():
    plan, q, images = inputs()
    bi, bd = spfel.new_best(images.shape[0], DEV)
    with pytest.raises(TypeError):
        plan.orient(q, spfel.ImagesF32(images), bi, bd, mode=spfel.MATCH_BF16_RESCORE8)
    with pytest.raises(TypeError):
        plan.orient(q, images, bi, bd)
    cplan = spfel.Plan(9, domain=spfel.COMPLEX, device=DEV)
    with pytest.raises(ValueError):
        cplan.orient(q, spfel.ImagesF32(images), bi, bd)
