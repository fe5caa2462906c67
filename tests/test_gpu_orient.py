"""The two-stream slice->match pipeline (spfel_orient) gives exactly the
result of slicing each chunk and matching it into the running best."""
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


def reference(plan, q, images, mode, chunk):
    dn = spfel.row_norm2(images)
    bi, bd = spfel.new_best(images.shape[0], DEV)
    ix = images if mode == spfel.MATCH_FP32 else (
        images.to(torch.bfloat16) if mode == spfel.MATCH_BF16_RESCORE8 else spfel.split_bf16(images))
    for c0 in range(0, q.shape[0], chunk):
        S, Sb, sn = plan.slice(q[c0:c0 + chunk], bf16=mode == spfel.MATCH_BF16_RESCORE8, norms=True)
        sl = S if mode == spfel.MATCH_FP32 else (Sb if mode == spfel.MATCH_BF16_RESCORE8 else spfel.split_bf16(S))
        spfel.match(sl, sn, ix, dn, bi, bd, m_offset=c0, mode=mode,
                    slices_f32=None if mode == spfel.MATCH_FP32 else S,
                    images_f32=None if mode == spfel.MATCH_FP32 else images)
    return host(bi), host(bd)


@pytest.mark.parametrize("mode", [spfel.MATCH_FP32, spfel.MATCH_BF16_RESCORE8, spfel.MATCH_BF16X3_RESCORE8])
@pytest.mark.parametrize("chunk,overlap", [(300, True), (1000, True), (256, False)])
def test_orient_equals_chunked_slice_and_match(mode, chunk, overlap):
    plan, q, images = inputs()
    ref = reference(plan, q, images, mode, chunk)
    dn = spfel.row_norm2(images)
    ix = images if mode == spfel.MATCH_FP32 else (
        images.to(torch.bfloat16) if mode == spfel.MATCH_BF16_RESCORE8 else spfel.split_bf16(images))
    bi, bd = spfel.new_best(images.shape[0], DEV)
    plan.orient(q, ix, dn, bi, bd, mode=mode, chunk=chunk,
                images_f32=None if mode == spfel.MATCH_FP32 else images, overlap=overlap)
    np.testing.assert_array_equal(host(bi), ref[0])
    np.testing.assert_array_equal(host(bd), ref[1])


def test_orient_fp32_equals_one_shot_match():
    plan, q, images = inputs()
    S, _, sn = plan.slice(q, norms=True)
    dn = spfel.row_norm2(images)
    b1 = spfel.new_best(images.shape[0], DEV)
    spfel.match(S, sn, images, dn, *b1)
    b2 = spfel.new_best(images.shape[0], DEV)
    plan.orient(q, images, dn, *b2, chunk=128)
    np.testing.assert_array_equal(host(b1[0]), host(b2[0]))
    np.testing.assert_array_equal(host(b1[1]), host(b2[1]))


def test_orient_validation():
    plan, q, images = inputs()
    dn = spfel.row_norm2(images)
    bi, bd = spfel.new_best(images.shape[0], DEV)
    with pytest.raises((TypeError, ValueError)):
        plan.orient(q, images.to(torch.bfloat16), dn, bi, bd, mode=spfel.MATCH_BF16_RESCORE8)
    cplan = spfel.Plan(9, domain=spfel.COMPLEX, device=DEV)
    with pytest.raises(ValueError):
        cplan.orient(q, images, dn, bi, bd)
