"""spfel_match_noalloc (workspace in the library's per-device scratch array)
against spfel_match with a caller workspace: bit-identical results on two
calls in a row, the second with smaller sizes, in both matcher modes."""
import numpy as np
import pytest
import torch

import paper_2109_05339_amd as spfel
from paper_2109_05339_amd import _lib
from oracle import match as om
from tests._common import DEV, gpu, host

pytestmark = pytest.mark.gpu


def fp32_case(seed, M, N, P):
    g = np.random.default_rng(seed)
    S = g.gamma(2.0, 15.0, (M, P)).astype(np.float32)
    D = g.poisson(S[g.integers(0, M, N)]).astype(np.float32)
    return gpu(S), gpu(D)


def run_pair(St, Dt, mode):
    """(idx, dist, flags) from spfel_match and from spfel_match_noalloc."""
    N = Dt.shape[0]
    out = []
    for fn in (spfel.match, spfel.match_noalloc):
        bi, bd = spfel.new_best(N, DEV)
        fl = torch.zeros(N, dtype=torch.int32, device=DEV)
        if mode == spfel.MATCH_FP32:
            fn(St, spfel.row_norm2(St), Dt, spfel.row_norm2(Dt), bi, bd)
        else:
            c = gpu(om.centre_rounded_mean(host(Dt)))
            im = spfel.ImagesBF16(Dt, centre=c)
            sb, sn, se = spfel.bf16_centred(St, c)
            fn(sb, sn, im.b16, im.norm2, bi, bd, mode=mode, slices_f32=St, images_f32=Dt,
               slice_err=se, image_err=im.err, flags=fl)
        torch.cuda.synchronize()
        out.append((host(bi), host(bd), host(fl)))
    return out


@pytest.mark.parametrize("mode,first,second", [
    # first FP32 launch has 16 tiles: split K in four (counters and partial
    # tiles in the scratch array), the second is smaller and unsplit
    (spfel.MATCH_FP32, (1000, 256, 16384), (300, 100, 1000)),
    (spfel.MATCH_BF16_RESCORE8, (2000, 500, 2048), (600, 200, 512)),
])
def test_noalloc_equals_workspace_entry_point(mode, first, second):
    assert spfel.match_workspace_bytes(*first, mode) <= 64 << 20
    for seed, (M, N, P) in enumerate((first, second)):
        St, Dt = fp32_case(seed + 10 * mode, M, N, P)
        (ia, da, fa), (ib, db, fb) = run_pair(St, Dt, mode)
        np.testing.assert_array_equal(ia, ib)
        np.testing.assert_array_equal(da, db)
        np.testing.assert_array_equal(fa, fb)
        assert np.all(ia >= 0)


def test_noalloc_rejects_sizes_beyond_the_scratch_array():
    L = spfel.lib()
    p = torch.zeros(64, device=DEV)
    ptr = p.data_ptr()
    # 100,000 x 100,000 FP32 images need 800 KB of keys: fine; BF16 candidates
    # for 100,000 model images x 100,000 images need 2.5 GB: rejected
    code = L.spfel_match_noalloc(ptr, ptr, ptr, ptr, 100000, 100000, 64, 0, 1, ptr, ptr, ptr,
                                 ptr, ptr, ptr, None, None)
    assert code == _lib.ERANGE
    assert "scratch" in L.spfel_last_error().decode()
