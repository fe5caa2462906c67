"""CPU-side checks of the C ABI: the library loads, exports every symbol
include/spfel.h declares, and rejects invalid arguments before any GPU work
(these paths never reach a HIP call)."""
import ctypes
import os
import re

import pytest

import paper_2109_05339_amd as spfel
from paper_2109_05339_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "spfel.h")).read()
    return sorted(set(re.findall(r"\b(spfel_\w+)\s*\(", text)))


def test_header_and_binding_agree_and_symbols_exist():
    names = header_functions()
    assert len(names) >= 12
    assert set(names) == set(_lib.SIGNATURES)
    raw = ctypes.CDLL(_lib.LIB_PATH)
    for n in names:
        assert hasattr(raw, n), n


def test_version_and_empty_error():
    L = spfel.lib()
    assert L.spfel_version() == 100


def _create(*args):
    h = ctypes.c_void_p()
    code = spfel.lib().spfel_plan_create(ctypes.byref(h), *args)
    return code, h


@pytest.mark.parametrize("args,code", [
    ((32, 6, 2.0, 2.3, 0, 0), _lib.EINVAL),          # even N
    ((1, 6, 2.0, 2.3, 0, 0), _lib.EINVAL),           # N < 3
    ((5, 7, 2.0, 2.3, 0, 0), _lib.EINVAL),           # w > N
    ((33, 3, 2.0, 2.3, 0, 0), _lib.EUNSUPPORTED),    # w outside 4..8
    ((33, 6, 1.5, 2.3, 0, 0), _lib.EUNSUPPORTED),    # sigma != 2
    ((33, 6, 2.0, -1.0, 0, 0), _lib.EINVAL),         # beta <= 0
    ((33, 6, 2.0, 2.3, 7, 0), _lib.EINVAL),          # domain
    ((513, 6, 2.0, 2.3, 0, 0), _lib.ERANGE),         # too large
])
def test_plan_create_validation(args, code):
    c, h = _create(*args)
    assert c == code
    assert h.value is None
    assert spfel.lib().spfel_last_error().decode() != ""


def test_null_out_pointer():
    assert spfel.lib().spfel_plan_create(None, 33, 6, 2.0, 2.3, 0, 0) == _lib.EINVAL


def test_dead_plan_handles_are_rejected():
    L = spfel.lib()
    bogus = ctypes.c_void_p(0x1234)
    assert L.spfel_plan_destroy(None) == _lib.ESTATE
    assert L.spfel_plan_destroy(bogus) == _lib.ESTATE
    assert L.spfel_set_model(bogus, bogus, None) == _lib.ESTATE
    assert L.spfel_slice(bogus, None, 1, None, 1, None, None, None, None) == _lib.ESTATE
    assert L.spfel_merge_adjoint(bogus, None, 1, None, 1, None, None, None, 0, None) == _lib.ESTATE
    assert L.spfel_weighted_residual(bogus, None, None, None, 1, 1.0, None, None, None, None) == _lib.ESTATE
    assert L.spfel_plan_info(bogus, None, None) == _lib.ESTATE
    with pytest.raises(spfel.SpfelStateError):
        _lib.check(L.spfel_plan_destroy(bogus))


def test_match_validation_before_launch():
    L = spfel.lib()
    p = ctypes.c_void_p(4096)
    args = dict(slices=p, sn=p, images=p, dn=p, M=10, N=10, P=64, off=0, mode=0, s32=None,
                d32=None, se=None, de=None, idx=p, dist=p, flags=None, ws=p, wsb=1 << 20, st=None)

    def call(**kw):
        a = dict(args)
        a.update(kw)
        return L.spfel_match(a["slices"], a["sn"], a["images"], a["dn"], a["M"], a["N"], a["P"],
                             a["off"], a["mode"], a["s32"], a["d32"], a["se"], a["de"], a["idx"],
                             a["dist"], a["flags"], a["ws"], a["wsb"], a["st"])
    assert call(M=-1) == _lib.EINVAL
    assert call(mode=5) == _lib.EINVAL
    assert call(mode=2) == _lib.EINVAL                        # no split-BF16 mode
    assert call(off=2 ** 31 - 5) == _lib.ERANGE
    assert call(slices=None) == _lib.EINVAL
    assert call(mode=1) == _lib.EINVAL                        # no float32 data to rescore
    assert call(mode=1, s32=p, d32=p) == _lib.EINVAL          # no rounding-error norms
    assert call(wsb=8) == _lib.EINVAL                         # workspace too small
    assert call(ws=ctypes.c_void_p(4096 + 16)) == _lib.EINVAL  # workspace not 256-byte aligned
    assert call(slices=ctypes.c_void_p(4098)) == _lib.EINVAL  # misaligned
    assert call(M=0) == _lib.OK and call(N=0) == _lib.OK      # empty: nothing to do


def test_operand_call_validation():
    L = spfel.lib()
    p = ctypes.c_void_p(4096)
    assert L.spfel_column_mean(p, 0, 8, 1, p, None) == _lib.EINVAL      # no rows
    assert L.spfel_column_mean(None, 3, 8, 1, p, None) == _lib.EINVAL
    assert L.spfel_column_mean(p, 3, 0, 1, p, None) == _lib.OK
    assert L.spfel_column_mean(ctypes.c_void_p(4098), 3, 8, 1, p, None) == _lib.EINVAL
    assert L.spfel_bf16_centred(p, -1, 8, None, p, p, p, None) == _lib.EINVAL
    assert L.spfel_bf16_centred(p, 0, 8, None, p, p, p, None) == _lib.OK
    assert L.spfel_bf16_centred(p, 3, 8, None, None, p, p, None) == _lib.EINVAL   # out NULL
    assert L.spfel_bf16_centred(p, 3, 8, ctypes.c_void_p(4097), p, p, p, None) == _lib.EINVAL


def test_workspace_sizes():
    ws = spfel.match_workspace_bytes
    assert ws(100, 256, 4096, spfel.MATCH_FP32) == 256 * 8
    assert ws(50000, 2048, 4096, spfel.MATCH_FP32) == 2048 * 8          # many rounds: no split-K
    assert ws(10000, 2048, 16384, spfel.MATCH_FP32) == 2048 * 8          # 2.5 rounds: no split-K
    # 8 x 16 tiles are a quarter of a round of resident blocks: split K in four
    assert ws(1000, 2048, 16384, spfel.MATCH_FP32) == 2048 * 8 + 512 + 128 * 4 * 128 * 128 * 4
    # 8 m-tiles of 128 x 8 candidates, then chunk maxima + count (256 B), the
    # fallback list (256-byte rounded) and its keys
    assert ws(1000, 256, 4096, spfel.MATCH_BF16_RESCORE8) == 8 * 256 * 8 * 4 + 256 + 1024 + 256 * 8
    assert ws(0, 0, 0, spfel.MATCH_FP32) == 256


def test_row_norm2_validation():
    L = spfel.lib()
    assert L.spfel_row_norm2(None, 7, 1, 1, None, None) == _lib.EINVAL
    assert L.spfel_row_norm2(None, 0, -1, 1, None, None) == _lib.EINVAL
    assert L.spfel_row_norm2(None, 0, 0, 5, None, None) == _lib.OK
    assert L.spfel_row_norm2(None, 0, 3, 5, None, None) == _lib.EINVAL


def test_exceptions_map_codes():
    with pytest.raises(spfel.SpfelInvalidArgument):
        _lib.check(spfel.lib().spfel_row_norm2(None, 7, 1, 1, None, None))


def test_noalloc_rejects_sizes_beyond_its_scratch_before_any_launch():
    L = spfel.lib()
    p = ctypes.c_void_p(4096)
    # BF16 candidates of 100,000 model images x 100,000 images: 2.5 GB > 64 MiB
    code = L.spfel_match_noalloc(p, p, p, p, 100000, 100000, 64, 0, 1, p, p, p, p, p, p, None,
                                 None)
    assert code == _lib.ERANGE
    assert "scratch" in L.spfel_last_error().decode()
    assert L.spfel_match_noalloc(p, p, p, p, -1, 10, 64, 0, 0, None, None, None, None, p, p,
                                 None, None) == _lib.EINVAL


@pytest.mark.parametrize("args", [
    (8, 0, 4, 0),       # even N
    (1, 0, 4, 0),       # N < 3
    (7, 5, 4, 0),       # domain
    (7, 0, 0, 0),       # no systems
    (7, 1, 17, 0),      # more than 16 systems
])
def test_normal_create_validation(args):
    h = ctypes.c_void_p()
    assert spfel.lib().spfel_normal_create(ctypes.byref(h), *args) == _lib.EINVAL
    assert h.value is None
    assert spfel.lib().spfel_normal_create(None, 7, 0, 4, 0) == _lib.EINVAL
    assert spfel.lib().spfel_normal_create(ctypes.byref(h), 513, 0, 4, 0) == _lib.ERANGE


def test_normal_calls_reject_dead_handles():
    L = spfel.lib()
    bogus = ctypes.c_void_p(0x1000)
    lam = (ctypes.c_float * 1)(1.0)
    assert L.spfel_normal_destroy(bogus) == _lib.ESTATE
    assert L.spfel_normal_set_psf(bogus, 0x2000, None) == _lib.ESTATE
    assert L.spfel_normal_apply(bogus, 0x2000, 1, lam, 0x3000, None) == _lib.ESTATE
    assert L.spfel_normal_solve(bogus, 0x2000, 0x2000, 1, lam, 5, 0x3000, None, None) == _lib.ESTATE
    assert L.spfel_normal_lcurve(bogus, 0x2000, 0x2000, 0x2000, 1, lam, 0.0, 0x3000, None,
                                 None) == _lib.ESTATE


def test_phase_create_validation_and_dead_handles():
    L = spfel.lib()
    h = ctypes.c_void_p()
    assert L.spfel_phase_create(ctypes.byref(h), 1, 0) == _lib.EINVAL
    assert L.spfel_phase_create(ctypes.byref(h), 1025, 0) == _lib.ERANGE
    assert L.spfel_phase_create(None, 16, 0) == _lib.EINVAL
    assert h.value is None
    bogus = ctypes.c_void_p(0x1000)
    assert L.spfel_phase_destroy(bogus) == _lib.ESTATE
    assert L.spfel_phase_iterate(bogus, 0x2000, 0x2000, None, 0x2000, 1, 0, 0.9, 1, None,
                                 None) == _lib.ESTATE
    assert L.spfel_phase_shrinkwrap(bogus, 0x2000, 1.0, 0.1, 0x2000, None, None) == _lib.ESTATE
