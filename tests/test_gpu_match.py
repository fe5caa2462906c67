"""GPU orientation matching (section II-B) against the oracle's FP64
distances on the same float32 inputs.  The argmin must agree exactly on
every image whose exact top-2 gap exceeds the two distances' float32 error
bounds; the returned distance must lie within its bound of the exact one."""
import functools

import numpy as np
import pytest
import torch

import synth
import paper_2109_05339_amd as spfel
from oracle import match as om
from tests._common import DEV, gpu, host, detector, molecule_slices

pytestmark = pytest.mark.gpu


def chain_fp32(P):      # the FP32 matcher's documented accumulation chain
    return 36 + -(-P // 32)


def chain_rescore(P):
    return 10 + -(-P // 64)


@functools.lru_cache(maxsize=None)
def c1_data(n_refs=1000, n_img=300):
    """C1-shaped matcher inputs: the molecule's intensity at the reference
    orientations and Poisson images of it at random orientations, made
    without the library (both sides read the same float32 values)."""
    cfg = synth.config(1)
    det = detector(cfg.n_det)
    lam0 = host(molecule_slices(1, synth.quaternions(cfg, "image_quats", n_img), det))
    alpha = synth.photon_scale(lam0, cfg.photons)
    S = alpha * host(molecule_slices(1, synth.quaternions(cfg, "ref_quats", n_refs), det))
    D = synth.poisson_counts(cfg, alpha * lam0)
    return S.astype(np.float32), D.astype(np.float32)


def run_fp32(S, D, chunks=None):
    St, Dt = gpu(S), gpu(D)
    sn, dn = spfel.row_norm2(St), spfel.row_norm2(Dt)
    bi, bd = spfel.new_best(D.shape[0], DEV)
    if chunks is None:
        chunks = [(0, S.shape[0])]
    for a, b in chunks:
        spfel.match(St[a:b], sn[a:b], Dt, dn, bi, bd, m_offset=a)
    return host(bi), host(bd), host(sn), host(dn)


def exact_and_bounds(S, D, L):
    S64, D64 = S.astype(np.float64), D.astype(np.float64)
    ex = om.distances_expanded(S64, D64)
    absdot = np.abs(S64) @ np.abs(D64).T
    E = om.fp32_distance_bound((S64 ** 2).sum(1)[:, None], (D64 ** 2).sum(1)[None, :], absdot, L)
    return ex, E


def check_decided(idx, dist, S, D, L, min_decided=0.0):
    ex, E = exact_and_bounds(S, D, L)
    am = om.argmin_first(ex)
    cols = np.arange(D.shape[0])
    order = np.argsort(ex, axis=0, kind="stable")
    m1, m2 = order[0], order[1]
    gap = ex[m2, cols] - ex[m1, cols]
    decided = gap > E[m1, cols] + E[m2, cols]
    assert np.all(idx[decided] == am[decided])
    # any returned index must be a near-minimiser within the bounds
    assert np.all(ex[idx, cols] - ex[m1, cols] <= E[idx, cols] + E[m1, cols])
    assert np.all(np.abs(dist - ex[idx, cols]) <= E[idx, cols])
    assert decided.mean() >= min_decided
    return decided


def test_fp32_matcher_c1_shape_ragged_tiles():
    S, D = c1_data()
    idx, dist, _, _ = run_fp32(S, D)
    decided = check_decided(idx, dist, S, D, chain_fp32(S.shape[1]), min_decided=0.75)
    print(f"decided {decided.mean():.3f} of {len(decided)} images")


def test_fp32_matcher_scalar_path_and_small_sizes():
    g = np.random.default_rng(7)
    S = (g.random((45, 1001)) * 40).astype(np.float32)
    D = g.poisson(S[[3, 44, 17, 17, 0]] + 1).astype(np.float32)
    idx, dist, _, _ = run_fp32(S, D)
    check_decided(idx, dist, S, D, chain_fp32(1001), min_decided=1.0)
    np.testing.assert_array_equal(idx, om.argmin_first(om.distances_direct(S, D)))


def test_ties_lowest_index_and_self_match():
    S, _ = c1_data()
    S = S[:300].copy()
    S[250] = S[7]            # duplicate model image: 7 must win
    D = S[[7, 250, 11, 299]].copy()
    idx, dist, sn, _ = run_fp32(S, D)
    np.testing.assert_array_equal(idx, [7, 7, 11, 299])
    assert np.all(np.abs(dist) <= om.gamma(chain_fp32(S.shape[1])) * 4 * sn[[7, 7, 11, 299]])


def test_chunked_streaming_equals_one_shot_bitwise():
    S, D = c1_data()
    a = run_fp32(S, D)
    b = run_fp32(S, D, chunks=[(0, 300), (300, 301), (301, 1000)])
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_running_best_is_respected():
    S, D = c1_data()
    St, Dt = gpu(S), gpu(D)
    sn, dn = spfel.row_norm2(St), spfel.row_norm2(Dt)
    bi = torch.full((D.shape[0],), 5000, dtype=torch.int32, device=DEV)
    bd = torch.full((D.shape[0],), -1.0, dtype=torch.float32, device=DEV)
    bd[:10] = float("inf")
    spfel.match(St, sn, Dt, dn, bi, bd)
    bi, bd = host(bi), host(bd)
    assert np.all(bi[10:] == 5000) and np.all(bd[10:] == -1.0)
    assert np.all(bi[:10] < 1000)


def run_bf16(S, D, chunks=None):
    St, Dt = gpu(S), gpu(D)
    Sb, Db = St.to(torch.bfloat16), Dt.to(torch.bfloat16)
    sn, dn = spfel.row_norm2(St), spfel.row_norm2(Dt)
    bi, bd = spfel.new_best(D.shape[0], DEV)
    if chunks is None:
        chunks = [(0, S.shape[0])]
    for a, b in chunks:
        spfel.match(Sb[a:b], sn[a:b], Db, dn, bi, bd, m_offset=a, mode=spfel.MATCH_BF16_RESCORE8,
                    slices_f32=St[a:b], images_f32=Dt)
    return host(bi), host(bd)


def test_bf16_rescore_matches_fp32_argmin_on_decided_images():
    S, D = c1_data()
    i32, d32, _, _ = run_fp32(S, D)
    ib, db = run_bf16(S, D)
    ex, E = exact_and_bounds(S, D, chain_fp32(S.shape[1]))
    cols = np.arange(D.shape[0])
    order = np.argsort(ex, axis=0, kind="stable")
    m1, m2 = order[0], order[1]
    gap = ex[m2, cols] - ex[m1, cols]
    decided = gap > E[m1, cols] + E[m2, cols]
    # certificate of the top-8 from the BF16 proxy bound (images are exact
    # small integers, so only the slices' rounding counts)
    S64, D64 = S.astype(np.float64), D.astype(np.float64)
    absdot = np.abs(S64) @ np.abs(D64).T
    b = (S64 ** 2).sum(1)[:, None] + (D64 ** 2).sum(1)[None, :] - 2 * (om.bf16_round(S).astype(np.float64) @ D64.T)
    ebf = om.bf16_proxy_bound(absdot, om.fp32_distance_bound((S64 ** 2).sum(1)[:, None], (D64 ** 2).sum(1)[None, :], absdot, S.shape[1] + 2), exact_images=True)
    cert = om.topk_certified(b, ebf, 8)
    # images whose exact argmin is in the true proxy top-8 and decided must agree
    top8 = om.topk(b, 8)
    in8 = np.array([m1[n] in top8[:, n] for n in cols])
    ok = decided & in8
    assert np.all(ib[ok] == i32[ok])
    assert np.all(ib[cert & decided] == i32[cert & decided])
    assert ok.mean() >= 0.8
    # the rescored distance is an exact float32 evaluation
    Lr = chain_rescore(S.shape[1])
    Eres = om.fp32_distance_bound((S64 ** 2).sum(1)[ib], (D64 ** 2).sum(1), absdot[ib, cols], Lr)
    assert np.all(np.abs(db - ex[ib, cols]) <= Eres + E[ib, cols])
    print(f"bf16: decided {decided.mean():.3f}, certified {cert.mean():.3f}, in-top8 {in8.mean():.4f}, "
          f"agree {np.mean(ib == i32):.4f}")


def test_bf16_chunked_streaming():
    """Streaming chunks rescore each chunk's own top-8 (a superset of the
    one-shot candidates), so both agree with the exact argmin wherever the
    exact minimiser is decided and inside the one-shot proxy top-8."""
    S, D = c1_data()
    a = run_bf16(S, D)
    b = run_bf16(S, D, chunks=[(0, 500), (500, 1000)])
    ex, E = exact_and_bounds(S, D, chain_fp32(S.shape[1]))
    cols = np.arange(D.shape[0])
    order = np.argsort(ex, axis=0, kind="stable")
    m1, m2 = order[0], order[1]
    decided = (ex[m2, cols] - ex[m1, cols]) > E[m1, cols] + E[m2, cols]
    S64, D64 = S.astype(np.float64), D.astype(np.float64)
    b16 = (S64 ** 2).sum(1)[:, None] + (D64 ** 2).sum(1)[None, :] - 2 * (om.bf16_round(S).astype(np.float64) @ D64.T)
    top8 = om.topk(b16, 8)
    ok = decided & np.array([m1[n] in top8[:, n] for n in cols])
    assert np.all(a[0][ok] == m1[ok]) and np.all(b[0][ok] == m1[ok])
    # chunked never does worse than one-shot in exact distance
    assert np.all(ex[b[0], cols] <= ex[a[0], cols] + E[b[0], cols] + E[a[0], cols])


@pytest.mark.parametrize("M,N,P,misalign", [
    (8192, 8192, 192, False),   # 256 x 256 tiles, all full
    (8300, 8150, 192, False),   # 256 x 256 tiles with ragged edge tiles
    (8192, 8192, 136, False),   # P not a multiple of 64: 128 x 128 tiles
    (8192, 8192, 192, True),    # operands not 16-byte aligned: 128 x 128 tiles
])
def test_bf16_large_shapes_against_oracle_on_sampled_images(M, N, P, misalign):
    """Shapes that fill >= 4 rounds of 256 x 256 tiles: the large-tile BF16
    kernel when P is a whole number of its K steps and the operands are
    16-byte aligned, else the 128-row kernel.  The oracle checks 192 sampled
    images exactly."""
    g = np.random.default_rng(11)
    base = g.gamma(2.0, 10.0, (M, P)).astype(np.float32)
    pick = g.integers(0, M, N)
    D = g.poisson(base[pick]).astype(np.float32)
    assert spfel.match_workspace_bytes(M, N, P, spfel.MATCH_BF16_RESCORE8) == -(-M // 128) * N * 32
    St, Dt = gpu(base), gpu(D)
    if misalign:   # views one element into a larger buffer
        Sb = torch.empty(M * P + 8, dtype=torch.bfloat16, device=DEV)[1:1 + M * P].view(M, P)
        Sb.copy_(St)
    else:
        Sb = St.to(torch.bfloat16)
    Db = Dt.to(torch.bfloat16)
    bi, bd = spfel.new_best(N, DEV)
    spfel.match(Sb, spfel.row_norm2(St), Db, spfel.row_norm2(Dt), bi, bd,
                mode=spfel.MATCH_BF16_RESCORE8, slices_f32=St, images_f32=Dt)
    ib, db = host(bi), host(bd)
    cols = np.sort(g.choice(N, 192, replace=False))
    S64, Ds = base.astype(np.float64), D[cols].astype(np.float64)
    ex = om.distances_expanded(S64, Ds)
    absdot = np.abs(S64) @ np.abs(Ds).T
    E = om.fp32_distance_bound((S64 ** 2).sum(1)[:, None], (Ds ** 2).sum(1)[None, :], absdot, chain_fp32(P))
    order = np.argsort(ex, axis=0, kind="stable")
    c = np.arange(len(cols))
    m1, m2 = order[0], order[1]
    decided = ex[m2, c] - ex[m1, c] > E[m1, c] + E[m2, c]
    b16 = (S64 ** 2).sum(1)[:, None] + (Ds ** 2).sum(1)[None, :] - 2 * (om.bf16_round(base).astype(np.float64) @ Ds.T)
    top8 = om.topk(b16, 8)
    ok = decided & np.array([m1[n] in top8[:, n] for n in c])
    assert ok.mean() >= 0.9
    np.testing.assert_array_equal(ib[cols][ok], m1[ok])
    assert np.all(np.abs(db[cols] - ex[ib[cols], c]) <= 2 * E[ib[cols], c])


@pytest.mark.parametrize("mode,M,N,P", [
    (spfel.MATCH_FP32, 10000, 2048, 16384),            # the default workload's launch
    (spfel.MATCH_BF16_RESCORE8, 8192, 16384, 65536),   # one chunk of workload 5
])
def test_full_size_launches_against_oracle_on_sampled_images(mode, M, N, P):
    """The launches bench.py times, at their full sizes: slice rows uniform
    in [0, 40) and Poisson images of randomly picked rows (seeded, made on
    the device with torch).  The oracle's float64 distances of 24 sampled
    images to every row decide the argmin and bound the returned distance."""
    g = torch.Generator(device=DEV).manual_seed(17)
    St = torch.rand((M, P), generator=g, device=DEV) * 40.0
    pick = torch.randint(0, M, (N,), generator=g, device=DEV)
    Dt = torch.poisson(St[pick], generator=g)
    sn, dn = spfel.row_norm2(St), spfel.row_norm2(Dt)
    bi, bd = spfel.new_best(N, DEV)
    if mode == spfel.MATCH_FP32:
        spfel.match(St, sn, Dt, dn, bi, bd)
        L = chain_fp32(P)
    else:
        spfel.match(St.to(torch.bfloat16), sn, Dt.to(torch.bfloat16), dn, bi, bd, mode=mode,
                    slices_f32=St, images_f32=Dt)
        L = chain_rescore(P)
    ib, db = host(bi), host(bd)
    cols = np.sort(np.random.default_rng(3).choice(N, 24, replace=False))
    Ds = host(Dt[torch.as_tensor(cols, device=DEV)]).astype(np.float64)
    ex = np.empty((M, len(cols)))
    E = np.empty((M, len(cols)))
    dn2 = (Ds ** 2).sum(1)[None, :]
    for r0 in range(0, M, 1024):       # float64 rows, a block at a time
        S64 = host(St[r0:r0 + 1024]).astype(np.float64)
        sn2 = (S64 ** 2).sum(1)[:, None]
        ex[r0:r0 + 1024] = om.distances_expanded(S64, Ds)
        E[r0:r0 + 1024] = om.fp32_distance_bound(sn2, dn2, S64 @ Ds.T, max(L, chain_fp32(P)))
    c = np.arange(len(cols))
    order = np.argsort(ex, axis=0, kind="stable")
    m1, m2 = order[0], order[1]
    decided = ex[m2, c] - ex[m1, c] > E[m1, c] + E[m2, c]
    assert decided.all()
    np.testing.assert_array_equal(ib[cols], m1)
    np.testing.assert_array_equal(m1, host(pick)[cols])
    assert np.all(np.abs(db[cols] - ex[m1, c]) <= 2 * E[m1, c])
