"""Slice-and-match throughput on one MI355X.

Default workload (the largest one-GPU configuration): 129^3 float32
intensity model of a 500-scatterer molecule, 256 x 256 detector (65,536
Ewald-sphere pixels), 100,000 reference orientations streamed in chunks of
8,192, 16,384 Poisson images at 5 photons/pixel.  One step is one pass of
the whole hot path over that batch:

  set_model (deconvolve + separable transform to the 258^3 fine grid)
  -> for each chunk of 8,192 orientations: type-2 slicing (float32), the
     centred BF16 operands, the BF16 distance GEMM with per-tile top-8,
     certified FP32 rescore into the running best
  -> type-1 merge (adjoint spread + transform) of every image at its
     matched orientation.

The JSON line reports pixel-comparisons/s = M * n_img * P / step time
(inputs resident in HBM), the per-kernel times measured with HIP events on
the launch stream inside the timed steps, the dominant kernel against its
roofline, BF16-vs-FP32 argmin agreement on an image subset, and the CPU
oracle timed on a bounded sample on this host.  ``--config 2`` times the
FP32 form (65^3, 128^2, 10^4 x 2,048); ``--config 4`` the loss + gradient.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
# 256 CUs x 64 lanes x 2 flop x 2.4 GHz: FP32 fused multiply-add without the
# packed (two-per-lane) form, which this build does not emit
PEAK_FP32_VECTOR_TFLOPS = 78.6
# algorithmic work of one interpolated (or spread) point at w = 6: w^3
# multiply-adds
INTERP_FLOP_PER_POINT = 2 * 6 ** 3


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=5, help="workload id (5: the default above)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the agreement check and the workload-2 figures")
    ap.add_argument("--cpu-sample", type=int, default=128,
                    help="orientations the oracle slices in the CPU baseline")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="oracle process pool size (0: the CPUs this process may use, at most 16)")
    ap.add_argument("--counters", action="store_true",
                    help="counter-collection run: one chunk of each hot kernel and a plain 1 GiB "
                         "device copy (the copy calibrates FETCH_SIZE/WRITE_SIZE), no timing")
    ap.add_argument("--write-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc runs of --counters (FETCH_SIZE, then "
                         "WRITE_SIZE) into profiles/traffic.json and exit (no GPU)")
    return ap.parse_args()


# HBM traffic of the roofline kernels, from rocprofv3 FETCH_SIZE / WRITE_SIZE
# counters (KiB per dispatch) scaled by what the same counters read for a
# plain 1 GiB device copy; valid only while the kernel's sources hash to the
# value recorded with the counters.
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")
CSRC = os.path.join(ROOT, "paper_2109_05339_amd", "csrc")
KERNEL_SOURCES = {
    "interp_tiled_kernel": ["interp.hip", "device_common.h", "internal.h"],
    "match_f32_kernel": ["match.hip", "device_common.h", "internal.h"],
    "match_bf16_big_kernel": ["match.hip", "device_common.h", "internal.h"],
    "spread_binned_kernel": ["spread_binned.hip", "device_common.h", "internal.h"],
}
COPY_BYTES = 1 << 30


def kernel_source_hash(kernel: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _pmc_dispatches(d: str, counter: str):
    """(kernel name, grid size, KiB, dispatch id) of every dispatch in a
    --pmc run."""
    import csv
    import glob
    per = {}
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                key = (int(r["Dispatch_Id"]), r["Kernel_Name"], int(r["Grid_Size"]))
                per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    return [(k[1], k[2], v, k[0]) for k, v in per.items()]


def write_traffic(fetch_dir: str, write_dir: str, config: int) -> int:
    out = {"method": "rocprofv3 --pmc FETCH_SIZE, then --pmc WRITE_SIZE, over `bench.py "
                     "--counters --config N`; KiB per dispatch scaled by the counter's "
                     "reading for a 1 GiB device copy; per launch at workload N",
           "config": config, "kernels": {}}
    fetch, write = _pmc_dispatches(fetch_dir, "FETCH_SIZE"), _pmc_dispatches(write_dir, "WRITE_SIZE")

    def largest(rows, pred):
        rows = [r for r in rows if pred(r[0])]
        return max(rows, key=lambda r: r[1]) if rows else None

    # the calibration copy is the run's last dispatch
    cf, cw = max(fetch, key=lambda r: r[3]), max(write, key=lambda r: r[3])
    if "copy" not in cf[0] or "copy" not in cw[0]:
        cf = cw = None
    if cf is None or cw is None:
        print("no copy dispatch found for calibration", file=sys.stderr)
        return 1
    f_fac, w_fac = COPY_BYTES / (cf[2] * 1024.0), COPY_BYTES / (cw[2] * 1024.0)
    out["calibration"] = {"copy_bytes": COPY_BYTES, "fetch_kib": cf[2], "write_kib": cw[2],
                          "fetch_factor": f_fac, "write_factor": w_fac}
    for k in KERNEL_SOURCES:
        a, b = largest(fetch, lambda n: k in n), largest(write, lambda n: k in n)
        if a is None or b is None:
            continue
        fb, wb = a[2] * 1024.0 * f_fac, b[2] * 1024.0 * w_fac
        out["kernels"][k] = {"source_sha256": kernel_source_hash(k), "grid_size": a[1],
                             "fetch_kib": a[2], "write_kib": b[2], "fetch_bytes": fb,
                             "write_bytes": wb, "bytes_per_launch": fb + wb}
    with open(TRAFFIC_JSON, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))
    return 0


def traffic_of(kernel: str, config: int):
    """HBM bytes per launch of `kernel`, or None if not measured for the
    current sources on this workload."""
    try:
        with open(TRAFFIC_JSON) as fh:
            data = json.load(fh)
        rec = data["kernels"][kernel]
        if data["config"] != config:
            return None
    except (OSError, KeyError, ValueError):
        return None
    return rec["bytes_per_launch"] if rec["source_sha256"] == kernel_source_hash(kernel) else None


def main() -> int:
    args = parse()
    if args.write_traffic:
        return write_traffic(*args.write_traffic, args.config)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); every box here has one "
              "GPU and the multi-GPU form of this path is a design, not a build", file=sys.stderr)
        return 2
    import synth
    cfg = synth.config(args.config)
    cpu = None
    if not args.no_cpu_baseline and not args.counters and args.config in (2, 5):
        # before the GPU is touched: the oracle's process pool forks from here
        cpu = cpu_baseline(cfg, args)
    import torch
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.config == 4:
        return bench_gradient(args, cfg, dev)
    if args.config == 5:
        out = bench_streaming(args, cfg, dev)
        if out is None:
            return 0
        if not args.no_extras:
            log("workload 2 figures (FP32 form)")
            out["workload2"] = bench_plain(args, synth.config(2), dev, steps=10, warmup=2)
    else:
        out = bench_plain(args, cfg, dev, args.steps, args.warmup)
        if out is None:
            return 0
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)
    return 0


class Timer:
    """HIP events recorded on the launch stream; durations per label."""

    def __init__(self, torch, stream, on=True):
        self.torch, self.stream, self.on = torch, stream, on
        self.marks = {}

    def span(self, label):
        timer = self

        class _Span:
            def __enter__(self):
                if timer.on:
                    self.a = timer.torch.cuda.Event(enable_timing=True)
                    self.a.record(timer.stream)

            def __exit__(self, *exc):
                if timer.on:
                    b = timer.torch.cuda.Event(enable_timing=True)
                    b.record(timer.stream)
                    timer.marks.setdefault(label, []).append((self.a, b))
        return _Span()

    def ms(self, label):
        return [a.elapsed_time(b) for a, b in self.marks.get(label, [])]


def roofline(kernel, bound, work, ms, peak, unit, traffic):
    achieved = work / (ms * 1e-3) / (1e12 if unit == "TFLOP/s" else 1e9)
    return {"kernel": kernel, "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": traffic, "launch_ms": ms}


def _render_images(plan, cfg, dev, quats, m_host, chunk=2048):
    """Noiseless slices at the image orientations (unscaled model), photon
    scale, then seeded Poisson counts drawn on the device (float32)."""
    import torch
    import synth
    plan.set_model(torch.from_numpy(m_host.astype(np.float32)).to(dev))
    n = quats.shape[0]
    lam = torch.empty((n, cfg.n_pix), dtype=torch.float32, device=dev)
    for c0 in range(0, n, chunk):
        lam[c0:c0 + chunk] = plan.slice(quats[c0:c0 + chunk])[0].clamp_(min=0)
    alpha = cfg.photons / float(lam.double().mean())
    lam.mul_(alpha)
    g = torch.Generator(device=dev)
    g.manual_seed(int(synth.rng(cfg.seed_id, "poisson").integers(0, 2 ** 62)))
    images = torch.poisson(lam, generator=g)
    del lam
    return images, alpha


def bench_streaming(args, cfg, dev):
    """Workload 5, the default: 100,000 reference orientations streamed in
    chunks of 8,192 (sliced and never stored in full), centred BF16 matcher
    with certified per-chunk FP32 rescoring into a running best, then the
    type-1 merge of all images at their matched orientations."""
    import torch
    import synth
    import paper_2109_05339_amd as spfel
    M, n_img, P, N, C = cfg.n_refs, cfg.n_images, cfg.n_pix, cfg.n_model, cfg.chunk
    t0 = time.time()
    m_host, _ = synth.intensity_model(cfg)
    det = torch.from_numpy(synth.detector_q(cfg.n_det).astype(np.float32)).to(dev)
    ref_q = torch.from_numpy(synth.quaternions(cfg, "ref_quats", M).astype(np.float32)).to(dev)
    img_q = torch.from_numpy(synth.quaternions(cfg, "image_quats", n_img).astype(np.float32)).to(dev)
    plan = spfel.Plan(N, device=dev)
    plan.set_detector(det)
    images, alpha = _render_images(plan, cfg, dev, img_q, m_host)
    model = torch.from_numpy((alpha * m_host).astype(np.float32)).to(dev)
    im = spfel.ImagesBF16(images)     # centre = rounded per-pixel image mean
    merged = torch.empty((N, N, N), dtype=torch.float32, device=dev)
    flags = torch.zeros((n_img,), dtype=torch.int32, device=dev)
    ws = torch.empty((spfel.match_workspace_bytes(C, n_img, P, spfel.MATCH_BF16_RESCORE8),),
                     dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    log(f"workload 5 inputs ready in {time.time() - t0:.1f}s")
    stream = torch.cuda.current_stream(dev)
    chunks = [(c0, min(M, c0 + C)) for c0 in range(0, M, C)]

    def step(tm):
        with tm.span("set_model"):
            plan.set_model(model)
        bi, bd = spfel.new_best(n_img, dev)
        flags.zero_()
        for c0, c1 in chunks:
            full = c1 - c0 == C
            with tm.span("slice" if full else "slice_tail"):
                S, _ = plan.slice(ref_q[c0:c1])
            with tm.span("centre" if full else "centre_tail"):
                sb, sn, se = spfel.bf16_centred(S, im.centre)
            with tm.span("match" if full else "match_tail"):
                spfel.match(sb, sn, im.b16, im.norm2, bi, bd, m_offset=c0,
                            mode=spfel.MATCH_BF16_RESCORE8, slices_f32=S, images_f32=images,
                            slice_err=se, image_err=im.err, flags=flags, workspace=ws)
            del S, sb
        with tm.span("merge"):
            plan.merge_adjoint(ref_q[bi.long()].contiguous(), None, images, out=merged)
        return bi, bd

    if args.counters:
        with torch.no_grad():
            S, _ = plan.slice(ref_q[:C])
            sb, sn, se = spfel.bf16_centred(S, im.centre)
            bi, bd = spfel.new_best(n_img, dev)
            spfel.match(sb, sn, im.b16, im.norm2, bi, bd, mode=spfel.MATCH_BF16_RESCORE8,
                        slices_f32=S, images_f32=images, slice_err=se, image_err=im.err,
                        workspace=ws)
            plan.merge_adjoint(ref_q[:n_img].contiguous(), None, images, out=merged)
            _copy_calibration(torch, dev)
        return None

    for _ in range(args.warmup):
        step(Timer(torch, stream, on=False))
    torch.cuda.synchronize()
    tm = Timer(torch, stream)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        bi, bd = step(tm)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps * 1e3
    comps = float(M) * n_img * P
    per = {k: float(np.mean(tm.ms(k))) for k in tm.marks}
    tot = {k: float(np.sum(tm.ms(k))) / args.steps for k in tm.marks}
    full = len([c for c in chunks if c[1] - c[0] == C])
    r_slice = roofline("interp_tiled_kernel", "alu", INTERP_FLOP_PER_POINT * C * P, per["slice"],
                       PEAK_FP32_VECTOR_TFLOPS, "TFLOP/s", traffic_of("interp_tiled_kernel", 5))
    r_match = roofline("match_bf16_big_kernel + rescore", "mfma", 2.0 * C * n_img * P,
                       per["match"], PEAK_BF16_MFMA_TFLOPS, "TFLOP/s",
                       traffic_of("match_bf16_big_kernel", 5))
    r_merge = roofline("binned spread + transform", "alu", INTERP_FLOP_PER_POINT * n_img * P,
                       per["merge"], PEAK_FP32_VECTOR_TFLOPS, "TFLOP/s",
                       traffic_of("spread_binned_kernel", 5))
    share = {"slice": tot["slice"], "match": tot["match"], "merge": tot["merge"]}
    dominant = {"slice": r_slice, "match": r_match, "merge": r_merge}[max(share, key=share.get)]
    fl = flags.cpu().numpy()
    out = {
        "metric": "slice+match pixel-comparisons/s",
        "value": comps / (wall * 1e-3),
        "unit": "pixel-comparisons/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16+f32", "data": "synthetic",
        "config": {"workload": (f"{N}^3 float32 model ({cfg.n_atoms} scatterers), {cfg.n_det}x"
                                f"{cfg.n_det} detector, {M} reference orientations streamed in "
                                f"chunks of {C}, {n_img} Poisson images at {cfg.photons:g} "
                                "photons/px; step = set_model + per chunk (type-2 slicing, "
                                "centred BF16 operands, BF16 distance GEMM with top-8, certified "
                                "FP32 rescore) + type-1 merge of all images at their matched "
                                "orientations"),
                   "M": M, "n_img": n_img, "P": P, "N": N, "chunk": C},
        "breakdown_ms_per_step": {k: tot[k] for k in sorted(tot)},
        "per_full_chunk_ms": {"slice": per["slice"], "centre": per["centre"], "match": per["match"],
                              "full_chunks": full},
        "nufft_type2_pts_per_s": C * P / (per["slice"] * 1e-3),
        "nufft_type1_pts_per_s": n_img * P / (per["merge"] * 1e-3),
        "certified_fraction": float(np.mean(fl == 0)),
        "roofline": dominant,
        "roofline_kernels": [r_slice, r_match, r_merge],
    }
    log(f"step {wall:.1f} ms; per full chunk slice {per['slice']:.2f} ms, centre "
        f"{per['centre']:.2f} ms, match {per['match']:.2f} ms; merge {per['merge']:.1f} ms; "
        f"certified {out['certified_fraction']:.4f}")
    if not args.no_extras:
        out["bf16_vs_fp32"] = agreement_subset(plan, model, ref_q, images, bi, chunks, dev)
        qm = ref_q[bi.long()].contiguous()
        del plan
        out["regularised_merge"] = bench_normal(cfg, dev, det, qm, merged, model)
        out["phasing"] = bench_phasing(cfg, dev)
    return out


def bench_phasing(cfg, dev, iters=20):
    """Phasing at the workload's grid size: HIO iterations (two N^3 DFTs,
    the amplitude and support projections) and one shrinkwrap, on a seeded
    positive density in a ball (amplitudes from torch's FFT of it: input
    preparation only)."""
    import torch
    import paper_2109_05339_amd as spfel
    N = cfg.n_model
    g = torch.Generator(device=dev)
    g.manual_seed(int(cfg.seed_id) * 7919)
    c = torch.arange(N, device=dev, dtype=torch.float32) - N // 2
    R2 = c[:, None, None] ** 2 + c[None, :, None] ** 2 + c[None, None, :] ** 2
    sup = (R2 <= (N / 4) ** 2)
    rho = torch.rand((N, N, N), generator=g, device=dev) * sup
    amp = torch.fft.fftn(rho.double()).abs().float().contiguous()
    x = (torch.rand((N, N, N), generator=g, device=dev) * sup).contiguous()
    s8 = sup.to(torch.uint8).contiguous()
    p = spfel.Phase(N, device=dev)
    p.iterate(x, amp, s8, 1)                   # warm-up
    stream = torch.cuda.current_stream(dev)
    tm = Timer(torch, stream)
    with tm.span("hio"):
        err = p.iterate(x, amp, s8, iters, errors=True)
    with tm.span("shrinkwrap"):
        p.shrinkwrap(x, 2.0, 0.1)
    torch.cuda.synchronize()
    ms = tm.ms("hio")[0] / iters
    # two 3D DFTs per iteration: 3 contractions of N^4 complex MACs each
    # (the first real x complex), 8 flop per complex MAC
    flop = 2 * 3 * 8.0 * N ** 4
    e = err.cpu().numpy()
    return {"N": N, "iteration_ms": ms, "shrinkwrap_ms": tm.ms("shrinkwrap")[0],
            "dft_tflops": flop / (ms * 1e-3) / 1e12, "error_first": float(e[0]),
            "error_last": float(e[-1])}


def bench_normal(cfg, dev, det, quats, rhs, x0, n_sys=8, iters=10):
    """Regularised merging of Eq. (2) at the workload's size: the Toeplitz
    kernel (type-1 of the unit weights of every image at its matched
    orientation on 2N - 1 modes), then batched CG over n_sys lambdas on
    (A* A + lambda I) x = A* b + lambda x0 with A* b the step's merge."""
    import torch
    import paper_2109_05339_amd as spfel
    N = cfg.n_model
    n_img, P = quats.shape[0], det.shape[0]
    big = spfel.Plan(2 * N - 1, device=dev)
    big.set_detector(det)
    ones = torch.ones((n_img, P), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    tm = Timer(torch, stream)
    with tm.span("psf"):
        psf = big.merge_adjoint(quats, None, ones)
    del big, ones
    nm = spfel.Normal(N, domain=spfel.REAL, max_systems=n_sys, device=dev)
    nm.set_psf(psf)
    lam = (float(n_img) * P / N ** 3 * np.logspace(-3, 0.5, n_sys)).astype(np.float32)
    nm.solve(rhs, x0, lam, 1)           # warm-up
    torch.cuda.synchronize()
    with tm.span("solve0"):
        nm.solve(rhs, x0, lam, 0)
    with tm.span("solve"):
        xs, hist = nm.solve(rhs, x0, lam, iters, residuals=True)
    with tm.span("lcurve"):
        re, corner = nm.lcurve(xs, rhs, x0, lam, 0.0)
    torch.cuda.synchronize()
    ms0 = tm.ms("solve0")[0]
    per_it = (tm.ms("solve")[0] - ms0) / iters
    L = 2 * N
    # one application per system: REAL input contraction (4 flop per
    # real x complex term), five complex ones (8 flop), pointwise product
    work = n_sys * (4.0 * N ** 3 * L + 8.0 * (N ** 2 * L * L + N * L ** 3 + L ** 3 * N
                                           + L ** 2 * N * N + L * N ** 3) + 6.0 * L ** 3)
    h = hist.cpu().numpy()
    return {"systems": n_sys, "N": N, "L": L, "psf_merge_ms": tm.ms("psf")[0],
            "cg_iteration_ms": per_it, "lcurve_ms": tm.ms("lcurve")[0],
            "apply_tflops": work / (per_it * 1e-3) / 1e12,
            "residual_drop": float(np.max(h[:, -1] / h[:, 0])),
            "corner": int(corner.item())}


def agreement_subset(plan, model, ref_q, images, bi_bf16, chunks, dev, n_sub=1024):
    """The FP32 matcher (expanded form, float32 MFMA GEMM) over every
    reference orientation for the first n_sub images; fraction of images on
    which its argmin equals the BF16 path's."""
    import torch
    import paper_2109_05339_amd as spfel
    sub = images[:n_sub].contiguous()
    dn = spfel.row_norm2(sub)
    bi, bd = spfel.new_best(n_sub, dev)
    plan.set_model(model)
    for c0, c1 in chunks:
        S, sn = plan.slice(ref_q[c0:c1], norms=True)
        spfel.match(S, sn, sub, dn, bi, bd, m_offset=c0)
        del S
    a = bi.cpu().numpy()
    b = bi_bf16[:n_sub].cpu().numpy()
    log(f"bf16 vs fp32 argmin agreement on {n_sub} images: {np.mean(a == b):.4f}")
    return {"images": n_sub, "argmin_agreement": float(np.mean(a == b))}


def _copy_calibration(torch, dev):
    src = torch.ones((1 << 28,), dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    log("counter run done: one chunk of each hot kernel, one merge, one 1 GiB copy")
    print(json.dumps({"counters_run": True, "copy_bytes": src.numel() * 4}), flush=True)


def bench_plain(args, cfg, dev, steps, warmup):
    """Workloads 1-3 (2 by default): the FP32 form.  One step = set_model +
    slicing of all orientations with norms + FP32 distance GEMM with argmin;
    the BF16 form's step on the same inputs is timed beside it."""
    import torch
    import synth
    import paper_2109_05339_amd as spfel
    M, n_img, P, N = cfg.n_refs, cfg.n_images, cfg.n_pix, cfg.n_model
    t0 = time.time()
    m_host, _ = synth.intensity_model(cfg)
    det = torch.from_numpy(synth.detector_q(cfg.n_det).astype(np.float32)).to(dev)
    ref_q = torch.from_numpy(synth.quaternions(cfg, "ref_quats", M).astype(np.float32)).to(dev)
    img_q = torch.from_numpy(synth.quaternions(cfg, "image_quats", n_img).astype(np.float32)).to(dev)
    plan = spfel.Plan(N, device=dev)
    plan.set_detector(det)
    images, alpha = _render_images(plan, cfg, dev, img_q, m_host)
    model = torch.from_numpy((alpha * m_host).astype(np.float32)).to(dev)
    f32 = spfel.ImagesF32(images)
    b16 = spfel.ImagesBF16(images)
    ws = torch.empty((max(spfel.match_workspace_bytes(M, n_img, P, m)
                          for m in (spfel.MATCH_FP32, spfel.MATCH_BF16_RESCORE8)),),
                     dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    log(f"workload {cfg.cid} inputs ready in {time.time() - t0:.1f}s: M={M} n_img={n_img} P={P}")
    stream = torch.cuda.current_stream(dev)

    def step_fp32(tm):
        with tm.span("set_model"):
            plan.set_model(model)
        with tm.span("slice"):
            S, sn = plan.slice(ref_q, norms=True)
        bi, bd = spfel.new_best(n_img, dev)
        with tm.span("match"):
            spfel.match(S, sn, f32.x, f32.norm2, bi, bd, workspace=ws)
        return bi

    def step_bf16(tm):
        with tm.span("set_model"):
            plan.set_model(model)
        with tm.span("slice"):
            S, _ = plan.slice(ref_q)
        with tm.span("centre"):
            sb, sn, se = spfel.bf16_centred(S, b16.centre)
        bi, bd = spfel.new_best(n_img, dev)
        with tm.span("match"):
            spfel.match(sb, sn, b16.b16, b16.norm2, bi, bd, mode=spfel.MATCH_BF16_RESCORE8,
                        slices_f32=S, images_f32=images, slice_err=se, image_err=b16.err,
                        workspace=ws)
        return bi

    if args.counters:
        step_fp32(Timer(torch, stream, on=False))
        step_bf16(Timer(torch, stream, on=False))
        plan.merge_adjoint(ref_q[:n_img].contiguous(), None, images)
        _copy_calibration(torch, dev)
        return None

    def timed(fn):
        for _ in range(warmup):
            fn(Timer(torch, stream, on=False))
        torch.cuda.synchronize()
        tm = Timer(torch, stream)
        t0 = time.perf_counter()
        for _ in range(steps):
            bi = fn(tm)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps * 1e3, tm, bi

    wall, tm, bi32 = timed(step_fp32)
    comps = float(M) * n_img * P
    per = {k: float(np.mean(tm.ms(k))) for k in tm.marks}
    r_slice = roofline("interp_tiled_kernel", "alu", INTERP_FLOP_PER_POINT * M * P, per["slice"],
                       PEAK_FP32_VECTOR_TFLOPS, "TFLOP/s",
                       traffic_of("interp_tiled_kernel", cfg.cid))
    r_match = roofline("match_f32_kernel", "mfma", 2.0 * comps, per["match"],
                       PEAK_FP32_MFMA_TFLOPS, "TFLOP/s", traffic_of("match_f32_kernel", cfg.cid))
    log(f"fp32 step {wall:.3f} ms; slice {per['slice']:.3f} ms, match {per['match']:.3f} ms")
    wall_b, tmb, bib = timed(step_bf16)
    perb = {k: float(np.mean(tmb.ms(k))) for k in tmb.marks}
    agree = float((bib == bi32).float().mean())
    log(f"bf16 step {wall_b:.3f} ms, agreement {agree:.4f}")
    # type-1 merge of every image at its matched orientation
    mq = ref_q[bi32.long()].contiguous()
    tmm = Timer(torch, stream)
    for _ in range(3):
        with tmm.span("merge"):
            plan.merge_adjoint(mq, None, images)
    torch.cuda.synchronize()
    merge_ms = float(np.mean(tmm.ms("merge")[1:]))
    return {
        "metric": "slice+match pixel-comparisons/s",
        "value": comps / (wall * 1e-3),
        "unit": "pixel-comparisons/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup, "ms_per_step": wall,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": (f"{N}^3 float32 intensity model ({cfg.n_atoms} scatterers), "
                                f"{cfg.n_det}x{cfg.n_det} detector, {M} reference orientations, "
                                f"{n_img} Poisson images at {cfg.photons:g} photons/px; step = "
                                "set_model + type-2 slicing + float32 distance GEMM with argmin"),
                   "M": M, "n_img": n_img, "P": P, "N": N},
        "kernel_ms": per,
        "nufft_type2_pts_per_s": M * P / (per["slice"] * 1e-3),
        "roofline": r_slice if per["slice"] >= per["match"] else r_match,
        "roofline_kernels": [r_slice, r_match],
        "bf16_rescore": {"ms_per_step": wall_b, "kernel_ms": perb,
                         "pixel_comparisons_per_s": comps / (wall_b * 1e-3),
                         "argmin_agreement_vs_fp32": agree},
        "merge_adjoint_ms": merge_ms,
        "nufft_type1_pts_per_s": n_img * P / (merge_ms * 1e-3),
    }


def bench_gradient(args, cfg, dev):
    """Workload 4: weighted slice-to-image loss of a 65^3 complex model over
    4,096 images at given orientations and its gradient (type-1 spread of
    the residual), slices recomputed per chunk of 1,024 images."""
    import torch
    import synth
    import paper_2109_05339_amd as spfel
    n_img, P, N = cfg.n_images, cfg.n_pix, cfg.n_model
    m_host, _ = synth.intensity_model(cfg)
    mc = synth.complex_perturbation(cfg, m_host)
    det = torch.from_numpy(synth.detector_q(cfg.n_det).astype(np.float32)).to(dev)
    img_q = torch.from_numpy(synth.quaternions(cfg, "image_quats", n_img).astype(np.float32)).to(dev)
    plan = spfel.Plan(N, domain=spfel.COMPLEX, device=dev)
    plan.set_detector(det)
    target = torch.from_numpy(m_host.astype(np.complex64)).to(dev)
    plan.set_model(target)
    d = torch.empty((n_img, P), dtype=torch.complex64, device=dev)
    for c0 in range(0, n_img, 1024):
        d[c0:c0 + 1024] = plan.slice(img_q[c0:c0 + 1024])[0]
    w = torch.from_numpy(synth.pixel_weights(cfg, n_img, P)).to(dev)
    model = torch.from_numpy(mc.astype(np.complex64)).to(dev)

    def step():
        mt = model.clone().requires_grad_(True)
        L = spfel.slice_loss(mt, img_q, None, d, w, plan, chunk=1024)
        L.backward()
        return L, mt.grad

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    pts = float(n_img) * P
    out = {
        "metric": "loss+gradient points/s", "value": pts / (ms * 1e-3), "unit": "points/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64", "data": "synthetic",
        "config": {"workload": (f"{N}^3 complex64 model, {cfg.n_det}x{cfg.n_det} detector, "
                                f"{n_img} images, per-pixel weights in [0.5, 1); forward = "
                                "type-2 slices + weighted loss, backward = recomputed slices + "
                                "type-1 spread of 2 w (s - d), chunks of 1,024 images"),
                   "n_img": n_img, "P": P, "N": N},
    }
    print(json.dumps(out), flush=True)
    return 0


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle as it stands, in a process pool on this host.

_ORACLE = {}


def _oracle_slice(task):
    from oracle import geometry, nufft
    q, det = task
    x = geometry.slice_points(q, det).reshape(-1, 3)
    return nufft.nufft2(_ORACLE["model"], x, real=True).reshape(len(q), -1)


def _oracle_merge(task):
    from oracle import geometry, nufft
    q, det, y = task
    x = geometry.slice_points(q, det).reshape(-1, 3)
    return nufft.nufft1(y.reshape(-1), x, _ORACLE["model"].shape[0], real=True)


def cpu_baseline(cfg, args):
    """The FP64 oracle on a bounded sample of the step, run before the GPU
    is initialised: type-2 slicing of the first ``--cpu-sample`` orientations
    of the first chunk (split over a process pool), their distances to the
    first 1,024 images (float64 BLAS) with argmin, and the type-1 merge of
    one image per worker.  Inputs come from synth alone (the workload's model
    and seeded Poisson images of the same shape and photon level).  Rates are
    measured on the sample; the step time is extrapolated linearly."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    import synth
    from oracle import match
    workers = args.cpu_workers or min(16, len(os.sched_getaffinity(0)))
    m_host, _ = synth.intensity_model(cfg)
    _ORACLE["model"] = m_host
    det = synth.detector_q(cfg.n_det).astype(np.float32).astype(np.float64)
    n_s = max(workers, args.cpu_sample)
    q = synth.quaternions(cfg, "ref_quats", n_s).astype(np.float32).astype(np.float64)
    n_match = min(1024, cfg.n_images)
    images = synth.poisson_counts(cfg, np.full((n_match, cfg.n_pix), float(cfg.photons)))
    log(f"cpu baseline: oracle slicing {n_s} orientations on {workers} processes")
    ctx = mp.get_context("fork")
    with ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        parts = np.array_split(np.arange(n_s), workers)
        t0 = time.perf_counter()
        S = np.concatenate(list(ex.map(_oracle_slice, [(q[p], det) for p in parts])))
        t_slice = time.perf_counter() - t0
        log(f"cpu baseline: merging {workers} images on {workers} processes")
        qi = synth.quaternions(cfg, "image_quats", workers).astype(np.float32).astype(np.float64)
        t0 = time.perf_counter()
        f = sum(ex.map(_oracle_merge, [(qi[i:i + 1], det, images[i]) for i in range(workers)]))
        t_merge = time.perf_counter() - t0
    del f
    t0 = time.perf_counter()
    Dm = match.distances_expanded(S, images.astype(np.float64))
    match.argmin_first(Dm)
    t_match = time.perf_counter() - t0
    pts_s = n_s * cfg.n_pix / t_slice
    comps_s = n_s * n_match * cfg.n_pix / t_match
    merge_pts_s = workers * cfg.n_pix / t_merge
    M, n_img, P = cfg.n_refs, cfg.n_images, cfg.n_pix
    t_step = M * P / pts_s + float(M) * n_img * P / comps_s + n_img * P / merge_pts_s
    try:
        from threadpoolctl import threadpool_info
        blas = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        blas = workers
    return {
        "value": float(M) * n_img * P / t_step,
        "unit": "pixel-comparisons/s",
        "cores": workers,
        "kind": "oracle",
        "sample": (f"float64 oracle: type-2 slicing of {n_s} of the first chunk's orientations "
                   f"({n_s * P:.3g} points) on a pool of {workers} processes; their distances "
                   f"to the first {n_match} images with argmin (float64 BLAS, {blas} threads); "
                   f"type-1 merge of {workers} images, one per process.  Measured rates below; "
                   "the full step time is extrapolated linearly from them"),
        "measured": {"type2_pts_per_s": pts_s, "match_pixel_comparisons_per_s": comps_s,
                     "type1_pts_per_s": merge_pts_s,
                     "seconds": {"slice": t_slice, "match": t_match, "merge": t_merge}},
        "extrapolated_step_s": t_step,
        "cpu_model": _cpu_model(),
    }


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    sys.exit(main())
