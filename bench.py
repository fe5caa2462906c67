"""Slice-and-match throughput on one MI355X.

Workload (default): 65^3 float32 intensity model of a 200-scatterer
molecule, 128 x 128 detector (16,384 Ewald-sphere pixels), 10,000 reference
orientations, 2,048 Poisson images at 20 photons/pixel.  One step is one
pass of the orientation-determination hot path over that batch:

  set_model (deconvolve + separable transform to the 130^3 fine grid)
  -> slice all 10,000 orientations (type-2 NUFFT, float32, + norms)
  -> match every image against every slice (float32 MFMA GEMM + argmin).

The JSON line reports pixel-comparisons/s = M * n_img * P / step time
(inputs resident in HBM), the float32 distance GEMM against the MI355X
float32 matrix peak, the BF16+rescore matcher on the same inputs (time and
argmin agreement with float32), the type-2 and type-1 NUFFT point rates,
and the CPU oracle timed on a bounded sample on this host.
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
# algorithmic work of one interpolated point at w = 6: w^3 multiply-adds
INTERP_FLOP_PER_POINT = 2 * 6 ** 3


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2, help="workload id (2: the default above)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip BF16 and spread side runs")
    ap.add_argument("--cpu-sample", type=int, default=200, help="orientations in the oracle sample")
    ap.add_argument("--counters", action="store_true",
                    help="counter-collection run: one step of each path and a plain 1 GiB "
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
    import torch
    import synth
    import paper_2109_05339_amd as spfel

    cfg = synth.config(args.config)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.config == 5:
        return bench_streaming(args, cfg, dev)
    if args.config == 4:
        return bench_gradient(args, cfg, dev)
    M, n_img, P, N = cfg.n_refs, cfg.n_images, cfg.n_pix, cfg.n_model

    # ---- inputs (not timed) ----
    t0 = time.time()
    m_host, _ = synth.intensity_model(cfg)
    det = torch.from_numpy(synth.detector_q(cfg.n_det).astype(np.float32)).to(dev)
    ref_q = torch.from_numpy(synth.quaternions(cfg, "ref_quats", M).astype(np.float32)).to(dev)
    img_q = torch.from_numpy(synth.quaternions(cfg, "image_quats", n_img).astype(np.float32)).to(dev)
    plan = spfel.Plan(N, device=dev)
    plan.set_detector(det)
    plan.set_model(torch.from_numpy(m_host.astype(np.float32)).to(dev))
    lam0 = plan.slice(img_q)[0].clamp_(min=0).cpu().numpy()
    alpha = synth.photon_scale(lam0, cfg.photons)
    images = torch.from_numpy(synth.poisson_counts(cfg, alpha * lam0)).to(dev)
    del lam0
    model = torch.from_numpy((alpha * m_host).astype(np.float32)).to(dev)
    dnorm = spfel.row_norm2(images)
    images_bf16 = images.to(torch.bfloat16)
    images_x3 = spfel.split_bf16(images)
    ws = torch.empty((max(spfel.match_workspace_bytes(M, n_img, P, m)
                          for m in (spfel.MATCH_FP32, spfel.MATCH_BF16_RESCORE8,
                                    spfel.MATCH_BF16X3_RESCORE8)),),
                     dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    log(f"inputs ready in {time.time() - t0:.1f}s: M={M} n_img={n_img} P={P} N={N}")

    stream = torch.cuda.current_stream(dev)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def step(mode, marks=None):
        """One pass: set_model, slice all orientations (with norms, and the
        BF16 forms the mode needs), match every image against every slice."""
        e = [ev() for _ in range(2)] if marks is not None else None
        if e: e[0].record(stream)
        plan.set_model(model)
        S, Sb, sn = plan.slice(ref_q, out=True, bf16=mode == spfel.MATCH_BF16_RESCORE8, norms=True)
        bi, bd = spfel.new_best(n_img, dev)
        if mode == spfel.MATCH_FP32:
            spfel.match(S, sn, images, dnorm, bi, bd, workspace=ws)
        elif mode == spfel.MATCH_BF16_RESCORE8:
            spfel.match(Sb, sn, images_bf16, dnorm, bi, bd, mode=mode, slices_f32=S,
                        images_f32=images, workspace=ws)
        else:
            spfel.match(spfel.split_bf16(S), sn, images_x3, dnorm, bi, bd, mode=mode,
                        slices_f32=S, images_f32=images, workspace=ws)
        if e: e[1].record(stream)
        if marks is not None:
            marks.append(e)
        return bi, bd

    step_fp32 = lambda marks=None: step(spfel.MATCH_FP32, marks)  # noqa: E731
    step_bf16 = lambda marks=None: step(spfel.MATCH_BF16_RESCORE8, marks)  # noqa: E731
    step_bf16x3 = lambda marks=None: step(spfel.MATCH_BF16X3_RESCORE8, marks)  # noqa: E731

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        marks = []
        t0 = time.perf_counter()
        for _ in range(steps):
            fn(marks)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        step_ms = float(np.mean([a.elapsed_time(b) for a, b in marks]))
        return wall * 1e3, step_ms

    def kernel_times(reps):
        """Unpipelined launches of the two hot kernels, each bracketed by
        HIP events on its own (the current) stream."""
        plan.set_model(model)
        S, _, sn = plan.slice(ref_q, norms=True)
        bi, bd = spfel.new_best(n_img, dev)
        spfel.match(S, sn, images, dnorm, bi, bd, workspace=ws)
        torch.cuda.synchronize()
        t_slice, t_match = [], []
        for _ in range(reps):
            a, b, c = ev(), ev(), ev()
            a.record(stream)
            plan.slice(ref_q, out=True, norms=False)
            b.record(stream)
            bi, bd = spfel.new_best(n_img, dev)
            c.record(stream)
            d = ev()
            spfel.match(S, sn, images, dnorm, bi, bd, workspace=ws)
            d.record(stream)
            t_slice.append((a, b))
            t_match.append((c, d))
        torch.cuda.synchronize()
        return (float(np.mean([a.elapsed_time(b) for a, b in t_slice])),
                float(np.mean([c.elapsed_time(d) for c, d in t_match])))

    if args.counters:
        kernel_times(1)
        step_bf16()
        plan.merge_adjoint(ref_q[:n_img].contiguous(), None, images)
        src = torch.ones((1 << 28,), dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("counter run done: unpipelined slice + fp32 match, one bf16 step, one merge, one 1 GiB copy")
        print(json.dumps({"counters_run": True, "copy_bytes": src.numel() * 4}), flush=True)
        return 0

    log(f"timing fp32 path: {args.warmup} warmup + {args.steps} steps")
    wall_ms, step_ms = timed(step_fp32, args.steps, args.warmup)
    ms_per_step = max(wall_ms, step_ms)
    comps = float(M) * n_img * P
    value = comps / (ms_per_step * 1e-3)
    slice_ms, match_ms = kernel_times(max(3, args.steps // 2))
    gemm_flops = 2.0 * comps
    gemm_tf = gemm_flops / (match_ms * 1e-3) / 1e12
    interp_tf = INTERP_FLOP_PER_POINT * M * P / (slice_ms * 1e-3) / 1e12
    log(f"fp32 step {ms_per_step:.3f} ms; unpipelined slice {slice_ms:.3f} ms, match {match_ms:.3f} ms")
    roof_match = {"kernel": "match_f32_kernel", "bound": "mfma", "achieved": gemm_tf,
                  "peak": PEAK_FP32_MFMA_TFLOPS, "unit": "TFLOP/s",
                  "frac": gemm_tf / PEAK_FP32_MFMA_TFLOPS,
                  "traffic": traffic_of("match_f32_kernel", args.config)}
    roof_interp = {"kernel": "interp_tiled_kernel", "bound": "alu", "achieved": interp_tf,
                   "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                   "frac": interp_tf / PEAK_FP32_VECTOR_TFLOPS,
                   "traffic": traffic_of("interp_tiled_kernel", args.config)}
    dominant = roof_interp if slice_ms >= match_ms else roof_match

    out = {
        "metric": "slice+match pixel-comparisons/s",
        "value": value,
        "unit": "pixel-comparisons/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{N}^3 float32 intensity model ({cfg.n_atoms} scatterers), "
                         f"{cfg.n_det}x{cfg.n_det} detector, {M} reference orientations, "
                         f"{n_img} Poisson images at {cfg.photons:g} photons/px; step = "
                         "set_model + type-2 slicing + float32 distance GEMM with argmin"),
            "M": M, "n_img": n_img, "P": P, "N": N, "kernel_width": 6, "upsampfac": 2.0,
        },
        "unpipelined_ms": {"slice_all": slice_ms, "match_fp32_all": match_ms},
        "nufft_type2_pts_per_s": M * P / (slice_ms * 1e-3),
        "roofline": dominant,
        "roofline_kernels": [roof_interp, roof_match],
    }

    if not args.no_extras:
        bi32, _ = step_fp32()
        for name, fn in (("bf16_rescore", step_bf16), ("bf16x3_rescore", step_bf16x3)):
            log(f"timing {name} path")
            wall_b, step_b = timed(fn, max(5, args.steps // 2), 2)
            bib, _ = fn()
            agree = float((bib == bi32).float().mean())
            out[name] = {
                "ms_per_step": max(wall_b, step_b),
                "pixel_comparisons_per_s": comps / (max(wall_b, step_b) * 1e-3),
                "argmin_agreement_vs_fp32": agree,
            }
            log(f"{name} step {max(wall_b, step_b):.3f} ms, agreement {agree:.4f}")
        # BF16 GEMM kernel alone (unpipelined) on the same slices
        plan.set_model(model)
        S, Sb, sn = plan.slice(ref_q, bf16=True, norms=True)
        a, b = ev(), ev()
        torch.cuda.synchronize()
        a.record(stream)
        for _ in range(5):
            bi, bd = spfel.new_best(n_img, dev)
            spfel.match(Sb, sn, images_bf16, dnorm, bi, bd, mode=spfel.MATCH_BF16_RESCORE8,
                        slices_f32=S, images_f32=images, workspace=ws)
        b.record(stream)
        torch.cuda.synchronize()
        t = a.elapsed_time(b) / 5
        out["bf16_rescore"]["match_ms_unpipelined"] = t
        del S, Sb, sn
        # type-1 spread of every image at its matched orientation (merge A* b)
        mq = ref_q[bi32.long()].contiguous()
        plan.merge_adjoint(mq, None, images)
        torch.cuda.synchronize()
        a, b = ev(), ev()
        reps = 5
        a.record(stream)
        for _ in range(reps):
            plan.merge_adjoint(mq, None, images)
        b.record(stream)
        torch.cuda.synchronize()
        t1 = a.elapsed_time(b) / reps
        out["merge_adjoint_ms"] = t1
        out["nufft_type1_pts_per_s"] = n_img * P / (t1 * 1e-3)
        log(f"merge_adjoint {t1:.3f} ms")

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, m_host, n_img, args.cpu_sample, comps)
    print(json.dumps(out), flush=True)
    return 0


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
    """Workload 5: 100,000 reference orientations streamed in chunks of 8,192
    (sliced and never stored in full), BF16 matcher with per-chunk top-8
    FP32 rescoring into a running best, then the type-1 merge of all images
    at their matched orientations."""
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
    dnorm = spfel.row_norm2(images)
    images_bf16 = images.to(torch.bfloat16)
    merged = torch.empty((N, N, N), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    log(f"workload 5 inputs ready in {time.time() - t0:.1f}s")
    stream = torch.cuda.current_stream(dev)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def step(marks=None):
        e = [ev() for _ in range(3)] if marks is not None else None
        if e: e[0].record(stream)
        plan.set_model(model)
        bi, bd = spfel.new_best(n_img, dev)
        plan.orient(ref_q, images_bf16, dnorm, bi, bd, mode=spfel.MATCH_BF16_RESCORE8, chunk=C,
                    images_f32=images, overlap=False)
        if e: e[1].record(stream)
        plan.merge_adjoint(ref_q[bi.long()].contiguous(), None, images, out=merged)
        if e: e[2].record(stream)
        if marks is not None:
            marks.append(e)
        return bi

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    marks = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(marks)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps * 1e3
    match_ms = float(np.mean([a.elapsed_time(b) for a, b, _ in marks]))
    merge_ms = float(np.mean([b.elapsed_time(c) for _, b, c in marks]))
    comps = float(M) * n_img * P
    out = {
        "metric": "slice+match pixel-comparisons/s",
        "value": comps / (match_ms * 1e-3),
        "unit": "pixel-comparisons/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16+f32", "data": "synthetic",
        "config": {"workload": (f"{N}^3 float32 model ({cfg.n_atoms} scatterers), {cfg.n_det}x"
                                f"{cfg.n_det} detector, {M} reference orientations streamed in "
                                f"chunks of {C}, {n_img} Poisson images at {cfg.photons:g} "
                                "photons/px; BF16 matcher with per-chunk top-8 FP32 rescore, "
                                "then the type-1 merge of all images at their matched orientations"),
                   "M": M, "n_img": n_img, "P": P, "N": N, "chunk": C},
        "breakdown_ms": {"stream_slice+match": match_ms, "merge_adjoint": merge_ms},
        "nufft_type1_pts_per_s": n_img * P / (merge_ms * 1e-3),
    }
    print(json.dumps(out), flush=True)
    return 0


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


def cpu_baseline(cfg, model, n_img, n_sample, comps_total):
    """The FP64 oracle on a bounded sample of the same step: the fine grid
    once, ``n_sample`` orientations sliced, and those slices matched against
    ``n_img`` images; scaled to the full step's pixel-comparisons/s.  Its
    inputs come from synth alone (the workload's model and seeded Poisson
    images of the same shape and photon level; the values do not change the
    oracle's running time)."""
    import synth
    from oracle import geometry, match, nufft
    images = synth.poisson_counts(cfg, np.full((n_img, cfg.n_pix), float(cfg.photons)))
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = len(os.sched_getaffinity(0))
    det = synth.detector_q(cfg.n_det).astype(np.float32).astype(np.float64)
    q = synth.quaternions(cfg, "ref_quats", n_sample).astype(np.float32).astype(np.float64)
    log(f"cpu baseline: oracle on {n_sample} orientations x {images.shape[0]} images")
    t0 = time.perf_counter()
    nufft.fine_grid(model, real=True)
    t_grid = time.perf_counter() - t0
    t0 = time.perf_counter()
    S = nufft.nufft2(model, geometry.slice_points(q, det).reshape(-1, 3), real=True).reshape(n_sample, -1)
    t_slice = time.perf_counter() - t0
    t0 = time.perf_counter()
    Dm = match.distances_expanded(S, images.astype(np.float64))
    match.argmin_first(Dm)
    t_match = time.perf_counter() - t0
    per_orient = (t_slice + t_match) / n_sample
    t_step = t_grid + per_orient * cfg.n_refs
    return {
        "value": comps_total / t_step,
        "unit": "pixel-comparisons/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"{n_sample} of {cfg.n_refs} orientations sliced by the float64 oracle "
                   f"(single-threaded NumPy) and matched against all {images.shape[0]} images "
                   f"(float64 BLAS, {threads} threads); fine grid once; step time "
                   f"extrapolated linearly in orientations"),
        "sample_seconds": t_grid + t_slice + t_match,
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
