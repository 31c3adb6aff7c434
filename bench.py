"""Throughput of per-slice parallel-beam filtered back-projection on one MI355X.

One step is the whole hot path over one slab: the windowed ramp filter of every
sinogram row (xct_filter) followed by the back-projection of every filtered row
into its slice (xct_backproject, weight pi/N_p).  The workload is the paper's
resolution: 16 slices of 8192^2, 6144 angles over a half turn, 8192 detector
bins, Hann window, seeded binder discs holding 200 aggregate / void ellipses
(closed-form line integrals, generated on the GPU before timing).  Inputs are
resident in HBM when the timed region starts.

value = voxel x angle updates per second (16 * 8192^2 * 6144 per step) / 1e9,
for the FP32-stored sinogram; the FP16- and BF16-stored runs (FP32 arithmetic)
are reported beside it, each with its relative L2 error against the FP64 oracle
on a sample of pixels.

    python bench.py [--steps K] [--warmup W] [--slices S] [--no-oracle]
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GUPS (voxel×angle updates/s) for FBP, fp32 vs fp16-storage, at stated L2 error"
FLOPS_PER_UPDATE = 6  # coordinate FMA (2), fraction (1), interpolation FMA (2), accumulate (1)
FP32_VECTOR_PEAK_TFLOPS = 157.3
LDS_BYTES_PER_UPDATE = 8  # one (a, d) FP32 pair per interpolation
HBM_PEAK_GBPS = 8000.0
# HBM bytes of one FP32 back-projection launch of the full 16-slice slab:
# rocprofv3 FETCH_SIZE x 2.0 plus WRITE_SIZE x 1.0 (the factors under which a
# plain 1 GiB device copy reads and writes 1 GiB), from the counter passes in
# profiles/bp_sym_kernel_slab16_8192.txt.  Valid for that kernel build only.
BP_TRAFFIC_BYTES = 45_915_450 * 1024 * 2 + 4_196_195 * 1024


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--slices", type=int, default=16, help="slices in the slab (16 = full workload)")
    ap.add_argument("--storage", default="f32,f16,bf16")
    ap.add_argument("--filtered", default="f32", choices=["f32", "f16"],
                    help="storage of the filtered rows between the two kernels")
    ap.add_argument("--no-oracle", action="store_true", help="skip the error and CPU-baseline legs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device-to-device copy three times (a known "
                         "traffic reference for hardware byte counters)")
    ap.add_argument("--main-only", action="store_true",
                    help="time only the 16 x 8192^2 slab (skip the uneven-batch and adjoint-pair legs)")
    ap.add_argument("--sample-rows", type=int, default=32,
                    help="rows of one slice checked against / timed on the FP64 oracle")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def _timed(torch, stream, fn, steps, warmup):
    """Mean milliseconds of fn() over `steps` launches, after `warmup` untimed
    ones, from HIP events on the stream the launches go to."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _alu_roofline(kernel, updates, ms):
    achieved = FLOPS_PER_UPDATE * updates / (ms * 1e-3) / 1e12
    return {"kernel": kernel, "bound": "alu", "achieved": achieved,
            "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP32_VECTOR_PEAK_TFLOPS}


def measure_raw_pipeline(xct, torch, synth, spec, p64, filt, stream, steps, warmup):
    """Raw detector counts to a uint16 CT-number volume for the slab: the
    fused front end (Beer-Lambert, blur sigma 1, Hann ramp filter, regrouping
    of the projection stack by detector row) and the back-projection with the
    CT-number epilogue (binder density as water, [-1000, 3000] HU)."""
    g = spec.geom
    S = p64.shape[0]
    kappa = synth.attenuation_scale(float(p64.max()))
    dark, flat = synth.detector_fields(S, g.n_det, 3, device="cuda")
    proj = synth.raw_counts(p64, dark, flat, kappa)          # [N_p][S][N_c] uint16
    codes = torch.empty((S, g.ny, g.nx), dtype=torch.uint16, device="cuda")
    scale = math.pi / g.n_angles / kappa                      # FBP of kappa p, in pixel units
    fe_ms = _timed(torch, stream, lambda: xct.xct_preprocess_filter(
        g, proj, dark, flat, 0, filt, spec.window, 1.0, 1.0), steps, warmup)
    bp_ms = _timed(torch, stream, lambda: xct.xct_backproject_u16(
        g, filt, codes, scale, 0.3, -1000.0, 3000.0), steps, warmup)
    updates = S * g.nx * g.ny * g.n_angles
    fe_bytes = proj.numel() * 2 + filt.numel() * filt.element_size() + 2 * dark.numel() * 4
    log(f"raw pipeline: front end {fe_ms:.3f} ms, back-projection to uint16 {bp_ms:.3f} ms")
    del proj, codes
    return {
        "workload": (f"{S} x 8192^2 slab from uint16 counts [6144][{S}][8192] with dark/flat fields: "
                     "xct_preprocess_filter (sigma 1, Hann) + xct_backproject_u16"),
        "front_end_ms": fe_ms, "front_end_gbps": fe_bytes / (fe_ms * 1e-3) / 1e9,
        "backproject_u16_ms": bp_ms, "ms": fe_ms + bp_ms,
        "gups": updates / ((fe_ms + bp_ms) * 1e-3) / 1e9,
    }


def measure_offset_scan(xct, torch, configs, stream, steps, warmup):
    """Full-turn offset scan through xct_fbp_batch: 8 x 4096^2, 8192 angles,
    4096 bins with the axis at bin 1024, redundancy overlap 1024, Hann
    (weighted rows filtered on the 6143-bin virtual detector, one symmetric
    back-projection launch over both half turns)."""
    spec = configs.c6()
    g = spec.geom
    S = spec.n_slices
    p = torch.empty((S, g.n_angles, g.n_det), dtype=torch.float32, device="cuda")
    for s in range(S):
        p[s] = spec.sinogram(s, device="cuda").to(torch.float32)
    img = torch.empty((S, g.ny, g.nx), dtype=torch.float32, device="cuda")
    slabs = [(g, p, img, spec.offset_overlap)]
    ws = torch.empty(xct.xct_fbp_workspace_bytes(slabs), dtype=torch.uint8, device="cuda")
    ms = _timed(torch, stream, lambda: xct.xct_fbp_batch(slabs, spec.window, workspace=ws),
                steps, warmup)
    log(f"offset scan: {ms:.3f} ms")
    del p, img, ws
    return {
        "workload": (
            "8 x 4096^2 offset scan, 8192 angles over a full turn, 4096 bins, axis at bin 1024, "
            "overlap 1024, Hann; xct_fbp_batch"),
        "ms": ms, "gups": spec.updates / (ms * 1e-3) / 1e9, "updates": spec.updates,
    }


def measure_uneven_batch(xct, torch, configs, encode_storage, stream, steps, warmup):
    """Filter + back-projection of the uneven batch (24 x 512^2, 12 x 1024^2,
    4 x 2048^2, BF16-stored, Ram-Lak) in one persistent launch per kernel,
    against the same slabs launched one at a time."""
    specs = configs.c5()
    slabs = []
    for spec in specs:
        g = spec.geom
        p = torch.stack([spec.sinogram(s, device="cuda") for s in range(spec.n_slices)])
        sb = encode_storage(p, "bf16").contiguous()
        slabs.append((g, sb, torch.empty((spec.n_slices, g.ny, g.nx), device="cuda")))
        del p
    ws = torch.empty(xct.xct_fbp_workspace_bytes(slabs), dtype=torch.uint8, device="cuda")
    updates = [spec.n_slices * spec.geom.nx * spec.geom.ny * spec.geom.n_angles for spec in specs]
    ms = _timed(torch, stream, lambda: xct.xct_fbp_batch(slabs, "ram_lak", workspace=ws),
                steps, warmup)
    alone = [_timed(torch, stream, lambda sl=sl: xct.xct_fbp_batch([sl], "ram_lak", workspace=ws),
                    steps, warmup) for sl in slabs]
    log(f"uneven batch: {ms:.3f} ms in one launch, {sum(alone):.3f} ms slab by slab")
    return {
        "workload": "24 x 512^2 (720 angles), 12 x 1024^2 (1440), 4 x 2048^2 (2048); bf16 storage, "
                    "Ram-Lak; xct_fbp_batch, one persistent back-projection launch",
        "ms": ms, "gups": sum(updates) / (ms * 1e-3) / 1e9,
        "slab_by_slab_ms": alone, "slab_by_slab_gups": sum(updates) / (sum(alone) * 1e-3) / 1e9,
        "updates": sum(updates),
    }


def measure_adjoint_pair(xct, torch, configs, stream, steps, warmup):
    """Forward projector P, its transpose, and one streamed least-squares
    gradient (loss ||P x - y||^2 and 2 P^T (P x - y)) on 32 x 1024^2, 1440
    angles, 1449 bins."""
    spec = configs.c4()
    g = spec.geom
    S = spec.n_slices
    y = torch.stack([spec.sinogram(s, device="cuda") for s in range(S)]).to(torch.float32)
    truth = torch.stack([spec.truth(s, device="cuda", supersample=2) for s in range(S)])
    gen = torch.Generator(device="cuda").manual_seed(4)
    x = (truth + 0.05 * torch.randn(truth.shape, generator=gen, device="cuda",
                                    dtype=torch.float64)).to(torch.float32).contiguous()
    del truth
    y = y.contiguous()
    px = torch.empty_like(y)
    ptg = torch.empty_like(x)
    sc = xct.adjoint_scale(g)
    updates = S * g.nx * g.ny * g.n_angles
    fp_ms = _timed(torch, stream, lambda: xct.xct_forward_project(g, x, px), steps, warmup)
    bp_ms = _timed(torch, stream, lambda: xct.xct_backproject(g, y, ptg, sc, False), steps, warmup)
    gr_ms = _timed(torch, stream, lambda: xct.ls_loss_and_grad(x, y, g), steps, warmup)
    log(f"adjoint pair: P {fp_ms:.3f} ms, P^T {bp_ms:.3f} ms, gradient {gr_ms:.3f} ms")
    return {
        "workload": "32 x 1024^2, 1440 angles, 1449 bins; x = phantom + 0.05 N(0,1), y = noisy "
                    "analytic sinogram",
        "forward_ms": fp_ms, "forward_gups": updates / (fp_ms * 1e-3) / 1e9,
        "transpose_ms": bp_ms, "transpose_gups": updates / (bp_ms * 1e-3) / 1e9,
        "ls_gradient_ms": gr_ms, "ls_gradient_gups": 2 * updates / (gr_ms * 1e-3) / 1e9,
        "updates_per_operator": updates,
        "roofline_forward": _alu_roofline("fp_tile_kernel<4>", updates, fp_ms),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): this build measures "
              "one GPU's share of the slice-sharded path, which needs no exchange between GPUs",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2505_13955_amd as xct
    from synth import configs, decode_storage, encode_storage

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    spec = configs.c3(n_slices=args.slices)
    g = spec.geom
    S = spec.n_slices
    updates = S * g.nx * g.ny * g.n_angles

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 3 x 1 GiB copies done")
        del src, dst

    t0 = time.time()
    p64 = torch.empty((S, g.n_angles, g.n_det), dtype=torch.float64, device=dev)
    for s in range(S):
        p64[s] = spec.sinogram(s, device=dev)
        torch.cuda.synchronize()
        log(f"sinogram {s + 1}/{S}")
    log(f"generated {S} sinograms in {time.time() - t0:.1f}s")

    storages = [s for s in args.storage.split(",") if s]
    fdt = torch.float32 if args.filtered == "f32" else torch.float16
    filt = torch.empty((S, g.n_angles, g.n_det), dtype=fdt, device=dev)
    image = torch.empty((S, g.ny, g.nx), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    w = math.pi / g.n_angles

    # oracle sample: one slice, every (N/sample_rows)-th row, all columns
    samp_slice = S // 2
    rows = np.linspace(0, g.ny - 1, args.sample_rows).round().astype(np.int64)
    pix = np.stack([np.zeros(rows.size * g.nx, np.int64), np.repeat(rows, g.nx),
                    np.tile(np.arange(g.nx, dtype=np.int64), rows.size)], 1)

    results = {}
    fp32_image_sample = None
    cpu = None
    ref64 = None
    for st in storages:
        sino = encode_storage(p64, st).contiguous()

        def step():
            xct.xct_filter(g, sino, filt, spec.window)
            xct.xct_backproject(g, filt, image, w, False)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
        torch.cuda.synchronize()
        t_wall = time.time()
        for k in range(args.steps):
            ev[k][0].record(stream)
            xct.xct_filter(g, sino, filt, spec.window)
            ev[k][1].record(stream)
            xct.xct_backproject(g, filt, image, w, False)
            ev[k][2].record(stream)
        torch.cuda.synchronize()
        t_wall = time.time() - t_wall
        f_ms = sum(e[0].elapsed_time(e[1]) for e in ev) / args.steps
        b_ms = sum(e[1].elapsed_time(e[2]) for e in ev) / args.steps
        step_ms = ev[0][0].elapsed_time(ev[-1][2]) / args.steps
        r = {
            "gups": updates / (step_ms * 1e-3) / 1e9,
            "ms_per_step": step_ms,
            "filter_ms": f_ms,
            "bp_ms": b_ms,
            "bp_gups": updates / (b_ms * 1e-3) / 1e9,
            "wall_ms_per_step": 1e3 * t_wall / args.steps,
        }
        log(st, json.dumps({k: round(v, 3) for k, v in r.items()}))
        got = image[samp_slice].cpu().numpy()[rows, :].ravel().astype(np.float64)
        if st == "f32":
            fp32_image_sample = got
        elif fp32_image_sample is not None:
            r["rel_l2_vs_gpu_f32"] = float(np.linalg.norm(got - fp32_image_sample)
                                            / np.linalg.norm(fp32_image_sample))
        if not args.no_oracle:
            import oracle

            stored = decode_storage(sino[samp_slice]).cpu().numpy()
            t1 = time.time()
            q = oracle.filter(stored, g.det_pitch, spec.window)
            t_filter = time.time() - t1
            t1 = time.time()
            ref = oracle.backproject_pixels(q, g, pix, oracle.fbp_weight(g))
            t_bp = time.time() - t1
            r["rel_l2_vs_oracle"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
            if st == "f32":
                samp_updates = pix.shape[0] * g.n_angles
                t_fbp = t_bp + t_filter * rows.size / g.ny
                cpu = {
                    "value": samp_updates / t_fbp / 1e9,
                    "unit": "GUPS",
                    "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
                    "kind": "oracle",
                    "sample": (f"FP64 oracle on slice {samp_slice}: filter of all {g.n_angles} rows "
                               f"({t_filter:.1f}s, prorated to the sampled rows) + back-projection of "
                               f"{rows.size} rows x {g.nx} columns x {g.n_angles} angles "
                               f"({t_bp:.1f}s)"),
                }
                ref64 = ref
            elif ref64 is not None:
                # the FP32-stored input is the unquantised line integrals to ~1e-7
                r["rel_l2_vs_oracle_f32_input"] = float(np.linalg.norm(got - ref64)
                                                        / np.linalg.norm(ref64))
            log(st, "rel L2 vs oracle", r["rel_l2_vs_oracle"])
        results[st] = r
        del sino

    extra = {}
    if not args.main_only:
        import synth

        extra["raw_pipeline"] = measure_raw_pipeline(xct, torch, synth, spec, p64, filt, stream,
                                                     args.steps, args.warmup)
    del p64, filt, image
    torch.cuda.empty_cache()
    if not args.main_only:
        # the legs of a few milliseconds per call get at least ten warm-up and
        # ten timed calls: the first calls after a pause run at a clock still
        # ramping up (the uneven batch settles from 5.5 to 4.9 ms per call)
        short_steps, short_warmup = max(args.steps, 10), max(args.warmup, 10)
        extra["uneven_batch"] = measure_uneven_batch(xct, torch, configs, encode_storage, stream,
                                                     short_steps, short_warmup)
        torch.cuda.empty_cache()
        extra["offset_scan"] = measure_offset_scan(xct, torch, configs, stream, args.steps,
                                                   args.warmup)
        torch.cuda.empty_cache()
        extra["adjoint_pair"] = measure_adjoint_pair(xct, torch, configs, stream, short_steps,
                                                     short_warmup)

    main_st = "f32" if "f32" in results else storages[0]
    m = results[main_st]
    bp_s = m["bp_ms"] * 1e-3
    achieved = FLOPS_PER_UPDATE * updates / bp_s / 1e12
    out = {
        "metric": METRIC,
        "value": m["gups"],
        "unit": "GUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if main_st == "f32" else f"{main_st}-storage/f32",
        "data": "synthetic",
        "config": {
            "workload": (f"slab of {S} slices at 8192x8192, 6144 angles over [0,pi), 8192 bins, "
                         "Hann, binder disc + 200 aggregate/void ellipses; sinogram stored as "
                         f"{main_st}, filtered rows {args.filtered}"),
            "slices": S, "nx": g.nx, "ny": g.ny, "n_angles": g.n_angles, "n_det": g.n_det,
            "window": spec.window, "updates_per_step": updates,
        },
        "rel_l2": m.get("rel_l2_vs_oracle"),
        "filter_ms": m["filter_ms"],
        "bp_ms": m["bp_ms"],
        "storage": {k: v for k, v in results.items()},
        "roofline": {
            "kernel": "bp_sym_kernel<float, 96, 2>",
            "bound": "alu",
            "achieved": achieved,
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
            "traffic": BP_TRAFFIC_BYTES if (main_st == "f32" and args.filtered == "f32"
                                            and S == 16) else None,
            "traffic_unit": "bytes per launch",
            "algorithmic_bytes": (S * g.n_angles * g.n_det * (4 if args.filtered == "f32" else 2)
                                  + 4 * S * g.nx * g.ny),
            "flops_per_update": FLOPS_PER_UPDATE,
            "updates_per_launch": updates,
            "lds_bytes_per_update": LDS_BYTES_PER_UPDATE,
            "lds_bytes_per_clk_per_cu": LDS_BYTES_PER_UPDATE * updates / bp_s / (256 * 2.4e9),
        },
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
