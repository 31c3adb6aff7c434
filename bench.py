"""Throughput of per-slice parallel-beam filtered back-projection on one MI355X.

One step is the whole hot path over one slab: the windowed ramp filter of every
sinogram row (xct_filter) followed by the back-projection of every filtered row
into its slice (xct_backproject, weight pi/N_p).  The workload is the paper's
resolution: 16 slices of 8192^2, 6144 angles over a half turn, 8192 detector
bins, Hann window, seeded binder discs holding 200 aggregate / void ellipses
(closed-form line integrals, generated on the GPU before timing).  Inputs are
resident in HBM when the timed region starts.

value = voxel x angle updates per second (16 * 8192^2 * 6144 per step) / 1e9,
for the FP32-stored sinogram, from the median of the per-step times; the FP16-
and BF16-stored runs (FP32 arithmetic) are reported beside it.  Every storage
leg carries its error against the FP64 oracle fed the decoded stored sinogram,
per slice (relative L2 and max-abs over one pixel of every 64 x 64 tile), and
its fraction of the FP32 vector and LDS rooflines.  Further legs: the
64 x 2048^2 slab through xct_fbp_batch, the slab with an odd angle count (the
back-projector without the quarter-turn symmetry), the raw-counts pipeline,
the uneven batch, the offset scan and the differentiable projector pair.

    python bench.py [--steps K] [--warmup W] [--slices S] [--no-oracle] [--main-only]
"""

from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GUPS (voxel×angle updates/s) for FBP, fp32 vs fp16-storage, at stated L2 error"
FLOPS_PER_UPDATE = 6  # coordinate FMA (2), fraction (1), interpolation FMA (2), accumulate (1)
FP32_VECTOR_PEAK_TFLOPS = 157.3
LDS_BYTES_PER_UPDATE = 8  # one (a, d) FP32 pair per interpolation
# LDS read peak: 64 banks x 4 bytes per clock per CU, 256 CUs, 2.4 GHz
LDS_PEAK_BYTES_PER_CLK_CU = 256
CUS, CLOCK_HZ = 256, 2.4e9
LDS_PEAK_TBPS = LDS_PEAK_BYTES_PER_CLK_CU * CUS * CLOCK_HZ / 1e12
HBM_PEAK_GBPS = 8000.0
# HBM bytes of one FP32 back-projection launch of the full 16-slice slab:
# rocprofv3 FETCH_SIZE x 2.0 plus WRITE_SIZE x 1.0 (the factors under which a
# plain 1 GiB device copy reads and writes 1 GiB), from the counter passes in
# profiles/bp_sym_kernel_slab16_8192.txt (None while no counter pass has been
# taken on the current kernel build).
BP_TRAFFIC_BYTES = 9.887e10


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
                    help="time only the 16 x 8192^2 slab (skip the other legs)")
    ap.add_argument("--legs", default="raw,c2,generic,batch,uneven,offset,adjoint",
                    help="comma list of the extra legs to run")
    ap.add_argument("--sample-rows", type=int, default=32,
                    help="rows of one slice the CPU baseline times the FP64 oracle on")
    return ap.parse_args()


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def _timed(torch, stream, fn, steps, warmup):
    """Median milliseconds of fn() over `steps` calls, after `warmup` untimed
    ones, from HIP events on the stream the launches go to."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    for e0, e1 in ev:
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    return statistics.median(e0.elapsed_time(e1) for e0, e1 in ev)


def _alu_roofline(kernel, updates, ms):
    achieved = FLOPS_PER_UPDATE * updates / (ms * 1e-3) / 1e12
    return {"kernel": kernel, "bound": "alu", "achieved": achieved,
            "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP32_VECTOR_PEAK_TFLOPS}


def _lds_roofline(kernel, updates, ms):
    achieved = LDS_BYTES_PER_UPDATE * updates / (ms * 1e-3) / 1e12
    return {"kernel": kernel, "bound": "lds", "achieved": achieved, "peak": LDS_PEAK_TBPS,
            "unit": "TB/s", "frac": achieved / LDS_PEAK_TBPS,
            "bytes_per_clk_per_cu": achieved * 1e12 / (CUS * CLOCK_HZ),
            "peak_bytes_per_clk_per_cu": LDS_PEAK_BYTES_PER_CLK_CU}


def tile_pixels(ny, nx, seed, full_rows=0):
    """One pixel at a seeded position inside every 64 x 64 tile (a wrong tile
    cannot hide), plus `full_rows` whole rows."""
    import numpy as np

    rng = np.random.default_rng(seed)
    ti, tj = np.meshgrid(np.arange((ny + 63) // 64), np.arange((nx + 63) // 64), indexing="ij")
    i = np.minimum(ti * 64 + rng.integers(0, 64, ti.shape), ny - 1).ravel()
    j = np.minimum(tj * 64 + rng.integers(0, 64, tj.shape), nx - 1).ravel()
    if full_rows:
        rows = rng.choice(ny, full_rows, replace=False)
        i = np.concatenate([i, np.repeat(rows, nx)])
        j = np.concatenate([j, np.tile(np.arange(nx), full_rows)])
    return np.stack([i, j], 1).astype(np.int64)


def slice_errors(torch, image_slice, stored_slice, geom, window, pixels, q=None):
    """(rel L2, max-abs / max|ref|) of one slice's sampled pixels against the
    FP64 oracle fed the decoded stored rows (q: the oracle's filtered rows if
    already computed)."""
    import numpy as np

    import oracle
    from synth import decode_storage

    if q is None:
        q = oracle.filter(decode_storage(stored_slice).cpu().numpy(), geom.det_pitch, window)
    pix3 = np.concatenate([np.zeros((len(pixels), 1), np.int64), pixels], 1)
    ref = oracle.backproject_pixels(q, geom, pix3, oracle.fbp_weight(geom))
    idx = torch.as_tensor(pixels, device=image_slice.device)
    got = image_slice[idx[:, 0], idx[:, 1]].double().cpu().numpy()
    l2 = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    mx = float(np.abs(got - ref).max() / np.abs(ref).max())
    return l2, mx, got, ref


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    return model, nproc


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
        "front_end_hbm_frac": fe_bytes / (fe_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
        "backproject_u16_ms": bp_ms, "ms": fe_ms + bp_ms,
        "gups": updates / ((fe_ms + bp_ms) * 1e-3) / 1e9,
    }


def measure_fbp_batch_c3(xct, torch, spec, p64, stream, steps, warmup):
    """The same FP32 slab through xct_fbp_batch (filter into the workspace,
    one persistent back-projection launch, the FBP weight applied by the
    library)."""
    g = spec.geom
    S = p64.shape[0]
    sino = p64.to(torch.float32).contiguous()
    img = torch.empty((S, g.ny, g.nx), dtype=torch.float32, device="cuda")
    slabs = [(g, sino, img)]
    ws = torch.empty(xct.xct_fbp_workspace_bytes(slabs), dtype=torch.uint8, device="cuda")
    ms = _timed(torch, stream, lambda: xct.xct_fbp_batch(slabs, spec.window, workspace=ws),
                steps, warmup)
    updates = S * g.nx * g.ny * g.n_angles
    log(f"c3 through xct_fbp_batch: {ms:.3f} ms")
    del sino, img, ws
    return {"workload": f"{S} x 8192^2, 6144 angles, Hann, FP32; xct_fbp_batch (one slab)",
            "ms": ms, "gups": updates / (ms * 1e-3) / 1e9}


def measure_c2(xct, torch, configs, stream, steps, warmup, with_oracle):
    """64 x 2048^2, 1800 angles, 2900 bins, Shepp-Logan, Poisson noise at 1e5
    photons, through xct_fbp_batch; error on one pixel per tile of slices 0
    and 63 against the FP64 oracle."""
    spec = configs.c2()
    g = spec.geom
    S = spec.n_slices
    p = torch.empty((S, g.n_angles, g.n_det), dtype=torch.float32, device="cuda")
    for s in range(S):
        p[s] = spec.sinogram(s, device="cuda").to(torch.float32)
    img = torch.empty((S, g.ny, g.nx), dtype=torch.float32, device="cuda")
    slabs = [(g, p, img)]
    ws = torch.empty(xct.xct_fbp_workspace_bytes(slabs), dtype=torch.uint8, device="cuda")
    ms = _timed(torch, stream, lambda: xct.xct_fbp_batch(slabs, spec.window, workspace=ws),
                steps, warmup)
    updates = spec.updates
    out = {"workload": "64 x 2048^2, 1800 angles over [0,pi), 2900 bins, Shepp-Logan, 20 drifting "
                       "ellipses, Poisson 1e5 photons; FP32; xct_fbp_batch",
           "ms": ms, "gups": updates / (ms * 1e-3) / 1e9, "updates": updates,
           "roofline": _alu_roofline("bp_sym_kernel<float, 96, 2>", updates, ms)}
    log(f"c2: {ms:.3f} ms, {out['gups']:.0f} GUPS")
    if with_oracle:
        per = {}
        for s in (0, S - 1):
            l2, mx, _, _ = slice_errors(torch, img[s], p[s], g, spec.window, tile_pixels(2048, 2048, 20 + s, 1))
            per[s] = {"rel_l2": l2, "max_abs_rel": mx}
        out["errors_vs_oracle"] = per
        log("c2 errors", per)
    del p, img, ws
    return out


def measure_generic_angles(xct, torch, configs, stream, steps, warmup, with_oracle):
    """The paper-resolution slab with 6143 angles over [0, pi): no quarter
    turn maps the angle set onto itself, so the back-projection runs without
    that symmetry.  xct_filter + xct_backproject, FP32."""
    spec = configs.c7()
    g = spec.geom
    S = spec.n_slices
    p = torch.empty((S, g.n_angles, g.n_det), dtype=torch.float32, device="cuda")
    for s in range(S):
        p[s] = spec.sinogram(s, device="cuda").to(torch.float32)
    filt = torch.empty_like(p)
    img = torch.empty((S, g.ny, g.nx), dtype=torch.float32, device="cuda")
    w = math.pi / g.n_angles
    xct.xct_filter(g, p, filt, spec.window)
    bp_ms = _timed(torch, stream, lambda: xct.xct_backproject(g, filt, img, w, False), steps, warmup)
    updates = spec.updates
    out = {"workload": f"{S} x 8192^2, 6143 angles over [0,pi) (odd count), 8192 bins, Hann, FP32; "
                       "xct_backproject",
           "bp_ms": bp_ms, "bp_gups": updates / (bp_ms * 1e-3) / 1e9, "updates": updates,
           "roofline": _alu_roofline("back-projection without quarter-turn symmetry", updates, bp_ms)}
    log(f"generic angles: back-projection {bp_ms:.3f} ms, {out['bp_gups']:.0f} GUPS")
    if with_oracle:
        l2, mx, _, _ = slice_errors(torch, img[0], p[0], g, spec.window, tile_pixels(8192, 8192, 70))
        out["errors_vs_oracle"] = {"slice": 0, "rel_l2": l2, "max_abs_rel": mx}
        log("generic angles errors", l2, mx)
    del p, filt, img
    return out


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
    updates = sum(spec.n_slices * spec.geom.nx * spec.geom.ny * spec.geom.n_angles for spec in specs)
    ms = _timed(torch, stream, lambda: xct.xct_fbp_batch(slabs, "ram_lak", workspace=ws),
                steps, warmup)
    alone = [_timed(torch, stream, lambda sl=sl: xct.xct_fbp_batch([sl], "ram_lak", workspace=ws),
                    steps, warmup) for sl in slabs]
    log(f"uneven batch: {ms:.3f} ms in one launch, {sum(alone):.3f} ms slab by slab")
    return {
        "workload": "24 x 512^2 (720 angles), 12 x 1024^2 (1440), 4 x 2048^2 (2048); bf16 storage, "
                    "Ram-Lak; xct_fbp_batch, one persistent back-projection launch",
        "ms": ms, "gups": updates / (ms * 1e-3) / 1e9,
        "slab_by_slab_ms": alone, "slab_by_slab_gups": updates / (sum(alone) * 1e-3) / 1e9,
        "updates": updates,
        "roofline": _alu_roofline("filter + bp_sym_kernel<float, 96, 2> (whole call)", updates, ms),
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
    updates = S * g.nx * g.ny * g.n_angles
    fp_ms = _timed(torch, stream, lambda: xct.xct_forward_project(g, x, px), steps, warmup)
    bp_ms = _timed(torch, stream, lambda: xct.xct_project_adjoint(g, y, ptg), steps, warmup)
    gr_ms = _timed(torch, stream, lambda: xct.ls_loss_and_grad(x, y, g), steps, warmup)
    log(f"adjoint pair: P {fp_ms:.3f} ms, P^T {bp_ms:.3f} ms, gradient {gr_ms:.3f} ms")
    return {
        "workload": "32 x 1024^2, 1440 angles, 1449 bins; x = phantom + 0.05 N(0,1), y = noisy "
                    "analytic sinogram",
        "forward_ms": fp_ms, "forward_gups": updates / (fp_ms * 1e-3) / 1e9,
        "transpose_ms": bp_ms, "transpose_gups": updates / (bp_ms * 1e-3) / 1e9,
        "ls_gradient_ms": gr_ms, "ls_gradient_gups": 2 * updates / (gr_ms * 1e-3) / 1e9,
        "updates_per_operator": updates,
        "roofline_forward": _alu_roofline("fp_quad_kernel + fp_tile_kernel<4> (whole call)", updates, fp_ms),
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
    from synth import configs, encode_storage

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    spec = configs.c3(n_slices=args.slices)
    g = spec.geom
    S = spec.n_slices
    updates = S * g.nx * g.ny * g.n_angles
    with_oracle = not args.no_oracle

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

    # CPU baseline sample: one slice, every (N/sample_rows)-th row, all columns
    samp_slice = S // 2
    rows = np.linspace(0, g.ny - 1, args.sample_rows).round().astype(np.int64)
    row_pix = np.stack([np.repeat(rows, g.nx), np.tile(np.arange(g.nx, dtype=np.int64), rows.size)], 1)

    results = {}
    fp32_image_sample = None
    cpu = None
    for st in storages:
        sino = encode_storage(p64, st).contiguous()
        for _ in range(args.warmup):
            xct.xct_filter(g, sino, filt, spec.window)
            xct.xct_backproject(g, filt, image, w, False)
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
        step_ms = [e[0].elapsed_time(e[2]) for e in ev]
        f_ms = statistics.median(e[0].elapsed_time(e[1]) for e in ev)
        b_ms = statistics.median(e[1].elapsed_time(e[2]) for e in ev)
        med = statistics.median(step_ms)
        filt_bytes = S * g.n_angles * g.n_det * (sino.element_size() + filt.element_size())
        r = {
            "gups": updates / (med * 1e-3) / 1e9,
            "ms_per_step": med,
            "ms_per_step_mean": sum(step_ms) / len(step_ms),
            "filter_ms": f_ms,
            "filter_gbps": filt_bytes / (f_ms * 1e-3) / 1e9,
            "filter_hbm_frac": filt_bytes / (f_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
            "bp_ms": b_ms,
            "bp_gups": updates / (b_ms * 1e-3) / 1e9,
            "wall_ms_per_step": 1e3 * t_wall / args.steps,
            "roofline": _alu_roofline("bp_sym_kernel<float, 96, 2>", updates, b_ms),
            "roofline_lds": _lds_roofline("bp_sym_kernel<float, 96, 2>", updates, b_ms),
        }
        log(st, json.dumps({k: round(v, 3) for k, v in r.items() if isinstance(v, float)}))
        got = image[samp_slice].cpu().numpy()[rows, :].ravel().astype(np.float64)
        if st == "f32":
            fp32_image_sample = got
        elif fp32_image_sample is not None:
            r["rel_l2_vs_gpu_f32"] = float(np.linalg.norm(got - fp32_image_sample)
                                            / np.linalg.norm(fp32_image_sample))
        if with_oracle:
            import oracle
            from synth import decode_storage

            # every slice for the FP32 sinogram, four for the reduced storage
            # types; one pixel in every 64 x 64 tile
            check = range(S) if st == "f32" else sorted({0, S // 3, (2 * S) // 3, S - 1})
            per = {}
            for s in check:
                q = None
                if st == "f32" and s == samp_slice:
                    # the CPU baseline: the FP64 oracle's filter of the whole
                    # slice and its back-projection of the sampled rows
                    stored = decode_storage(sino[s]).cpu().numpy()
                    t1 = time.time()
                    q = oracle.filter(stored, g.det_pitch, spec.window)
                    t_filter = time.time() - t1
                    pix3 = np.concatenate([np.zeros((len(row_pix), 1), np.int64), row_pix], 1)
                    t1 = time.time()
                    ref_rows = oracle.backproject_pixels(q, g, pix3, oracle.fbp_weight(g))
                    t_bp = time.time() - t1
                    samp_updates = row_pix.shape[0] * g.n_angles
                    t_fbp = t_bp + t_filter * rows.size / g.ny
                    model, nproc = cpu_info()
                    cpu = {
                        "value": samp_updates / t_fbp / 1e9,
                        "unit": "GUPS",
                        "cores": oracle.threads(),
                        "nproc": nproc,
                        "cpu_model": model,
                        "kind": "oracle",
                        "sample": (f"FP64 oracle on slice {s}: filter of all {g.n_angles} rows "
                                   f"({t_filter:.1f}s, prorated to the sampled rows) + back-projection "
                                   f"of {rows.size} rows x {g.nx} columns x {g.n_angles} angles "
                                   f"({t_bp:.1f}s)"),
                    }
                    r["rel_l2_vs_oracle_sampled_rows"] = float(
                        np.linalg.norm(got - ref_rows) / np.linalg.norm(ref_rows))
                l2, mx, _, _ = slice_errors(torch, image[s], sino[s], g, spec.window,
                                            tile_pixels(g.ny, g.nx, 100 + s), q)
                per[s] = {"rel_l2": l2, "max_abs_rel": mx}
            r["errors_vs_oracle"] = per
            r["rel_l2_vs_oracle"] = max(v["rel_l2"] for v in per.values())
            r["max_abs_rel_vs_oracle"] = max(v["max_abs_rel"] for v in per.values())
            log(st, "worst slice: rel L2", r["rel_l2_vs_oracle"], "max-abs/max", r["max_abs_rel_vs_oracle"])
        results[st] = r
        del sino

    legs = set() if args.main_only else {x for x in args.legs.split(",") if x}
    short_steps, short_warmup = max(args.steps, 10), max(args.warmup, 10)
    extra = {}
    if "raw" in legs:
        import synth

        extra["raw_pipeline"] = measure_raw_pipeline(xct, torch, synth, spec, p64, filt, stream,
                                                     args.steps, args.warmup)
    del filt, image
    torch.cuda.empty_cache()
    if "batch" in legs:
        extra["fbp_batch_c3"] = measure_fbp_batch_c3(xct, torch, spec, p64, stream, args.steps,
                                                     args.warmup)
    del p64
    torch.cuda.empty_cache()
    if "c2" in legs:
        extra["c2"] = measure_c2(xct, torch, configs, stream, args.steps, args.warmup, with_oracle)
        torch.cuda.empty_cache()
    if "generic" in legs:
        extra["generic_angles"] = measure_generic_angles(xct, torch, configs, stream, max(args.steps // 2, 1),
                                                         1, with_oracle)
        torch.cuda.empty_cache()
    if "uneven" in legs:
        # the legs of a few milliseconds per call get at least ten warm-up and
        # ten timed calls: the first calls after a pause run at a clock still
        # ramping up
        extra["uneven_batch"] = measure_uneven_batch(xct, torch, configs, encode_storage, stream,
                                                     short_steps, short_warmup)
        torch.cuda.empty_cache()
    if "offset" in legs:
        extra["offset_scan"] = measure_offset_scan(xct, torch, configs, stream, args.steps,
                                                   args.warmup)
        torch.cuda.empty_cache()
    if "adjoint" in legs:
        extra["adjoint_pair"] = measure_adjoint_pair(xct, torch, configs, stream, short_steps,
                                                     short_warmup)

    main_st = "f32" if "f32" in results else storages[0]
    m = results[main_st]
    roof = dict(m["roofline"])
    roof.update({
        "traffic": BP_TRAFFIC_BYTES if (main_st == "f32" and args.filtered == "f32" and S == 16) else None,
        "traffic_unit": "bytes per launch",
        "algorithmic_bytes": (S * g.n_angles * g.n_det * (4 if args.filtered == "f32" else 2)
                              + 4 * S * g.nx * g.ny),
        "flops_per_update": FLOPS_PER_UPDATE,
        "updates_per_launch": updates,
    })
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
        "max_abs_rel": m.get("max_abs_rel_vs_oracle"),
        "error_reference": "FP64 oracle fed the decoded stored sinogram; worst slice",
        "filter_ms": m["filter_ms"],
        "bp_ms": m["bp_ms"],
        "storage": results,
        "roofline": roof,
        "roofline_lds": m["roofline_lds"],
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
