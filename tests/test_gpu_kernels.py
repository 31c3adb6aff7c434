"""GPU parity of each kernel against the FP64 oracle at sizes the oracle runs in
seconds: several 64x64 tiles plus ragged tails, odd and even sizes, every
window and storage type, both back-projection paths, the forward projector,
the FP64 reductions, and the degenerate cases (one angle, one bin, one pixel)."""

import math

import numpy as np
import pytest
import torch

import oracle
import synth
from synth import configs
from tests.gpu_util import rel_l2, say, sample_pixels, to_dev

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-4  # relative L2 vs the FP64 oracle, FP32 path


@pytest.fixture(scope="module")
def xct():
    import paper_2505_13955_amd as pkg

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pkg.load_library()
    return pkg


def _geom(**kw):
    return synth.Geometry(**kw)


# ---------------------------------------------------------------- filter
@pytest.mark.parametrize("window", ["ram_lak", "shepp_logan", "hann"])
@pytest.mark.parametrize("nc", [1, 2, 7, 64, 100, 367, 701, 1000, 1500, 1501, 2900, 4095, 5001, 8192])
def test_filter_matches_oracle(xct, window, nc):
    rng = np.random.default_rng(nc)
    rows = 5 if nc >= 2900 else 9
    p = rng.standard_normal((1, rows, nc)) * 3 + 1
    g = _geom(n_angles=rows, n_det=nc, nx=4, ny=4, det_pitch=0.75)
    say("filter", window, nc)
    q = xct.filter(to_dev(p), g, window)
    torch.cuda.synchronize()
    ref = oracle.filter(p, 0.75, window)
    err = rel_l2(q.cpu().numpy(), ref)
    assert err < 5e-6, err


@pytest.mark.parametrize("sin_t,sout_t", [(torch.float16, torch.float32), (torch.bfloat16, torch.float32),
                                          (torch.float32, torch.float16), (torch.float32, torch.bfloat16),
                                          (torch.bfloat16, torch.bfloat16)])
def test_filter_storage_types(xct, sin_t, sout_t):
    rng = np.random.default_rng(5)
    p = torch.as_tensor(rng.standard_normal((2, 7, 300)) * 10)
    stored = p.to(torch.float32).to(sin_t)
    g = _geom(n_angles=7, n_det=300, nx=4, ny=4)
    say("filter storage", sin_t, sout_t)
    q = xct.filter(stored.to("cuda").contiguous(), g, "hann", out_dtype=sout_t)
    torch.cuda.synchronize()
    ref = oracle.filter(stored.to(torch.float64).numpy(), 1.0, "hann")
    got = q.to(torch.float64).cpu().numpy()
    tol = 5e-6 if sout_t == torch.float32 else (1e-3 if sout_t == torch.float16 else 8e-3)
    assert rel_l2(got, ref) < tol
    if sout_t != torch.float32:
        # output is the FP32 result rounded to the storage type
        q32 = xct.filter(stored.to("cuda").contiguous(), g, "hann")
        assert torch.equal(q32.to(sout_t), q)


@pytest.mark.parametrize("sout_t", [torch.float16, torch.bfloat16])
def test_filter_odd_rows_reduced_output(xct, sout_t):
    """FP32 rows of odd length (the persistent kernel's sample-by-sample form)
    stored as FP16 / BF16: the FP32 result rounded to the storage type."""
    rng = np.random.default_rng(301)
    p = rng.standard_normal((3, 7, 301)) * 5
    g = _geom(n_angles=7, n_det=301, nx=4, ny=4)
    say("filter odd rows", sout_t)
    q32 = xct.filter(to_dev(p), g, "hann")
    q = xct.filter(to_dev(p), g, "hann", out_dtype=sout_t)
    torch.cuda.synchronize()
    assert rel_l2(q32.cpu().numpy(), oracle.filter(p.astype(np.float32).astype(np.float64), 1.0, "hann")) < 5e-6
    assert torch.equal(q32.to(sout_t), q)


def test_filter_in_place(xct):
    rng = np.random.default_rng(6)
    p = rng.standard_normal((1, 8, 100))
    g = _geom(n_angles=8, n_det=100, nx=4, ny=4)
    t = to_dev(p)
    xct.xct_filter(g, t, t, "shepp_logan")
    torch.cuda.synchronize()
    assert rel_l2(t.cpu().numpy(), oracle.filter(p, 1.0, "shepp_logan")) < 5e-6


# ---------------------------------------------------------------- back-projection
BP_CASES = [
    # (nx, ny, n_angles, n_det, pitch, pixel, center, angles)
    # generic path: 2c not integral
    dict(nx=130, ny=70, n_angles=45, n_det=181, det_pitch=1.0, pixel_size=1.0, center=88.3, angles="rand"),
    # mirror path: any angles and shape, 2c integral
    dict(nx=64, ny=64, n_angles=33, n_det=97, det_pitch=0.8, pixel_size=1.1, center=47.0, angles="rand"),
    dict(nx=1, ny=1, n_angles=3, n_det=5, det_pitch=1.0, pixel_size=1.0, center=2.0, angles="rand"),
    dict(nx=200, ny=3, n_angles=7, n_det=50, det_pitch=2.0, pixel_size=0.5, center=24.5, angles="rand"),
    dict(nx=97, ny=97, n_angles=1, n_det=1, det_pitch=1.0, pixel_size=1.0, center=0.0, angles="rand"),
    # symmetric path: square, even, angle set closed under +pi/2, 2c integral
    dict(nx=256, ny=256, n_angles=360, n_det=367, det_pitch=1.0, pixel_size=1.0, center=183.0, angles="uni"),
    dict(nx=100, ny=100, n_angles=60, n_det=143, det_pitch=1.0, pixel_size=1.0, center=71.0, angles="uni"),
    dict(nx=130, ny=130, n_angles=2, n_det=186, det_pitch=1.0, pixel_size=1.0, center=92.5, angles="uni"),
    dict(nx=2, ny=2, n_angles=4, n_det=3, det_pitch=1.0, pixel_size=1.0, center=1.0, angles="uni"),
    dict(nx=192, ny=192, n_angles=48, n_det=150, det_pitch=1.3, pixel_size=0.9, center=74.5, angles="uni"),
    dict(nx=128, ny=128, n_angles=36, n_det=100, det_pitch=1.0, pixel_size=1.0, center=40.0, angles="uni"),
    # pixels 1.5 bins wide: the symmetric kernel's 192-entry windows
    dict(nx=128, ny=128, n_angles=40, n_det=280, det_pitch=1.0, pixel_size=1.5, center=139.5, angles="uni"),
    # pixels 3 bins wide: generic kernel with wide windows
    dict(nx=60, ny=44, n_angles=21, n_det=260, det_pitch=0.5, pixel_size=1.5, center=129.5, angles="rand"),
    # mirror path: odd width and height (a middle row that reflects onto
    # itself), several tiles and ragged tails
    dict(nx=151, ny=77, n_angles=61, n_det=181, det_pitch=1.0, pixel_size=1.0, center=90.0, angles="rand"),
    dict(nx=64, ny=129, n_angles=50, n_det=160, det_pitch=1.0, pixel_size=1.0, center=79.5, angles="rand"),
    # mirror path, uniform angles of odd count, pixels 1.5 bins wide (192-entry windows)
    dict(nx=100, ny=100, n_angles=45, n_det=220, det_pitch=1.0, pixel_size=1.5, center=109.5, angles="uni"),
    # mirror path, axis off the detector centre (mirrored bins partly off the detector)
    dict(nx=90, ny=90, n_angles=37, n_det=140, det_pitch=1.0, pixel_size=1.0, center=80.0, angles="uni"),
]


def _case_geom(c, rng):
    c = dict(c)
    if c["angles"] == "rand":
        c["angles"] = rng.uniform(-math.pi, 2 * math.pi, c["n_angles"])
    else:
        c["angles"] = synth.uniform_angles(c["n_angles"])
    return _geom(**c)


@pytest.mark.parametrize("case", range(len(BP_CASES)))
@pytest.mark.parametrize("dtype", [torch.float32, torch.float16, torch.bfloat16])
def test_backproject_matches_oracle(xct, case, dtype):
    rng = np.random.default_rng(100 + case)
    g = _case_geom(BP_CASES[case], rng)
    S = 2
    q = rng.standard_normal((S, g.n_angles, g.n_det))
    stored = torch.as_tensor(q).to(torch.float32).to(dtype)
    say("bp", case, dtype, g.nx, g.ny, g.n_angles, g.n_det)
    img = xct.backproject(stored.to("cuda").contiguous(), g, scale=0.37)
    torch.cuda.synchronize()
    ref = oracle.backproject(stored.to(torch.float64).numpy(), g, 0.37)
    err = rel_l2(img.cpu().numpy(), ref)
    assert err < 2e-5, err


def test_backproject_accumulate_and_scale(xct):
    rng = np.random.default_rng(9)
    g = _geom(n_angles=40, n_det=90, nx=64, ny=64)
    q = rng.standard_normal((1, 40, 90))
    base = rng.standard_normal((1, 64, 64))
    img = to_dev(base)
    xct.xct_backproject(g, to_dev(q), img, -1.5, accumulate=True)
    torch.cuda.synchronize()
    ref = base - 1.5 * oracle.backproject(q.astype(np.float32).astype(np.float64), g)
    assert rel_l2(img.cpu().numpy(), ref) < 2e-5


@pytest.mark.parametrize("S", [1, 3])
def test_mirror_path_slice_counts(xct, S):
    """The mirror kernel with one slice per item (S = 1) and with a last
    two-slice group holding one slice (S = 3), odd sizes."""
    rng = np.random.default_rng(30 + S)
    g = _geom(n_angles=29, n_det=150, nx=99, ny=71, center=74.5, angles=rng.uniform(0, math.pi, 29))
    q = rng.standard_normal((S, 29, 150))
    img = xct.backproject(to_dev(q), g, scale=1.3)
    torch.cuda.synchronize()
    ref = oracle.backproject(q.astype(np.float32).astype(np.float64), g, 1.3)
    assert rel_l2(img.cpu().numpy(), ref) < 2e-5


def test_symmetric_and_mirror_paths_agree(xct):
    """The same uniform geometry through the symmetric path, and through the
    mirror path (angles nudged so the quarter-turn pairing no longer holds)."""
    rng = np.random.default_rng(10)
    g = _geom(n_angles=90, n_det=181, nx=128, ny=128)
    ang = g.angles.copy()
    ang[-1] += 1e-7
    g2 = g.replace(angles=ang)
    q = to_dev(rng.standard_normal((1, 90, 181)))
    a = xct.backproject(q, g)
    b = xct.backproject(q, g2)
    torch.cuda.synchronize()
    assert rel_l2(a.cpu().numpy(), b.cpu().numpy()) < 2e-5


def test_backproject_is_deterministic(xct):
    rng = np.random.default_rng(11)
    for g in (_geom(n_angles=128, n_det=300, nx=200, ny=200),
              _geom(n_angles=61, n_det=300, nx=150, ny=170, center=140.2)):
        q = to_dev(rng.standard_normal((2, g.n_angles, 300)))
        a = xct.backproject(q, g)
        b = xct.backproject(q, g)
        torch.cuda.synchronize()
        assert torch.equal(a, b)


# ---------------------------------------------------------------- front end
FE_CASES = [
    # (N_p, N_r, N_c, row_begin, slices, sigma, counts dtype, filtered dtype, window)
    (37, 5, 97, 1, 3, 0.0, torch.uint16, torch.float32, "ram_lak"),
    (37, 5, 97, 0, 5, 1.3, torch.float32, torch.float32, "hann"),
    (20, 3, 250, 2, 1, 4.0, torch.uint16, torch.float32, "shepp_logan"),
    (21, 4, 300, 1, 3, 2.2, torch.uint16, torch.float16, "hann"),   # 63 rows: a lone last row
    (6, 2, 8192, 0, 2, 1.0, torch.uint16, torch.float32, "hann"),   # widest detector
    (9, 2, 1, 0, 2, 0.5, torch.float32, torch.float32, "ram_lak"),  # one channel
    (11, 3, 40, 0, 3, 15.0, torch.uint16, torch.float32, "ram_lak"),  # blur wider than the row
    # uint16 counts over N_c a multiple of 4 take the persistent front end:
    # 600 rows of 8192 (more rows than one pass of the grid), 18,000 rows of
    # 256 in groups of 32 (563 groups), and a row count that leaves the last
    # group partial
    (300, 2, 8192, 0, 2, 1.0, torch.uint16, torch.float32, "hann"),
    (6000, 3, 256, 0, 3, 1.0, torch.uint16, torch.float32, "ram_lak"),
    (4001, 4, 1024, 2, 2, 2.0, torch.uint16, torch.bfloat16, "shepp_logan"),
    # persistent front end with a three-tap blur (radius 2) and without blur
    (50, 2, 512, 0, 2, 0.5, torch.uint16, torch.float32, "hann"),
    (40, 2, 1024, 1, 1, 0.0, torch.uint16, torch.float32, "ram_lak"),
]


@pytest.mark.parametrize("case", range(len(FE_CASES)))
def test_preprocess_filter_matches_oracle(xct, case):
    from oracle import pipeline as pl

    n_p, n_r, n_c, r0, S, sigma, cdt, fdt, window = FE_CASES[case]
    rng = np.random.default_rng(400 + case)
    g = _geom(n_angles=n_p, n_det=n_c, nx=8, ny=8, det_pitch=0.9)
    dark, flat = synth.detector_fields(n_r, n_c, 400 + case)
    lines = torch.as_tensor(rng.uniform(0.0, 3.0, (n_r, n_p, n_c)))
    proj = synth.raw_counts(lines, dark, flat, 1.0, dtype=cdt)
    if cdt == torch.uint16:
        # dead and saturated pixels: counts below the dark current, a flat
        # field below it, both clamped at the floor
        pn = proj.numpy()
        pn[0, r0, 0] = 20
        pn[n_p - 1, n_r - 1, n_c - 1] = 0
        flat[r0, n_c // 2] = dark[r0, n_c // 2] - 5.0
    out = torch.empty((S, n_p, n_c), dtype=fdt, device="cuda")
    say("front end", case)
    proj_dev = proj.view(torch.int16).cuda().view(torch.uint16) if cdt == torch.uint16 else proj.cuda()
    xct.xct_preprocess_filter(g, proj_dev, dark.cuda(), flat.cuda(), r0, out, window, 1.0, sigma)
    torch.cuda.synchronize()
    counts = proj.numpy().astype(np.float64)
    p = pl.preprocess(counts, dark.numpy(), flat.numpy(), r0, S, 1.0, sigma)
    ref = oracle.filter(p, g.det_pitch, window)
    got = out.to(torch.float32).cpu().numpy()
    err = rel_l2(got, ref)
    tol = 2e-5 if fdt == torch.float32 else 2e-3
    assert err < tol, err


# seeded shapes for the persistent front end: N_c a multiple of 4 from 132 to
# 8192 (every transform length from 256 to 8192), blur radii 0 to 12
FE_RANDOM = [(int(n_c), int(n_p), int(s), float(sig)) for n_c, n_p, s, sig in zip(
    np.random.default_rng(2505).integers(33, 2049, 6) * 4,
    np.random.default_rng(2506).integers(7, 90, 6),
    np.random.default_rng(2507).integers(1, 4, 6),
    np.random.default_rng(2508).choice([0.0, 0.4, 1.0, 1.7, 3.0], 6))]


@pytest.mark.parametrize("case", range(len(FE_RANDOM)))
def test_preprocess_filter_seeded_shapes(xct, case):
    from oracle import pipeline as pl

    n_c, n_p, S, sigma = FE_RANDOM[case]
    n_r, r0 = S + 1, 1
    rng = np.random.default_rng(600 + case)
    g = _geom(n_angles=n_p, n_det=n_c, nx=8, ny=8, det_pitch=1.0)
    dark, flat = synth.detector_fields(n_r, n_c, 600 + case)
    lines = torch.as_tensor(rng.uniform(0.0, 3.0, (n_r, n_p, n_c)))
    proj = synth.raw_counts(lines, dark, flat, 1.0, dtype=torch.uint16)
    out = torch.empty((S, n_p, n_c), dtype=torch.float32, device="cuda")
    say("front end seeded", case, n_c, n_p, S, sigma)
    xct.xct_preprocess_filter(g, proj.view(torch.int16).cuda().view(torch.uint16), dark.cuda(), flat.cuda(),
                              r0, out, "hann", 1.0, sigma)
    torch.cuda.synchronize()
    p = pl.preprocess(proj.numpy().astype(np.float64), dark.numpy(), flat.numpy(), r0, S, 1.0, sigma)
    ref = oracle.filter(p, g.det_pitch, "hann")
    err = rel_l2(out.cpu().numpy(), ref)
    say("  rel L2", err)
    assert err < 2e-5, err


def test_preprocess_filter_persistent_and_fallback_forms_agree(xct):
    """uint16 counts over N_c = 1024 take the persistent front end when the
    stack is 8-byte and the fields 16-byte aligned; the same data through
    fields one float off that alignment, and through a stack one count off
    it, take the one-row-per-workgroup form.  All three against the oracle,
    and the two forms within the FP32 gate of each other."""
    from oracle import pipeline as pl

    n_p, n_r, n_c, r0, S, sigma = 700, 3, 1024, 1, 2, 1.0
    rng = np.random.default_rng(77)
    g = _geom(n_angles=n_p, n_det=n_c, nx=8, ny=8, det_pitch=1.0)
    dark, flat = synth.detector_fields(n_r, n_c, 77)
    lines = torch.as_tensor(rng.uniform(0.0, 3.0, (n_r, n_p, n_c)))
    proj = synth.raw_counts(lines, dark, flat, 1.0, dtype=torch.uint16)
    counts = proj.numpy().astype(np.float64)
    p = pl.preprocess(counts, dark.numpy(), flat.numpy(), r0, S, 1.0, sigma)
    ref = oracle.filter(p, g.det_pitch, "hann")

    def run(proj_dev, dark_dev, flat_dev):
        out = torch.empty((S, n_p, n_c), dtype=torch.float32, device="cuda")
        xct.xct_preprocess_filter(g, proj_dev, dark_dev, flat_dev, r0, out, "hann", 1.0, sigma)
        torch.cuda.synchronize()
        return out.cpu().numpy()

    say("front end: persistent form and fallbacks")
    p16 = proj.view(torch.int16).cuda().view(torch.uint16)
    aligned = run(p16, dark.cuda(), flat.cuda())
    # fields one float past a 16-byte boundary
    dbuf = torch.empty(dark.numel() + 1, device="cuda")
    fbuf = torch.empty(flat.numel() + 1, device="cuda")
    d1 = dbuf[1:].view(n_r, n_c)
    f1 = fbuf[1:].view(n_r, n_c)
    d1.copy_(dark.cuda())
    f1.copy_(flat.cuda())
    shifted_fields = run(p16, d1, f1)
    # stack one count past an 8-byte boundary
    sbuf = torch.empty(proj.numel() + 1, dtype=torch.int16, device="cuda")
    s1 = sbuf[1:].view(proj.shape)
    s1.copy_(proj.view(torch.int16).cuda())
    shifted_stack = run(s1.view(torch.uint16), dark.cuda(), flat.cuda())
    for name, got in (("aligned", aligned), ("fields off", shifted_fields), ("stack off", shifted_stack)):
        err = rel_l2(got, ref)
        say(f"  {name}: rel L2 {err:.3e}")
        assert err < 2e-5, (name, err)
    assert rel_l2(shifted_fields, aligned.astype(np.float64)) < 2e-5
    assert np.array_equal(shifted_fields, shifted_stack)


def test_preprocess_filter_without_blur_equals_filter_of_line_integrals(xct):
    """sigma = 0 and FP32 line integrals given as counts of a unit flat field and
    zero dark current (I = exp(-p)): the front end reduces to xct_filter of p,
    up to the FP32 logarithm."""
    rng = np.random.default_rng(17)
    n_p, n_r, n_c = 30, 4, 120
    g = _geom(n_angles=n_p, n_det=n_c, nx=8, ny=8)
    p = rng.uniform(0.0, 2.0, (n_r, n_p, n_c))
    proj = torch.as_tensor(np.exp(-p).transpose(1, 0, 2).copy(), dtype=torch.float32).cuda()
    dark = torch.zeros((n_r, n_c), device="cuda")
    flat = torch.ones((n_r, n_c), device="cuda")
    a = torch.empty((n_r, n_p, n_c), device="cuda")
    xct.xct_preprocess_filter(g, proj, dark, flat, 0, a, "shepp_logan", 1e-30, 0.0)
    b = torch.empty_like(a)
    xct.xct_filter(g, to_dev(p), b, "shepp_logan")
    torch.cuda.synchronize()
    assert rel_l2(a.cpu().numpy(), b.cpu().numpy().astype(np.float64)) < 1e-5


# ---------------------------------------------------------------- offset scans
OFFSET_CASES = [
    # (n, full-turn angles, N_c, centre, overlap, pitch): axis left of the detector centre,
    # right of it, a set not closed under quarter turns (generic kernel), an odd slice
    (64, 120, 60, 14.0, 14.0, 1.0),
    (64, 120, 60, 45.0, 10.0, 1.0),
    (50, 90, 70, 20.5, 12.0, 1.0),
    (63, 100, 80, 25.0, 25.0, 0.9),
    (128, 256, 120, 30.0, 20.0, 1.0),
]


def _offset_geom(n, na, nd, c, pitch):
    return _geom(n_angles=na, n_det=nd, nx=n, ny=n, center=c, det_pitch=pitch,
                 angles=2.0 * math.pi * np.arange(na) / na)


@pytest.mark.parametrize("case", range(len(OFFSET_CASES)))
def test_filter_offset_matches_oracle(xct, case):
    n, na, nd, c, ov, pitch = OFFSET_CASES[case]
    g = _offset_geom(n, na, nd, c, pitch)
    rng = np.random.default_rng(500 + case)
    p = rng.standard_normal((2, na, nd))
    nv, cv = xct.xct_offset_detector(g)
    want_nv, want_cv, _ = oracle.offset_virtual_detector(nd, c)
    assert (nv, cv) == (want_nv, want_cv)
    q = torch.empty((2, na, nv), device="cuda")
    xct.xct_filter_offset(g, to_dev(p), q, "shepp_logan", ov)
    torch.cuda.synchronize()
    ref = oracle.filter(oracle.offset_rows(p.astype(np.float32).astype(np.float64), nd, c, ov),
                        pitch, "shepp_logan")
    assert rel_l2(q.cpu().numpy(), ref) < 2e-5


@pytest.mark.parametrize("case", range(len(OFFSET_CASES)))
def test_fbp_offset_matches_oracle(xct, case):
    n, na, nd, c, ov, pitch = OFFSET_CASES[case]
    g = _offset_geom(n, na, nd, c, pitch)
    rng = np.random.default_rng(600 + case)
    p = rng.standard_normal((3, na, nd))
    say("offset fbp", case)
    img = xct.fbp_offset(to_dev(p), g, "hann", ov)
    torch.cuda.synchronize()
    ref = oracle.fbp_offset(p.astype(np.float32).astype(np.float64), g, "hann", ov)
    assert rel_l2(img.cpu().numpy(), ref) < 2e-5


def test_full_turn_symmetric_and_mirror_paths_agree(xct):
    """A full-turn angle set (two half-turn sets) through the symmetric kernel,
    and through the mirror one (one angle nudged)."""
    rng = np.random.default_rng(19)
    g = _offset_geom(128, 160, 200, 99.5, 1.0)
    ang = g.angles.copy()
    ang[-1] += 1e-7
    g2 = g.replace(angles=ang)
    q = to_dev(rng.standard_normal((2, 160, 200)))
    a = xct.backproject(q, g)
    b = xct.backproject(q, g2)
    torch.cuda.synchronize()
    assert rel_l2(a.cpu().numpy(), b.cpu().numpy()) < 2e-5
    ref = oracle.backproject(q.cpu().numpy().astype(np.float64), g)
    assert rel_l2(a.cpu().numpy(), ref) < 2e-5


def test_fbp_batch_mixes_offset_and_normal_scans(xct):
    rng = np.random.default_rng(20)
    g_off = _offset_geom(96, 160, 90, 22.0, 1.0)
    g_norm = _geom(n_angles=90, n_det=140, nx=96, ny=96)
    p_off = to_dev(rng.standard_normal((3, 160, 90)))
    p_norm = to_dev(rng.standard_normal((4, 90, 140)))
    i_off = torch.empty((3, 96, 96), device="cuda")
    i_norm = torch.empty((4, 96, 96), device="cuda")
    xct.xct_fbp_batch([(g_norm, p_norm, i_norm), (g_off, p_off, i_off, 18.0)], "ram_lak")
    alone = torch.empty_like(i_off)
    xct.xct_fbp_batch([(g_off, p_off, alone, 18.0)], "ram_lak")
    torch.cuda.synchronize()
    assert torch.equal(alone, i_off)
    ref_off = oracle.fbp_offset(p_off.cpu().numpy().astype(np.float64), g_off, "ram_lak", 18.0)
    ref_norm = oracle.fbp(p_norm.cpu().numpy().astype(np.float64), g_norm, "ram_lak")
    assert rel_l2(i_off.cpu().numpy(), ref_off) < 2e-5
    assert rel_l2(i_norm.cpu().numpy(), ref_norm) < 2e-5


# ---------------------------------------------------------------- CT-number codes
def _hu_params(a, b, d=4000.0):
    """(mu_water, hu_min, hu_max) whose code map is code = a mu + b."""
    span = 65535.0 / d
    mu_w = 1000.0 * span / a
    hu_min = -1000.0 - b / span
    return mu_w, hu_min, hu_min + d


@pytest.mark.parametrize("case", [0, 5, 11])   # generic path, symmetric 96- and 192-entry windows
@pytest.mark.parametrize("clip", ["low", "high"])
def test_backproject_u16_matches_oracle_codes(xct, case, clip):
    """CT-number codes against the FP64 definition (oracle.pipeline.hu_codes of
    the FP64 back-projection): exact wherever the FP64 value A mu + B lies
    farther from a rounding boundary than the kernel's FP32 decision can
    stray from it, and never more than one code apart elsewhere."""
    from oracle import pipeline as pl

    rng = np.random.default_rng(300 + case)
    g = _case_geom(BP_CASES[case], rng)
    S = 3
    q32 = rng.standard_normal((S, g.n_angles, g.n_det)).astype(np.float32)
    ref = oracle.backproject(q32.astype(np.float64), g, 0.37)
    sigma = float(ref.std())
    # about 300 codes per standard deviation; a third of the voxels clip at
    # one end of the code range
    a = 300.0 / sigma
    b = 150.0 if clip == "low" else 65535.0 - 150.0
    mu_w, lo, hi = _hu_params(a, b)
    out = torch.empty((S, g.ny, g.nx), dtype=torch.uint16, device="cuda")
    img = torch.empty((S, g.ny, g.nx), dtype=torch.float32, device="cuda")
    say("u16", case, clip)
    xct.xct_backproject_u16(g, to_dev(q32), out, 0.37, mu_w, lo, hi)
    xct.xct_backproject(g, to_dev(q32), img, 0.37, False)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.int64)
    want = pl.hu_codes(ref, mu_w, lo, hi).astype(np.int64)
    # Bound on |kernel pre-rounding value - (A ref + B)|: the FP32 image error
    # times A (the image bound 2e-5 max|mu| is checked on the same input
    # through xct_backproject, whose accumulation the u16 store shares), plus
    # one FP32 rounding (2^-24 relative) each for a = fl(A), b = fl(B), the
    # product and the sum.
    A, B = pl.hu_affine(mu_w, lo, hi)
    img_bound = 2e-5 * float(np.abs(ref).max())
    assert float(np.abs(img.cpu().numpy() - ref).max()) <= img_bound
    u = 2.0 ** -24
    margin = A * img_bound + u * (2.0 * np.abs(ref * A) + 2.0 * abs(B) + np.abs(ref * A + B)) + 1e-9
    far = pl.hu_rounding_distance(ref, mu_w, lo, hi) > margin
    say("  codes decided exactly:", float(far.mean()))
    assert far.mean() > 0.9
    np.testing.assert_array_equal(got[far], want[far])
    assert np.abs(got - want).max() <= 1
    edge = 0 if clip == "low" else 65535
    assert np.mean(want == edge) > 0.1 and np.array_equal(got[want == edge], want[want == edge])


def test_backproject_u16_follows_the_documented_rounding(xct):
    """Self-consistency of the ABI's documented epilogue (not oracle parity,
    which the test above checks): the codes equal fl(fl(v a) + b), rounded
    half to even and clamped, applied to the FP32 image v that
    xct_backproject returns for the same input, bit for bit."""
    rng = np.random.default_rng(13)
    g = _geom(n_angles=90, n_det=181, nx=128, ny=128)
    q = to_dev(rng.standard_normal((2, 90, 181)))
    img = torch.empty((2, 128, 128), device="cuda")
    codes = torch.empty((2, 128, 128), dtype=torch.uint16, device="cuda")
    mu_w, lo, hi = 0.05, -1500.0, 2500.0
    xct.xct_backproject(g, q, img, 0.1, False)
    xct.xct_backproject_u16(g, q, codes, 0.1, mu_w, lo, hi)
    torch.cuda.synchronize()
    span = 65535.0 / (hi - lo)
    a32, b32 = np.float32(1000.0 / mu_w * span), np.float32((-1000.0 - lo) * span)
    v = img.cpu().numpy()
    t = (v * a32).astype(np.float32) + b32
    want = np.clip(np.rint(t.astype(np.float32)), 0, 65535).astype(np.uint16)
    np.testing.assert_array_equal(codes.cpu().numpy(), want)


def test_forward_accumulate_and_scale(xct):
    """sino = sino0 - 0.7 P x in one pass (the residual form)."""
    rng = np.random.default_rng(14)
    g = _geom(n_angles=30, n_det=80, nx=50, ny=50, det_pitch=1.2, center=40.3,
              angles=rng.uniform(0, math.pi, 30))
    x = rng.standard_normal((2, 50, 50))
    y0 = rng.standard_normal((2, 30, 80))
    y = to_dev(y0)
    xct.xct_forward_project(g, to_dev(x), y, -0.7, accumulate=True)
    torch.cuda.synchronize()
    ref = y0.astype(np.float32).astype(np.float64) - 0.7 * oracle.forward(
        x.astype(np.float32).astype(np.float64), g)
    assert rel_l2(y.cpu().numpy(), ref) < 2e-5


# ---------------------------------------------------------------- forward projector
FP_CASES = [
    # random angles (blocks of one or few angles), the two walk axes, both diagonals
    dict(nx=64, ny=64, n_angles=37, n_det=97, det_pitch=1.0, pixel_size=1.0, center=48.0, angles="rand"),
    dict(nx=90, ny=50, n_angles=23, n_det=120, det_pitch=0.7, pixel_size=1.2, center=61.3, angles="rand"),
    dict(nx=1, ny=1, n_angles=5, n_det=3, det_pitch=1.0, pixel_size=1.0, center=1.0, angles="rand"),
    dict(nx=33, ny=129, n_angles=16, n_det=200, det_pitch=1.5, pixel_size=1.0, center=99.5, angles="rand"),
    # uniform angles (blocks of many angles), several bin blocks, bins beyond the image
    dict(nx=48, ny=40, n_angles=90, n_det=600, det_pitch=1.0, pixel_size=1.0, center=300.0, angles="uni"),
    dict(nx=100, ny=80, n_angles=128, n_det=300, det_pitch=1.0, pixel_size=1.0, center=149.5, angles="uni"),
    dict(nx=300, ny=300, n_angles=180, n_det=425, det_pitch=1.0, pixel_size=1.0, center=212.0, angles="uni"),
    # pixels 1/16 of a bin (one walk step per stage, wide strips) and 16 bins wide
    dict(nx=40, ny=40, n_angles=24, n_det=300, det_pitch=16.0, pixel_size=1.0, center=150.0, angles="uni"),
    dict(nx=30, ny=30, n_angles=24, n_det=30, det_pitch=1.0, pixel_size=16.0, center=14.5, angles="uni"),
    # every strip misses the image
    dict(nx=70, ny=70, n_angles=64, n_det=99, det_pitch=1.0, pixel_size=1.0, center=-150.0, angles="uni"),
]


@pytest.mark.parametrize("case", range(len(FP_CASES)))
@pytest.mark.parametrize("n_slices", [2, 5, 8, 16])
def test_forward_matches_oracle(xct, case, n_slices):
    rng = np.random.default_rng(200 + case)
    c = dict(FP_CASES[case])
    if c["angles"] == "rand":
        c["angles"] = rng.uniform(0, 2 * math.pi, c["n_angles"])
        c["angles"][:4] = [0.0, math.pi / 2, math.pi / 4, math.pi][: len(c["angles"][:4])]
    else:
        c["angles"] = synth.uniform_angles(c["n_angles"])
    g = _geom(**c)
    # two slices: one per workgroup; five: four per workgroup and a partial
    # group; eight and sixteen: full groups of four
    x = rng.standard_normal((n_slices, g.ny, g.nx))
    say("fp", case, n_slices)
    y = xct.forward_project(to_dev(x), g)
    torch.cuda.synchronize()
    ref = oracle.forward(x.astype(np.float32).astype(np.float64), g)
    if np.linalg.norm(ref) == 0:
        assert np.all(y.cpu().numpy() == 0)
    else:
        assert rel_l2(y.cpu().numpy(), ref) < 2e-5


@pytest.mark.parametrize("n_slices", [2, 7])
def test_forward_residual_equals_accumulated_projection(xct, n_slices):
    """r = y - P x from the residual entry point equals y copied and then
    accumulated with alpha = -1, bit for bit (one FP32 multiply-add per
    element either way), written to another buffer and in place."""
    c = dict(FP_CASES[6])
    c["angles"] = synth.uniform_angles(c["n_angles"])
    g = _geom(**c)
    rng = np.random.default_rng(77)
    x = to_dev(rng.standard_normal((n_slices, g.ny, g.nx)))
    y = to_dev(rng.standard_normal((n_slices, g.n_angles, g.n_det)))
    say("fp residual", n_slices)
    want = y.clone()
    xct.xct_forward_project(g, x, want, -1.0, accumulate=True)
    r = torch.empty_like(y)
    xct.xct_forward_residual(g, x, y, r, -1.0)
    inplace = y.clone()
    xct.xct_forward_residual(g, x, inplace, inplace, -1.0)
    torch.cuda.synchronize()
    assert torch.equal(r, want)
    assert torch.equal(inplace, want)
    ref = y.double().cpu().numpy() - oracle.forward(x.double().cpu().numpy(), g)
    assert rel_l2(r.cpu().numpy(), ref) < 2e-5


def test_forward_project_in_chunks_of_slice_groups(xct):
    """Eleven slices of 4096^2: a group of four slices needs 512 MiB of
    four-slice copies, so the call works in two chunks (two groups, then a
    partial group of three slices).  Slices on both sides of the chunk
    boundary and the partial group are checked against the oracle."""
    n, na, nd = 4096, 8, 5795
    g = _geom(nx=n, ny=n, n_angles=na, n_det=nd, det_pitch=1.0, pixel_size=1.0, center=(nd - 1) / 2,
              angles=synth.uniform_angles(na))
    rng = np.random.default_rng(4096)
    x = rng.standard_normal((11, n, n), dtype=np.float32)
    say("fp chunks", n, na, nd, 11)
    y = xct.forward_project(to_dev(x), g)
    torch.cuda.synchronize()
    for s in (0, 7, 8, 10):
        ref = oracle.forward(x[s:s + 1].astype(np.float64), g)
        assert rel_l2(y[s:s + 1].cpu().numpy(), ref) < 2e-5, s
    # the residual form over the same two chunks: bit for bit the
    # accumulated projection (each chunk reads y at its own slices)
    xd = to_dev(x)
    yb = to_dev(rng.standard_normal((11, na, nd)))
    r = torch.empty_like(yb)
    xct.xct_forward_residual(g, xd, yb, r, -1.0)
    want = yb.clone()
    xct.xct_forward_project(g, xd, want, -1.0, accumulate=True)
    torch.cuda.synchronize()
    assert torch.equal(r, want)


# seeded geometries for the forward projector's per-block staging shapes:
# image sides 40 to 400, 30 to 400 uniform angles, detectors covering the
# image diagonal, the axis up to 20 bins off the detector centre
FP_RANDOM = [dict(nx=int(nx), ny=int(ny), n_angles=int(na), off=float(off)) for nx, ny, na, off in zip(
    np.random.default_rng(3505).integers(40, 401, 4), np.random.default_rng(3506).integers(40, 401, 4),
    np.random.default_rng(3507).integers(30, 401, 4), np.random.default_rng(3508).uniform(-20, 20, 4))]


@pytest.mark.parametrize("case", range(len(FP_RANDOM)))
def test_forward_seeded_geometries(xct, case):
    c = FP_RANDOM[case]
    n_det = int(math.ceil(math.hypot(c["nx"], c["ny"]))) + 3
    g = _geom(nx=c["nx"], ny=c["ny"], n_angles=c["n_angles"], n_det=n_det,
              center=(n_det - 1) / 2.0 + c["off"], angles=synth.uniform_angles(c["n_angles"]))
    rng = np.random.default_rng(700 + case)
    x = rng.standard_normal((8, c["ny"], c["nx"]))
    say("fp seeded", case, c, n_det)
    y = xct.forward_project(to_dev(x), g)
    torch.cuda.synchronize()
    ref = oracle.forward(x.astype(np.float32).astype(np.float64), g)
    assert rel_l2(y.cpu().numpy(), ref) < 2e-5


def test_forward_is_deterministic(xct):
    rng = np.random.default_rng(15)
    g = _geom(n_angles=200, n_det=450, nx=300, ny=260, center=230.7)
    x = to_dev(rng.standard_normal((3, 260, 300)))
    a = xct.forward_project(x, g)
    b = xct.forward_project(x, g)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_adjoint_identity_fp64(xct):
    rng = np.random.default_rng(12)
    g = _geom(n_angles=50, n_det=150, nx=100, ny=100, det_pitch=1.1, pixel_size=0.9, center=74.2,
              angles=rng.uniform(0, math.pi, 50))
    x = to_dev(rng.standard_normal((2, 100, 100)))
    y = to_dev(rng.standard_normal((2, 50, 150)))
    Px = xct.forward_project(x, g)
    PTy = xct.project_adjoint(y, g)
    lhs = float(xct.xct_dot_f64(Px, y))
    rhs = float(xct.xct_dot_f64(x, PTy))
    nrm = float(torch.linalg.norm(Px.double())) * float(torch.linalg.norm(y.double()))
    assert abs(lhs - rhs) / nrm < 1e-5


# ---------------------------------------------------------------- reductions
@pytest.mark.parametrize("n", [1, 255, 256 * 8 + 3, 1_000_003])
def test_fp64_reductions(xct, n):
    rng = np.random.default_rng(n)
    a = rng.standard_normal(n).astype(np.float32)
    b = rng.standard_normal(n).astype(np.float32)
    da, db = to_dev(a), to_dev(b)
    dot = float(xct.xct_dot_f64(da, db))
    sq = float(xct.xct_sqdist_f64(da, db))
    a64, b64 = a.astype(np.float64), b.astype(np.float64)
    assert abs(dot - np.dot(a64, b64)) <= 1e-12 * np.abs(a64 * b64).sum()
    assert abs(sq - np.sum((a64 - b64) ** 2)) <= 1e-12 * np.sum((a64 - b64) ** 2)
    assert float(xct.xct_dot_f64(da, db)) == dot  # reproducible


# ---------------------------------------------------------------- FBP
def test_fbp_c1_full_slice(xct):
    """The 256^2 / 360-angle / 367-bin / centre-183 Ram-Lak slice, whole image."""
    spec = configs.c1()
    p = spec.slab()
    say("fbp c1")
    img = xct.fbp(p.to(torch.float32).to("cuda"), spec.geom, spec.window)
    torch.cuda.synchronize()
    ref = oracle.fbp(p.to(torch.float32).to(torch.float64).numpy(), spec.geom, spec.window)
    err = rel_l2(img.cpu().numpy(), ref)
    say("fbp c1 rel L2", err)
    assert err < TOL_F32


def test_fbp_c1_golden_samples(xct):
    import json
    import os

    with open(os.path.join(os.path.dirname(__file__), "golden", "c1_oracle_fbp.json")) as f:
        gold = json.load(f)
    spec = configs.c1()
    img = xct.fbp(spec.slab().to(torch.float32).to("cuda"), spec.geom, spec.window)
    pix = np.array(gold["pixels"])
    got = img.cpu().numpy()[pix[:, 0], pix[:, 1], pix[:, 2]]
    # the stored oracle values used the FP64 sinogram; FP32 input rounding is ~1e-7
    assert rel_l2(got, gold["values"]) < TOL_F32


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("fdt", [torch.float32, torch.float16])
def test_fbp_small_slabs_storage(xct, storage, fdt):
    """Shrunk versions of the slab recipes, every storage type, FP32 or FP16
    filtered rows; the oracle sees the decoded stored sinogram."""
    for name, spec in (("c2", configs.shrink(configs.c2(), 160, 120, 3)),
                       ("c3", configs.shrink(configs.c3(), 192, 144, 2))):
        p = spec.slab()
        stored = synth.encode_storage(p, storage)
        say("fbp small", name, storage, fdt)
        img = xct.fbp(stored.to("cuda"), spec.geom, spec.window, filtered_dtype=fdt)
        torch.cuda.synchronize()
        ref = oracle.fbp(synth.decode_storage(stored).numpy(), spec.geom, spec.window)
        err = rel_l2(img.cpu().numpy(), ref)
        say("  rel L2", err)
        tol = TOL_F32 if (storage == "f32" and fdt == torch.float32) else 2e-3
        assert err < tol, (name, storage, fdt, err)


def test_fbp_batch_uneven_small(xct):
    """Three slabs of different sizes (the uneven-batch recipe at 1/8 scale) in
    one persistent launch, BF16 storage."""
    specs = configs.c5(scale=8)
    slabs, refs = [], []
    for spec in specs:
        p = synth.encode_storage(spec.slab(), "bf16")
        img = torch.empty((spec.n_slices, spec.geom.ny, spec.geom.nx), device="cuda")
        slabs.append((spec.geom, p.to("cuda"), img))
        refs.append(oracle.fbp(synth.decode_storage(p).numpy(), spec.geom, spec.window))
    say("fbp batch small")
    xct.xct_fbp_batch(slabs, "ram_lak")
    torch.cuda.synchronize()
    for (g, _, img), ref in zip(slabs, refs):
        err = rel_l2(img.cpu().numpy(), ref)
        assert err < 2e-3, err


def test_fbp_batch_mixed_paths(xct):
    """One slab takes the symmetric kernel, one the generic kernel (odd size),
    one a non-uniform angle set; all in a single call."""
    rng = np.random.default_rng(13)
    geoms = [_geom(n_angles=64, n_det=150, nx=100, ny=100),
             _geom(n_angles=50, n_det=120, nx=81, ny=81),
             _geom(n_angles=31, n_det=140, nx=90, ny=70, center=70.3,
                   angles=np.sort(rng.uniform(0, math.pi, 31)))]
    slabs, refs = [], []
    for g in geoms:
        p = rng.standard_normal((2, g.n_angles, g.n_det))
        slabs.append((g, to_dev(p), torch.empty((2, g.ny, g.nx), device="cuda")))
        refs.append(oracle.fbp(p.astype(np.float32).astype(np.float64), g, "shepp_logan"))
    xct.xct_fbp_batch(slabs, "shepp_logan")
    torch.cuda.synchronize()
    for (g, _, img), ref in zip(slabs, refs):
        assert rel_l2(img.cpu().numpy(), ref) < TOL_F32


def _many_slab_geometry(i, rng):
    """Slab i of a 40-slab batch: symmetric half turns, generic (odd,
    rectangular, random angles, off-grid centre) and full-turn offset scans."""
    kind = i % 4
    if kind == 0:      # symmetric kernel: even square, uniform half turn, 2c integral
        n = 2 * int(rng.integers(10, 48))
        na = 2 * int(rng.integers(6, 30))
        nd = int(math.ceil(math.sqrt(2) * n)) + 3
        return _geom(n_angles=na, n_det=nd, nx=n, ny=n), 0.0
    if kind == 1:      # generic kernel: rectangular, random angles
        nx, ny = int(rng.integers(17, 90)), int(rng.integers(9, 70))
        na = int(rng.integers(5, 40))
        nd = int(math.ceil(math.hypot(nx, ny))) + 4
        return _geom(n_angles=na, n_det=nd, nx=nx, ny=ny, center=(nd - 1) / 2 + 0.37,
                     angles=np.sort(rng.uniform(0, math.pi, na))), 0.0
    if kind == 2:      # offset scan: full turn, axis off the detector centre
        n = 2 * int(rng.integers(12, 40))
        na = 4 * int(rng.integers(8, 20))
        nd = n + 8
        c = float(int(rng.integers(6, nd // 3)))
        return _offset_geom(n, na, nd, c, 1.0), float(min(c, nd - 1 - c))
    n = int(rng.integers(20, 80)) | 1  # odd square: generic kernel
    na = int(rng.integers(10, 50))
    nd = int(math.ceil(math.sqrt(2) * n)) + 3
    return _geom(n_angles=na, n_det=nd, nx=n, ny=n), 0.0


@pytest.mark.parametrize("slices", [1, 2])
def test_fbp_batch_many_slabs(xct, slices):
    """A batch of 40 slabs, more than one launch's arguments carry (the slab
    descriptors are read from the table in the workspace): every image equals
    its own single-slab call bit for bit, and the FP64 oracle within the FP32
    gate."""
    rng = np.random.default_rng(77 + slices)
    slabs, refs, geo = [], [], []
    for i in range(40):
        g, overlap = _many_slab_geometry(i, rng)
        S = slices + (i % 3 == 0)   # some slabs carry one more slice
        p = rng.standard_normal((S, g.n_angles, g.n_det))
        img = torch.empty((S, g.ny, g.nx), device="cuda")
        slabs.append((g, to_dev(p), img, overlap) if overlap else (g, to_dev(p), img))
        p32 = p.astype(np.float32).astype(np.float64)
        refs.append(oracle.fbp_offset(p32, g, "hann", overlap) if overlap else oracle.fbp(p32, g, "hann"))
    say("fbp batch 40 slabs", slices)
    xct.xct_fbp_batch(slabs, "hann")
    torch.cuda.synchronize()
    for i, (sl, ref) in enumerate(zip(slabs, refs)):
        alone = torch.empty_like(sl[2])
        xct.xct_fbp_batch([(sl[0], sl[1], alone) + tuple(sl[3:])], "hann")
        torch.cuda.synchronize()
        assert torch.equal(alone, sl[2]), i
        err = rel_l2(sl[2].cpu().numpy(), ref)
        assert err < 2e-5, (i, err)
