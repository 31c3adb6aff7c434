"""GPU parity at the full sizes of the measured workloads, on pixels and voxels
the FP64 oracle computes one by one:

* the 16 x 8192^2 slab (6144 angles, 8192 bins, Hann) in the launch
  configuration the benchmark times (xct_filter then xct_backproject), with
  the sinogram stored as FP32, FP16 and BF16;
* the 64 x 2048^2 slab (1800 angles, 2900 bins, Shepp-Logan, Poisson noise)
  through xct_fbp_batch;
* the uneven batch (24 x 512^2, 12 x 1024^2, 4 x 2048^2, BF16) in one
  persistent launch, bitwise equal to per-slab launches;
* the differentiable pair on 32 x 1024^2 (1440 angles, 1449 bins): central
  finite differences on 64 voxels, the adjoint identity in FP64, and the
  gradient against the oracle's.
"""

import math

import numpy as np
import pytest
import torch

import oracle
import synth
from synth import configs
from tests.gpu_util import rel_l2, say

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-4
TOL_REDUCED = 2e-3


@pytest.fixture(scope="module")
def xct():
    import paper_2505_13955_amd as pkg

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pkg.load_library()
    return pkg


def _oracle_pixels(stored_slice, geom, window, pixels):
    """FP64 oracle FBP of one decoded slice at (row, col) pixels."""
    q = oracle.filter(synth.decode_storage(stored_slice.cpu()).numpy(), geom.det_pitch, window)
    pix = np.concatenate([np.zeros((len(pixels), 1), np.int64), pixels], 1)
    return oracle.backproject_pixels(q, geom, pix, oracle.fbp_weight(geom))


def _pixel_sample(rng, ny, nx, n):
    return np.stack([rng.integers(0, ny, n), rng.integers(0, nx, n)], 1).astype(np.int64)


# ---------------------------------------------------------------- 16 x 8192^2
@pytest.fixture(scope="module")
def c3_lines(xct):
    spec = configs.c3()
    say("generating 16 x 6144 x 8192 line integrals")
    p = torch.empty((16, 6144, 8192), dtype=torch.float64, device="cuda")
    for s in range(16):
        p[s] = spec.sinogram(s, device="cuda")
    torch.cuda.synchronize()
    yield spec, p
    del p
    torch.cuda.empty_cache()


def c3_pixels(s):
    """Fixed pixel sample of slice s of the 8192^2 slab: one pixel at a seeded
    position inside every 64 x 64 tile (so a wrong tile cannot hide) plus two
    full rows (every thread-lattice column of the tiles they cross)."""
    rng = np.random.default_rng(1000 + s)
    ti, tj = np.meshgrid(np.arange(128), np.arange(128), indexing="ij")
    i = (ti * 64 + rng.integers(0, 64, ti.shape)).ravel()
    j = (tj * 64 + rng.integers(0, 64, tj.shape)).ravel()
    rows = rng.choice(8192, 2, replace=False)
    i = np.concatenate([i, np.repeat(rows, 8192)])
    j = np.concatenate([j, np.tile(np.arange(8192), 2)])
    return np.stack([i, j], 1).astype(np.int64)


_C3_REF = {}  # storage -> per-slice oracle values at c3_pixels(s)


def _c3_reference(sino, g, window, storage):
    if storage not in _C3_REF:
        refs = []
        for s in range(sino.shape[0]):
            refs.append(_oracle_pixels(sino[s], g, window, c3_pixels(s)))
        _C3_REF[storage] = refs
    return _C3_REF[storage]


@pytest.mark.parametrize("storage,fdt", [("f32", torch.float32), ("f16", torch.float32),
                                         ("bf16", torch.float32), ("f16", torch.float16)])
def test_c3_slab_bench_configuration(xct, c3_lines, storage, fdt):
    """The 16 x 8192^2 slab as the benchmark launches it (xct_filter, then
    xct_backproject with weight pi/N_p) against the FP64 oracle fed the
    decoded stored sinogram, on every slice: relative L2 and max-abs error
    (against the slice's largest reference value) over 32,768 pixels per
    slice, each gated at the stated tolerance."""
    spec, p64 = c3_lines
    g = spec.geom
    sino = synth.encode_storage(p64, storage).contiguous()
    filt = torch.empty(sino.shape, dtype=fdt, device="cuda")
    img = torch.empty((16, 8192, 8192), dtype=torch.float32, device="cuda")
    say("c3", storage, fdt)
    xct.xct_filter(g, sino, filt, spec.window)
    xct.xct_backproject(g, filt, img, math.pi / g.n_angles, False)
    torch.cuda.synchronize()
    assert torch.isfinite(img).all()
    del filt
    refs = _c3_reference(sino, g, spec.window, storage)
    tol = TOL_F32 if storage == "f32" and fdt == torch.float32 else TOL_REDUCED
    worst_l2, worst_max = 0.0, 0.0
    for s in range(16):
        pix = c3_pixels(s)
        got = img[s][torch.as_tensor(pix[:, 0], device="cuda"),
                     torch.as_tensor(pix[:, 1], device="cuda")].cpu().numpy().astype(np.float64)
        ref = refs[s]
        l2 = rel_l2(got, ref)
        mx = float(np.abs(got - ref).max() / np.abs(ref).max())
        say(f"  slice {s:2d}: rel L2 {l2:.3e}  max-abs/max {mx:.3e}")
        worst_l2, worst_max = max(worst_l2, l2), max(worst_max, mx)
        assert l2 < tol and mx < tol, (s, l2, mx)
    say("  worst rel L2", worst_l2, "worst max-abs/max", worst_max)
    del sino, img


def test_c3_front_end_bench_configuration(xct, c3_lines):
    """Raw counts of the 16 x 6144 x 8192 slab through the fused front end
    (Beer-Lambert, blur sigma 1, Hann filter) as the benchmark launches it;
    sampled rows against the oracle."""
    from oracle import pipeline as pl

    spec, p64 = c3_lines
    g = spec.geom
    kappa = synth.attenuation_scale(float(p64.max()))
    dark, flat = synth.detector_fields(16, 8192, 3, device="cuda")
    proj = synth.raw_counts(p64, dark, flat, kappa)           # [6144][16][8192] uint16
    out = torch.empty((16, 6144, 8192), dtype=torch.float32, device="cuda")
    say("c3 front end")
    xct.xct_preprocess_filter(g, proj, dark, flat, 0, out, spec.window, 1.0, 1.0)
    torch.cuda.synchronize()
    rng = np.random.default_rng(33)
    ks = np.sort(rng.choice(6144, 6, replace=False))
    d, f = dark.cpu().numpy(), flat.cpu().numpy()
    for s in (0, 9, 15):
        sub = proj.view(torch.int16)[ks][:, s:s + 1, :].cpu().numpy().view(np.uint16)
        sub = sub.astype(np.float64)                                      # [6][1][8192]
        p = pl.preprocess(sub, d[s:s + 1], f[s:s + 1], 0, 1, 1.0, 1.0)   # [1][6][8192]
        ref = oracle.filter(p, g.det_pitch, spec.window)[0]
        got = out[s][ks].cpu().numpy()
        err = rel_l2(got, ref)
        say("  slice", s, "rel L2", err)
        # FP32 forms I - D with up to 2^-24 (F / (I - D)) relative rounding in
        # the line integral; the ramp filter lifts that white noise against
        # the smooth blurred rows (2.6e-5 measured), under the FP32 gate
        assert err < TOL_F32
    del proj, out


def test_c3_slab_is_deterministic(xct, c3_lines):
    spec, p64 = c3_lines
    g = spec.geom
    sino = p64[:4].to(torch.float32).contiguous()
    filt = torch.empty_like(sino)
    outs = []
    for _ in range(2):
        img = torch.empty((4, 8192, 8192), dtype=torch.float32, device="cuda")
        xct.xct_filter(g, sino, filt, spec.window)
        xct.xct_backproject(g, filt, img, math.pi / g.n_angles, False)
        outs.append(img)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])


# ---------------------------------------------------------------- 64 x 2048^2
def test_c2_slab_fbp_batch(xct):
    spec = configs.c2()
    g = spec.geom
    say("c2 generate")
    p = torch.empty((64, g.n_angles, g.n_det), dtype=torch.float32, device="cuda")
    for s in range(64):
        p[s] = spec.sinogram(s, device="cuda").to(torch.float32)
    img = torch.empty((64, 2048, 2048), dtype=torch.float32, device="cuda")
    say("c2 fbp")
    xct.xct_fbp_batch([(g, p, img)], spec.window)
    torch.cuda.synchronize()
    rng = np.random.default_rng(2)
    for s in (0, 37, 63):
        pix = _pixel_sample(rng, 2048, 2048, 2000)
        ref = _oracle_pixels(p[s], g, spec.window, pix)
        err = rel_l2(img[s].cpu().numpy()[pix[:, 0], pix[:, 1]], ref)
        say("  slice", s, "rel L2", err)
        assert err < TOL_F32


# ---------------------------------------------------------------- offset scan
def test_c6_offset_slab_fbp_batch(xct):
    """8 x 4096^2 offset scan (8192 angles over a full turn, axis at bin 1024 of
    4096) through xct_fbp_batch as the benchmark launches it; sampled pixels
    against the oracle's virtual-detector FBP."""
    spec = configs.c6()
    g = spec.geom
    say("c6 generate")
    p = torch.empty((8, g.n_angles, g.n_det), dtype=torch.float32, device="cuda")
    for s in range(8):
        p[s] = spec.sinogram(s, device="cuda").to(torch.float32)
    img = torch.empty((8, 4096, 4096), dtype=torch.float32, device="cuda")
    say("c6 fbp")
    xct.xct_fbp_batch([(g, p, img, spec.offset_overlap)], spec.window)
    torch.cuda.synchronize()
    nv, cv, _ = oracle.offset_virtual_detector(g.n_det, g.center)
    virt = g.replace(n_det=nv, center=cv)
    rng = np.random.default_rng(6)
    for s in (0, 5):
        rows = oracle.offset_rows(p[s].cpu().numpy(), g.n_det, g.center, spec.offset_overlap)
        q = oracle.filter(rows, g.det_pitch, spec.window)
        pix = _pixel_sample(rng, 4096, 4096, 2000)
        pix3 = np.concatenate([np.zeros((len(pix), 1), np.int64), pix], 1)
        ref = oracle.backproject_pixels(q, virt, pix3, 2.0 * math.pi / g.n_angles)
        err = rel_l2(img[s].cpu().numpy()[pix[:, 0], pix[:, 1]], ref)
        say("  slice", s, "rel L2", err)
        assert err < TOL_F32


# ---------------------------------------------------------------- uneven batch
def test_c5_uneven_batch_one_launch(xct):
    specs = configs.c5()
    slabs, stored = [], []
    for spec in specs:
        g = spec.geom
        say("c5 generate", spec.name)
        p = torch.stack([spec.sinogram(s, device="cuda") for s in range(spec.n_slices)])
        sb = synth.encode_storage(p, "bf16").contiguous()
        stored.append(sb)
        slabs.append((g, sb, torch.empty((spec.n_slices, g.ny, g.nx), device="cuda")))
    say("c5 fbp batch")
    xct.xct_fbp_batch(slabs, "ram_lak")
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    for spec, (g, sb, img) in zip(specs, slabs):
        # the persistent multi-slab launch equals a launch per slab, bit for bit
        alone = torch.empty_like(img)
        xct.xct_fbp_batch([(g, sb, alone)], "ram_lak")
        torch.cuda.synchronize()
        assert torch.equal(alone, img), spec.name
        s = spec.n_slices - 1
        pix = _pixel_sample(rng, g.ny, g.nx, 1500)
        ref = _oracle_pixels(sb[s], g, spec.window, pix)
        err = rel_l2(img[s].cpu().numpy()[pix[:, 0], pix[:, 1]], ref)
        say("  ", spec.name, "rel L2", err)
        assert err < TOL_REDUCED


# ---------------------------------------------------------------- differentiable pair
@pytest.fixture(scope="module")
def c4_problem(xct):
    spec = configs.c4()
    g = spec.geom
    say("c4 generate")
    y = torch.stack([spec.sinogram(s, device="cuda") for s in range(32)]).to(torch.float32)
    truth = torch.stack([spec.truth(s, device="cuda", supersample=2) for s in range(32)])
    gen = torch.Generator(device="cuda").manual_seed(4)
    x = (truth + 0.05 * torch.randn(truth.shape, generator=gen, device="cuda",
                                    dtype=torch.float64)).to(torch.float32)
    return spec, g, x.contiguous(), y.contiguous()


def test_c4_autograd_finite_differences(xct, c4_problem):
    """Central differences of the loss at h = 1e-3 on 64 seeded voxels, with
    the GPU's own column a_j = P e_j and residual r in FP64 inner products
    (the quadratic makes the difference exact up to FP64 rounding, so it
    equals 2 <a_j, r> for the GPU's r).  The gradient component g_j from the
    autograd backward is a sum of about 2 N_p FP32 terms 2 (a_j)_i r_i, so
    its error is measured against that sum's absolute terms,
    sum_i |2 (a_j)_i r_i| (the condition of the sum): the gate is 1e-3 of it."""
    spec, g, x, y = c4_problem
    xr = x.clone().requires_grad_(True)
    say("c4 forward/backward")
    Px = xct.project(xr, g)
    loss = ((Px - y) ** 2).sum()
    loss.backward()
    grad = xr.grad.detach()
    r = (Px.detach() - y)
    rng = np.random.default_rng(44)
    h = 1e-3
    worst, worst_plain = 0.0, 0.0
    for _ in range(64):
        s, i, j = int(rng.integers(0, 32)), int(rng.integers(0, 1024)), int(rng.integers(0, 1024))
        e = torch.zeros((1, 1024, 1024), dtype=torch.float32, device="cuda")
        e[0, i, j] = 1.0
        a = xct.forward_project(e, g)[0].double()  # column j of P, from the GPU kernel
        r64 = r[s].double()
        fd = float((torch.sum((r64 + h * a) ** 2) - torch.sum((r64 - h * a) ** 2)) / (2 * h))
        cond = float(torch.sum(torch.abs(2.0 * a * r64)))
        gj = float(grad[s, i, j])
        worst = max(worst, abs(fd - gj) / cond)
        if abs(fd) > 0.1 * cond:
            worst_plain = max(worst_plain, abs(fd - gj) / abs(fd))
    say("  worst |fd - g| / sum|2 a r|", worst, " worst |fd - g|/|fd| (well-conditioned)", worst_plain)
    assert worst < 1e-3


def test_c4_adjoint_identity_fp64(xct, c4_problem):
    spec, g, x, y = c4_problem
    Px = xct.forward_project(x, g)
    PTy = xct.project_adjoint(y, g)
    lhs = float(xct.xct_dot_f64(Px, y))
    rhs = float(xct.xct_dot_f64(x, PTy))
    nrm = math.sqrt(float(xct.xct_dot_f64(Px, Px))) * math.sqrt(float(xct.xct_dot_f64(y, y)))
    mism = abs(lhs - rhs) / nrm
    say("  adjoint mismatch", mism)
    assert mism < 1e-5


def test_c4_streamed_loss_and_gradient_against_oracle(xct, c4_problem):
    """ls_loss_and_grad over the 32-slice stack with 16-slice chunks (two full
    chunks) and with 5-slice chunks (a partial last chunk of 2 slices, the
    residual buffer reused six times): the loss against the oracle's
    ||P x - y||^2 over all 32 slices, and the gradient against the oracle's
    on slices 0, 15, 16 and 31, on both sides of the chunk boundaries, and
    against the autograd pair; and the default chunk (the whole stack in one
    chunk here)."""
    spec, g, x, y = c4_problem
    say("c4 streamed gradient, chunks of 16 and 5 and the default")
    loss16, grad16 = xct.ls_loss_and_grad(x, y, g, chunk=16)
    loss5, grad5 = xct.ls_loss_and_grad(x, y, g, chunk=5)
    lossd, gradd = xct.ls_loss_and_grad(x, y, g)
    xr = x.clone().requires_grad_(True)
    ((xct.project(xr, g) - y) ** 2).sum().backward()
    torch.cuda.synchronize()
    x64 = x.double().cpu().numpy()
    y64 = y.double().cpu().numpy()
    say("c4 oracle loss over 32 slices")
    lref, rho = 0.0, 0.0
    resid = {}
    for s in range(32):
        Px = oracle.forward(x64[s], g)
        r = Px - y64[s]
        lref += float(np.sum(r * r))
        rho = max(rho, float(np.linalg.norm(Px) / np.linalg.norm(r)))
        if s in (0, 15, 16, 31):
            resid[s] = r
    # FP32 ray sums round at ~2^-24 |P x|; relative to the residual that is
    # rho = ||P x|| / ||r|| times larger, accumulated over ~sqrt(N) terms
    tol = max(1e-4, 2 * rho * math.sqrt(g.nx) * 2.0 ** -24)
    for name, loss in (("chunk 16", loss16), ("chunk 5", loss5), ("default chunk", lossd)):
        el = abs(float(loss) - lref) / lref
        say(f"  loss {name}: rel err {el:.3e}")
        assert el < 1e-5
    for s in (0, 15, 16, 31):
        gref = 2.0 * oracle.backproject(resid[s], g, oracle.adjoint_scale(g))
        e16 = rel_l2(grad16[s].cpu().numpy(), gref)
        e5 = rel_l2(grad5[s].cpu().numpy(), gref)
        ed = rel_l2(gradd[s].cpu().numpy(), gref)
        ea = rel_l2(xr.grad[s].cpu().numpy(), gref)
        say(f"  slice {s}: rho {rho:.1f} tol {tol:.2e}  chunk16 {e16:.3e} chunk5 {e5:.3e} default {ed:.3e} "
            f"autograd {ea:.3e}")
        assert e16 < tol and e5 < tol and ed < tol and ea < tol
    # chunking changes no slice's arithmetic beyond the forward projector's
    # variant for a 1- or 2-slice chunk: equal within the oracle gate
    assert rel_l2(grad5.cpu().numpy(), grad16.cpu().numpy()) < tol
    same = [s for s in range(32) if torch.equal(grad5[s], grad16[s])]
    say("  slices bitwise equal between chunkings:", len(same))
