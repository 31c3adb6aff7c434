"""The C ABI without a GPU: the library loads, exports every entry point the
header declares, and rejects bad arguments with the documented status codes
before it makes any HIP call (so these run on a machine with no GPU)."""

import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_2505_13955_amd as pkg
from paper_2505_13955_amd import xct as X

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EINVAL, EDTYPE, EWORKSPACE, ETOOBIG = -1, -2, -3, -4
FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation
FAKE2 = ctypes.c_void_p(0x7F0000000000)  # a second such pointer, far from the first


def header_functions():
    src = open(os.path.join(ROOT, "include", "xct.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(xct_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    return pkg.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(X.EXPORTS) == names


def test_version_and_status_strings(lib):
    assert lib.xct_version() == 10100
    assert lib.xct_status_string(0) == b"ok"
    for code in (-1, -2, -3, -4, -5):
        assert lib.xct_status_string(code) not in (b"ok", b"unknown status")
    assert lib.xct_last_hip_error() == 0


def _geom(**kw):
    base = dict(n_angles=8, n_det=16, nx=8, ny=8, det_pitch=1.0, pixel_size=1.0, center=7.5,
                angles=np.linspace(0, math.pi, 8, endpoint=False))
    base.update(kw)
    ang = np.ascontiguousarray(base.pop("angles"), dtype=np.float64)
    g = X.XctGeometry(base["n_angles"], base["n_det"], base["nx"], base["ny"], base["det_pitch"],
                      base["pixel_size"], base["center"],
                      ang.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return g, ang


@pytest.mark.parametrize("kw,code", [
    (dict(n_angles=0), EINVAL), (dict(n_det=-1), EINVAL), (dict(nx=0), EINVAL),
    (dict(det_pitch=0.0), EINVAL), (dict(pixel_size=-1.0), EINVAL),
    (dict(center=float("nan")), EINVAL), (dict(det_pitch=float("inf")), EINVAL),
    (dict(n_det=70000), ETOOBIG), (dict(pixel_size=100.0), ETOOBIG),
    (dict(pixel_size=0.01), ETOOBIG), (dict(center=1e7), ETOOBIG),
])
def test_geometry_validation(lib, kw, code):
    g, ang = _geom(**kw)
    assert lib.xct_backproject(ctypes.byref(g), 1, FAKE, 0, FAKE, 1.0, 0, None) == code
    assert lib.xct_forward_project(ctypes.byref(g), 1, FAKE, FAKE, 1.0, 0, None) == code
    assert lib.xct_project_adjoint(ctypes.byref(g), 1, FAKE, FAKE, 1.0, 0, None) == code


def test_angle_validation(lib):
    ang = np.linspace(0, 1, 8)
    ang[3] = np.nan
    g, keep = _geom(angles=ang)
    assert lib.xct_backproject(ctypes.byref(g), 1, FAKE, 0, FAKE, 1.0, 0, None) == EINVAL
    g2 = X.XctGeometry(8, 16, 8, 8, 1.0, 1.0, 7.5, None)
    assert lib.xct_backproject(ctypes.byref(g2), 1, FAKE, 0, FAKE, 1.0, 0, None) == EINVAL


def test_filter_validation(lib):
    g, ang = _geom()
    assert lib.xct_filter(ctypes.byref(g), 0, FAKE, 0, FAKE, 0, 0, None) == EINVAL
    assert lib.xct_filter(ctypes.byref(g), 1, None, 0, FAKE, 0, 0, None) == EINVAL
    assert lib.xct_filter(ctypes.byref(g), 1, FAKE, 3, FAKE, 0, 0, None) == EDTYPE
    assert lib.xct_filter(ctypes.byref(g), 1, FAKE, 0, FAKE, 0, 3, None) == EDTYPE
    assert lib.xct_filter(ctypes.byref(g), 1, FAKE, 1, FAKE, 0, 0, None) == EINVAL  # in place, dtype change
    big, ang2 = _geom(n_det=8193)
    assert lib.xct_filter(ctypes.byref(big), 1, FAKE, 0, ctypes.c_void_p(0x2000), 0, 0, None) == ETOOBIG
    huge, ang3 = _geom(n_angles=1 << 20, angles=np.zeros(1 << 20), n_det=1 << 16)
    assert lib.xct_filter(ctypes.byref(huge), 1 << 30, FAKE, 0, FAKE, 0, 0, None) == ETOOBIG


def test_backproject_validation(lib):
    g, ang = _geom()
    assert lib.xct_backproject(ctypes.byref(g), 1, FAKE, 0, FAKE, float("nan"), 0, None) == EINVAL
    assert lib.xct_backproject(ctypes.byref(g), 1, FAKE, 7, FAKE, 1.0, 0, None) == EDTYPE
    assert lib.xct_backproject(None, 1, FAKE, 0, FAKE, 1.0, 0, None) == EINVAL
    assert lib.xct_forward_project(ctypes.byref(g), 70000, FAKE, FAKE, 1.0, 0, None) == ETOOBIG
    assert lib.xct_forward_project(ctypes.byref(g), 1, FAKE, FAKE, float("inf"), 0, None) == EINVAL
    assert lib.xct_forward_project(ctypes.byref(g), 1, None, FAKE, 1.0, 0, None) == EINVAL
    assert lib.xct_forward_residual(ctypes.byref(g), 1, FAKE, None, FAKE, -1.0, None) == EINVAL
    assert lib.xct_forward_residual(ctypes.byref(g), 1, None, FAKE, FAKE, -1.0, None) == EINVAL
    assert lib.xct_forward_residual(ctypes.byref(g), 1, FAKE, FAKE, FAKE, float("nan"), None) == EINVAL
    assert lib.xct_forward_residual(ctypes.byref(g), 70000, FAKE, FAKE, FAKE, -1.0, None) == ETOOBIG
    assert lib.xct_project_adjoint(ctypes.byref(g), 1, FAKE, FAKE, float("nan"), 0, None) == EINVAL
    assert lib.xct_project_adjoint(ctypes.byref(g), 1, FAKE, None, 1.0, 0, None) == EINVAL
    assert lib.xct_project_adjoint(ctypes.byref(g), 0, FAKE, FAKE, 1.0, 0, None) == EINVAL


def test_preprocess_filter_validation(lib):
    g, _ = _geom()
    f = lib.xct_preprocess_filter
    ok = dict(n_rows=4, row_begin=1, n_slices=2, proj_t=3, floor=1.0, sigma=1.0, out_t=0, window=0)

    def call(**kw):
        a = dict(ok, **kw)
        return f(ctypes.byref(g), a["n_rows"], a["row_begin"], a["n_slices"], FAKE, a["proj_t"], FAKE,
                 FAKE, a["floor"], a["sigma"], FAKE2, a["out_t"], a["window"], None)

    assert call(row_begin=3) == EINVAL              # rows 3, 4 of 4
    assert call(row_begin=-1) == EINVAL
    assert call(n_rows=0) == EINVAL
    assert call(n_slices=0) == EINVAL
    assert call(floor=0.0) == EINVAL
    assert call(floor=1e-39) == EINVAL               # below the smallest normal float
    assert call(floor=float("nan")) == EINVAL
    assert call(sigma=-0.5) == EINVAL
    assert call(sigma=float("inf")) == EINVAL
    assert call(sigma=16.125) == ETOOBIG             # blur radius int(65.0) > 64
    assert call(proj_t=1) == EDTYPE                  # FP16 counts are not accepted
    assert call(out_t=3) == EDTYPE
    assert call(window=5) == EDTYPE
    assert f(ctypes.byref(g), 4, 1, 2, None, 3, FAKE, FAKE, 1.0, 1.0, FAKE2, 0, 0, None) == EINVAL
    # the output may not overlap the projection stack
    assert f(ctypes.byref(g), 4, 1, 2, FAKE, 3, FAKE, FAKE, 1.0, 1.0, FAKE, 0, 0, None) == EINVAL


def test_offset_detector_layout(lib):
    """Host-only: the virtual detector of an offset scan."""
    for n_det, center, want in ((60, 14.0, (91, 45.0)), (60, 45.0, (91, 45.0)), (61, 40.5, (82, 40.5)),
                                (4096, 1024.0, (6143, 3071.0))):
        g, _ = _geom(n_det=n_det, center=center)
        nv, cv = ctypes.c_int32(), ctypes.c_double()
        assert lib.xct_offset_detector(ctypes.byref(g), ctypes.byref(nv), ctypes.byref(cv)) == 0
        assert (nv.value, cv.value) == want
    g, _ = _geom(n_det=60, center=14.3)   # 2c not integral
    nv, cv = ctypes.c_int32(), ctypes.c_double()
    assert lib.xct_offset_detector(ctypes.byref(g), ctypes.byref(nv), ctypes.byref(cv)) == EINVAL
    g, _ = _geom(n_det=60, center=-2.0)   # axis off the detector
    assert lib.xct_offset_detector(ctypes.byref(g), ctypes.byref(nv), ctypes.byref(cv)) == EINVAL


def test_filter_offset_validation(lib):
    g, _ = _geom(n_det=60, center=14.0)
    f = lib.xct_filter_offset
    assert f(ctypes.byref(g), 1, FAKE, 0, FAKE2, 0, 0, 0.0, None) == EINVAL      # overlap 0
    assert f(ctypes.byref(g), 1, FAKE, 0, FAKE2, 0, 0, 14.5, None) == EINVAL     # beyond the short side
    assert f(ctypes.byref(g), 1, FAKE, 0, FAKE2, 0, 0, float("nan"), None) == EINVAL
    assert f(ctypes.byref(g), 1, FAKE, 0, FAKE, 0, 0, 10.0, None) == EINVAL      # in place
    assert f(ctypes.byref(g), 1, FAKE, 5, FAKE2, 0, 0, 10.0, None) == EDTYPE
    g2, _ = _geom(n_det=60, center=14.25)
    assert f(ctypes.byref(g2), 1, FAKE, 0, FAKE2, 0, 0, 10.0, None) == EINVAL    # 2c not integral
    big, _ = _geom(n_det=8192, center=100.0)                                     # 16183 virtual bins
    assert f(ctypes.byref(big), 1, FAKE, 0, FAKE2, 0, 0, 50.0, None) == ETOOBIG


def test_backproject_u16_validation(lib):
    g, _ = _geom()
    f = lib.xct_backproject_u16
    assert f(ctypes.byref(g), 1, FAKE, 0, FAKE, 1.0, 0.0, -1000.0, 3000.0, None) == EINVAL  # mu_water
    assert f(ctypes.byref(g), 1, FAKE, 0, FAKE, 1.0, -0.2, -1000.0, 3000.0, None) == EINVAL
    assert f(ctypes.byref(g), 1, FAKE, 0, FAKE, 1.0, 0.2, 3000.0, 3000.0, None) == EINVAL  # empty range
    assert f(ctypes.byref(g), 1, FAKE, 0, FAKE, 1.0, 0.2, float("nan"), 3000.0, None) == EINVAL
    assert f(ctypes.byref(g), 1, FAKE, 0, FAKE, float("inf"), 0.2, -1000.0, 3000.0, None) == EINVAL
    assert f(ctypes.byref(g), 1, FAKE, 0, FAKE, 1.0, 1e-300, -1000.0, 3000.0, None) == EINVAL  # a overflows
    assert f(ctypes.byref(g), 1, FAKE, 7, FAKE, 1.0, 0.2, -1000.0, 3000.0, None) == EDTYPE
    assert f(ctypes.byref(g), 1, None, 0, FAKE, 1.0, 0.2, -1000.0, 3000.0, None) == EINVAL


def test_fbp_batch_validation(lib):
    g, ang = _geom()
    slabs = (X.XctSlab * 2)()
    for s in slabs:
        s.geom = g
        s.n_slices = 2
        s.sino = FAKE
        s.image = FAKE
    need = lib.xct_fbp_workspace_bytes(slabs, 2, 0)
    # counters (256 B), the slab table (two descriptors, 256-aligned), then two
    # slabs of 2*8*16 FP32 values
    assert need == 256 + 256 + 2 * 1024
    assert lib.xct_fbp_workspace_bytes(slabs, 2, 1) == 256 + 256 + 2 * 512
    assert lib.xct_fbp_workspace_bytes(slabs, 0, 0) == 0
    ws = ctypes.c_void_p(0x10000)
    assert lib.xct_fbp_batch(slabs, 2, 0, 0, 0, ws, need - 1, None) == EWORKSPACE
    assert lib.xct_fbp_batch(slabs, 2, 0, 0, 0, ctypes.c_void_p(0x10010), need, None) == EWORKSPACE
    assert lib.xct_fbp_batch(slabs, 2, 0, 0, 0, None, need, None) == EWORKSPACE
    assert lib.xct_fbp_batch(slabs, 2, 0, 9, 0, ws, need, None) == EDTYPE
    assert lib.xct_fbp_batch(slabs, 65537, 0, 0, 0, ws, need, None) == ETOOBIG  # entries not read
    assert lib.xct_fbp_workspace_bytes(slabs, 65537, 0) == 0
    slabs[1].image = None
    assert lib.xct_fbp_batch(slabs, 2, 0, 0, 0, ws, need, None) == EINVAL


def test_reduce_validation(lib):
    assert lib.xct_reduce_workspace_bytes(0) == 0
    assert lib.xct_reduce_workspace_bytes(10) == 8
    assert lib.xct_reduce_workspace_bytes(10**9) == 8 * 1024
    assert lib.xct_dot_f64(FAKE, FAKE, 0, FAKE, FAKE, 8, None) == EINVAL
    assert lib.xct_dot_f64(FAKE, FAKE, 100, FAKE, FAKE, 0, None) == EWORKSPACE
    assert lib.xct_sqdist_f64(FAKE, FAKE, 100, FAKE, ctypes.c_void_p(0x1004), 8, None) == EWORKSPACE
    assert lib.xct_dot_f64_noalloc(FAKE, FAKE, 0, FAKE, None) == EINVAL
    assert lib.xct_dot_f64_noalloc(None, FAKE, 10, FAKE, None) == EINVAL
    assert lib.xct_dot_f64_noalloc(FAKE, FAKE, 10, None, None) == EINVAL


def test_binding_rejects_host_tensors():
    import torch

    g, ang = _geom()

    class G:
        n_angles, n_det, nx, ny, det_pitch, pixel_size, center = 8, 16, 8, 8, 1.0, 1.0, 7.5
        angles = np.zeros(8)

    with pytest.raises(ValueError):
        pkg.xct_backproject(G, torch.zeros(1, 8, 16), torch.zeros(1, 8, 8), 1.0)


def test_fbp_workspace_grows_with_the_slab_table(lib):
    """More slabs than one launch's arguments hold: the descriptor table takes
    its own 256-byte-aligned region of the workspace, growing with the slab
    count (no cap below 65536 slabs)."""
    g, ang = _geom()
    n = 40
    slabs = (X.XctSlab * n)()
    for s in slabs:
        s.geom = g
        s.n_slices = 1
        s.sino = FAKE
        s.image = FAKE
    rows = 8 * 16 * 4  # one slice of filtered FP32 rows: 512 bytes, already aligned
    table = [lib.xct_fbp_workspace_bytes(slabs, k, 0) - 256 - k * rows for k in range(1, n + 1)]
    assert all(t > 0 and t % 256 == 0 for t in table)
    assert all(b >= a for a, b in zip(table, table[1:])) and table[-1] > table[0]
    assert table[-1] >= n * 64  # a descriptor holds at least its 8 pointers and sizes


def test_no_device_reports_hip_error(lib):
    """With no GPU present, a call that passes validation fails cleanly with
    XCT_EHIP at its first HIP call (hipErrorNoDevice) and launches nothing."""
    import torch

    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present: this case needs a machine without one")
    g, ang = _geom()
    assert lib.xct_filter(ctypes.byref(g), 1, FAKE, 0, FAKE2, 0, 0, None) == -5
    assert lib.xct_last_hip_error() != 0
    assert lib.xct_backproject(ctypes.byref(g), 1, FAKE, 0, FAKE2, 1.0, 0, None) == -5
    assert lib.xct_forward_project(ctypes.byref(g), 1, FAKE, FAKE2, 1.0, 0, None) == -5
    assert lib.xct_dot_f64(FAKE, FAKE2, 10, FAKE, ctypes.c_void_p(0x10000), 8, None) == -5
    assert lib.xct_dot_f64_noalloc(FAKE, FAKE2, 10, FAKE, None) == -5


def test_default_chunk_holds_a_gigabyte_of_projections():
    """The projector pair's default slice chunk keeps one chunk's FP32
    projections within 1 GiB: 128 slices of 1440 x 1449 bins, at least one
    slice however wide the sinogram."""
    import types

    from paper_2505_13955_amd.autograd import CHUNK_BYTES, default_chunk

    assert CHUNK_BYTES == 1 << 30
    assert default_chunk(types.SimpleNamespace(n_angles=1440, n_det=1449)) == 128
    assert default_chunk(types.SimpleNamespace(n_angles=6144, n_det=8192)) == 5
    assert default_chunk(types.SimpleNamespace(n_angles=1 << 20, n_det=8192)) == 1
