"""ctypes binding of libxct.so.

Each ``xct_*`` function here has the name of the C entry point it calls and
only marshals arguments: torch tensors become device pointers, the geometry
becomes an ``xct_geometry`` struct, the current torch stream becomes the HIP
stream.  Every step of the computation runs in the library's HIP kernels; a
non-zero status raises ``XctError``.  There is no fallback: if ``libxct.so``
is missing, importing the library raises.

Geometry objects are duck-typed: anything with ``n_angles, n_det, nx, ny,
det_pitch, pixel_size, center`` and a float64 ``angles`` array of length
``n_angles`` (radians).
"""

from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libxct.so")

XCT_F32, XCT_F16, XCT_BF16, XCT_U16 = 0, 1, 2, 3
WINDOWS = {"ram_lak": 0, "shepp_logan": 1, "hann": 2}
DTYPES = {torch.float32: XCT_F32, torch.float16: XCT_F16, torch.bfloat16: XCT_BF16}
TORCH_DTYPES = {v: k for k, v in DTYPES.items()}


class XctError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str, hip: int = 0):
        super().__init__(f"{fn} failed: {msg} (status {status}" + (f", hipError {hip})" if hip else ")"))
        self.status = status
        self.hip_error = hip


class XctGeometry(ctypes.Structure):
    _fields_ = [
        ("n_angles", ctypes.c_int32),
        ("n_det", ctypes.c_int32),
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("det_pitch", ctypes.c_double),
        ("pixel_size", ctypes.c_double),
        ("center", ctypes.c_double),
        ("angles", ctypes.POINTER(ctypes.c_double)),
    ]


class XctSlab(ctypes.Structure):
    _fields_ = [
        ("geom", XctGeometry),
        ("n_slices", ctypes.c_int32),
        ("sino", ctypes.c_void_p),
        ("image", ctypes.c_void_p),
        ("offset_overlap", ctypes.c_double),
    ]


EXPORTS = (
    "xct_filter",
    "xct_preprocess_filter",
    "xct_offset_detector",
    "xct_filter_offset",
    "xct_backproject",
    "xct_backproject_u16",
    "xct_forward_project",
    "xct_forward_residual",
    "xct_project_adjoint",
    "xct_fbp_workspace_bytes",
    "xct_fbp_batch",
    "xct_reduce_workspace_bytes",
    "xct_dot_f64",
    "xct_dot_f64_noalloc",
    "xct_sqdist_f64",
    "xct_status_string",
    "xct_version",
    "xct_last_hip_error",
    "xct_cache_clear",
)

_lib = None


def load_library(path: str | None = None) -> ctypes.CDLL:
    """Load libxct.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2505_13955_amd.build`")
    lib = ctypes.CDLL(path)
    i32, i64, vp, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
    gp = ctypes.POINTER(XctGeometry)
    sp = ctypes.POINTER(XctSlab)
    sig = {
        "xct_filter": ([gp, i32, vp, i32, vp, i32, i32, vp], ctypes.c_int),
        "xct_offset_detector": ([gp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "xct_filter_offset": ([gp, i32, vp, i32, vp, i32, i32, ctypes.c_double, vp], ctypes.c_int),
        "xct_preprocess_filter": ([gp, i32, i32, i32, vp, i32, vp, vp, ctypes.c_float, ctypes.c_float,
                                   vp, i32, i32, vp], ctypes.c_int),
        "xct_backproject": ([gp, i32, vp, i32, vp, ctypes.c_float, i32, vp], ctypes.c_int),
        "xct_backproject_u16": ([gp, i32, vp, i32, vp, ctypes.c_float, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, vp], ctypes.c_int),
        "xct_forward_project": ([gp, i32, vp, vp, ctypes.c_float, i32, vp], ctypes.c_int),
        "xct_forward_residual": ([gp, i32, vp, vp, vp, ctypes.c_float, vp], ctypes.c_int),
        "xct_project_adjoint": ([gp, i32, vp, vp, ctypes.c_float, i32, vp], ctypes.c_int),
        "xct_fbp_workspace_bytes": ([sp, i32, i32], sz),
        "xct_fbp_batch": ([sp, i32, i32, i32, i32, vp, sz, vp], ctypes.c_int),
        "xct_reduce_workspace_bytes": ([i64], sz),
        "xct_dot_f64": ([vp, vp, i64, vp, vp, sz, vp], ctypes.c_int),
        "xct_dot_f64_noalloc": ([vp, vp, i64, vp, vp], ctypes.c_int),
        "xct_sqdist_f64": ([vp, vp, i64, vp, vp, sz, vp], ctypes.c_int),
        "xct_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "xct_version": ([], ctypes.c_int),
        "xct_last_hip_error": ([], ctypes.c_int),
        "xct_cache_clear": ([], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(fn: str, rc: int):
    if rc != 0:
        lib = load_library()
        raise XctError(fn, rc, lib.xct_status_string(rc).decode(), lib.xct_last_hip_error())


def make_geometry(geom) -> tuple[XctGeometry, np.ndarray]:
    """ctypes struct for a duck-typed geometry; also returns the angle array
    that the struct points into (keep it alive for the call)."""
    ang = np.ascontiguousarray(geom.angles, dtype=np.float64)
    if ang.shape != (int(geom.n_angles),):
        raise ValueError("geometry angles must have shape (n_angles,)")
    g = XctGeometry(int(geom.n_angles), int(geom.n_det), int(geom.nx), int(geom.ny),
                    float(geom.det_pitch), float(geom.pixel_size), float(geom.center),
                    ang.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return g, ang


def _stream(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _dev(t: torch.Tensor, name: str, dtypes=None, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device (cuda) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtypes is not None and t.dtype not in dtypes:
        raise ValueError(f"{name} has dtype {t.dtype}, expected one of {dtypes}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _slices(t: torch.Tensor, geom, image: bool) -> int:
    tail = (geom.ny, geom.nx) if image else (geom.n_angles, geom.n_det)
    if t.dim() != 3 or tuple(t.shape[1:]) != tuple(tail):
        kind = "image" if image else "sinogram"
        raise ValueError(f"{kind} must have shape (S, {tail[0]}, {tail[1]}), got {tuple(t.shape)}")
    return int(t.shape[0])


# ---------------------------------------------------------------- entry points

def xct_filter(geom, sino: torch.Tensor, filtered: torch.Tensor, window: str) -> None:
    """filtered = (1/pitch) h_W * sino along every detector row."""
    lib = load_library()
    S = _slices(sino, geom, False)
    p_in = _dev(sino, "sino", DTYPES)
    p_out = _dev(filtered, "filtered", DTYPES, sino.shape)
    g, ang = make_geometry(geom)
    rc = lib.xct_filter(ctypes.byref(g), S, p_in, DTYPES[sino.dtype], p_out, DTYPES[filtered.dtype],
                        WINDOWS[window], _stream(sino))
    _check("xct_filter", rc)


def xct_offset_detector(geom) -> tuple[int, float]:
    """(n_virtual, center_virtual): the mirrored detector an offset scan is
    filtered and back-projected on."""
    lib = load_library()
    g, ang = make_geometry(geom)
    nv = ctypes.c_int32()
    cv = ctypes.c_double()
    _check("xct_offset_detector", lib.xct_offset_detector(ctypes.byref(g), ctypes.byref(nv), ctypes.byref(cv)))
    return nv.value, cv.value


def xct_filter_offset(geom, sino: torch.Tensor, filtered: torch.Tensor, window: str,
                      overlap: float) -> None:
    """filtered [S][N_p][n_virtual] = ramp filter of the redundancy-weighted rows
    of a full-turn offset scan placed on the virtual detector."""
    lib = load_library()
    S = _slices(sino, geom, False)
    nv, _ = xct_offset_detector(geom)
    p_in = _dev(sino, "sino", DTYPES)
    p_out = _dev(filtered, "filtered", DTYPES, (S, geom.n_angles, nv))
    g, ang = make_geometry(geom)
    rc = lib.xct_filter_offset(ctypes.byref(g), S, p_in, DTYPES[sino.dtype], p_out, DTYPES[filtered.dtype],
                               WINDOWS[window], float(overlap), _stream(sino))
    _check("xct_filter_offset", rc)


def fbp_offset(sino: torch.Tensor, geom, window: str, overlap: float,
               filtered_dtype=torch.float32, workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Full-turn offset-scan FBP of sino (S, N_p, N_c) through xct_fbp_batch
    (redundancy-weighted filter on the virtual detector, back-projection
    through it; every constant is applied by the library)."""
    img = torch.empty((sino.shape[0], geom.ny, geom.nx), dtype=torch.float32, device=sino.device)
    xct_fbp_batch([(geom, sino, img, overlap)], window, filtered_dtype, workspace)
    return img


def xct_preprocess_filter(geom, proj: torch.Tensor, dark: torch.Tensor, flat: torch.Tensor,
                          row_begin: int, filtered: torch.Tensor, window: str, floor: float = 1.0,
                          blur_sigma: float = 0.0) -> None:
    """filtered[s] = ramp filter of the blurred Beer-Lambert line integrals of
    detector row row_begin + s, from the raw projection stack proj
    [N_p][N_r][N_c] (uint16 counts or float32) and the dark / flat fields
    [N_r][N_c]; filtered is [S][N_p][N_c]."""
    lib = load_library()
    if proj.dim() != 3 or proj.shape[0] != geom.n_angles or proj.shape[2] != geom.n_det:
        raise ValueError(f"proj must be (N_p, N_r, N_c) = ({geom.n_angles}, *, {geom.n_det})")
    n_rows = proj.shape[1]
    S = _slices(filtered, geom, False)
    p_in = _dev(proj, "proj", (torch.uint16, torch.float32))
    p_d = _dev(dark, "dark", (torch.float32,), (n_rows, geom.n_det))
    p_f = _dev(flat, "flat", (torch.float32,), (n_rows, geom.n_det))
    p_out = _dev(filtered, "filtered", DTYPES)
    g, ang = make_geometry(geom)
    pt = XCT_U16 if proj.dtype == torch.uint16 else XCT_F32
    rc = lib.xct_preprocess_filter(ctypes.byref(g), n_rows, int(row_begin), S, p_in, pt, p_d, p_f,
                                   float(floor), float(blur_sigma), p_out, DTYPES[filtered.dtype],
                                   WINDOWS[window], _stream(proj))
    _check("xct_preprocess_filter", rc)


def xct_backproject(geom, sino: torch.Tensor, image: torch.Tensor, scale: float,
                    accumulate: bool = False) -> None:
    """image = (accumulate ? image : 0) + scale * A^T sino."""
    lib = load_library()
    S = _slices(sino, geom, False)
    p_in = _dev(sino, "sino", DTYPES)
    p_out = _dev(image, "image", (torch.float32,), (S, geom.ny, geom.nx))
    g, ang = make_geometry(geom)
    rc = lib.xct_backproject(ctypes.byref(g), S, p_in, DTYPES[sino.dtype], p_out, float(scale),
                             1 if accumulate else 0, _stream(sino))
    _check("xct_backproject", rc)


def xct_backproject_u16(geom, sino: torch.Tensor, image: torch.Tensor, scale: float,
                        mu_water: float, hu_min: float, hu_max: float) -> None:
    """image (uint16) = CT-number codes of scale * A^T sino: HU = 1000 (mu -
    mu_water) / mu_water, [hu_min, hu_max] mapped onto [0, 65535]."""
    lib = load_library()
    S = _slices(sino, geom, False)
    p_in = _dev(sino, "sino", DTYPES)
    p_out = _dev(image, "image", (torch.uint16,), (S, geom.ny, geom.nx))
    g, ang = make_geometry(geom)
    rc = lib.xct_backproject_u16(ctypes.byref(g), S, p_in, DTYPES[sino.dtype], p_out, float(scale),
                                 float(mu_water), float(hu_min), float(hu_max), _stream(sino))
    _check("xct_backproject_u16", rc)


def xct_forward_project(geom, image: torch.Tensor, sino: torch.Tensor, alpha: float = 1.0,
                        accumulate: bool = False) -> None:
    """sino = (accumulate ? sino : 0) + alpha * P image, P = (pixel^2/pitch) A."""
    lib = load_library()
    S = _slices(image, geom, True)
    p_in = _dev(image, "image", (torch.float32,))
    p_out = _dev(sino, "sino", (torch.float32,), (S, geom.n_angles, geom.n_det))
    g, ang = make_geometry(geom)
    rc = lib.xct_forward_project(ctypes.byref(g), S, p_in, p_out, float(alpha), 1 if accumulate else 0,
                                 _stream(image))
    _check("xct_forward_project", rc)


def xct_forward_residual(geom, image: torch.Tensor, y: torch.Tensor, r: torch.Tensor,
                         alpha: float = -1.0) -> None:
    """r = y + alpha * P image (alpha = -1: the residual y - P x)."""
    lib = load_library()
    S = _slices(image, geom, True)
    p_in = _dev(image, "image", (torch.float32,))
    p_y = _dev(y, "y", (torch.float32,), (S, geom.n_angles, geom.n_det))
    p_r = _dev(r, "r", (torch.float32,), (S, geom.n_angles, geom.n_det))
    g, ang = make_geometry(geom)
    rc = lib.xct_forward_residual(ctypes.byref(g), S, p_in, p_y, p_r, float(alpha), _stream(image))
    _check("xct_forward_residual", rc)


def xct_project_adjoint(geom, sino: torch.Tensor, image: torch.Tensor, alpha: float = 1.0,
                        accumulate: bool = False) -> None:
    """image = (accumulate ? image : 0) + alpha * P^T sino (FP32 sinogram)."""
    lib = load_library()
    S = _slices(sino, geom, False)
    p_in = _dev(sino, "sino", (torch.float32,))
    p_out = _dev(image, "image", (torch.float32,), (S, geom.ny, geom.nx))
    g, ang = make_geometry(geom)
    rc = lib.xct_project_adjoint(ctypes.byref(g), S, p_in, p_out, float(alpha), 1 if accumulate else 0,
                                 _stream(sino))
    _check("xct_project_adjoint", rc)


def _slab_array(slabs):
    arr = (XctSlab * len(slabs))()
    keep = []
    for i, slab in enumerate(slabs):
        geom, sino, image = slab[:3]
        overlap = float(slab[3]) if len(slab) > 3 else 0.0
        S = _slices(sino, geom, False)
        g, ang = make_geometry(geom)
        keep.append(ang)
        arr[i].geom = g
        arr[i].n_slices = S
        arr[i].sino = _dev(sino, f"slab {i} sino", DTYPES) if sino is not None else None
        arr[i].image = (_dev(image, f"slab {i} image", (torch.float32,), (S, geom.ny, geom.nx))
                        if image is not None else None)
        arr[i].offset_overlap = overlap
    return arr, keep


def xct_fbp_workspace_bytes(slabs, filtered_dtype=torch.float32) -> int:
    """slabs: list of (geom, sino, image[, offset_overlap]) (image may be None)."""
    lib = load_library()
    arr, keep = _slab_array(slabs)
    return int(lib.xct_fbp_workspace_bytes(arr, len(slabs), DTYPES[filtered_dtype]))


def xct_fbp_batch(slabs, window: str, filtered_dtype=torch.float32,
                  workspace: torch.Tensor | None = None) -> None:
    """image = (pi/N_p) A^T ((1/pitch) h_W * sino) for every slab (geom, sino,
    image), or the full-turn offset-scan FBP for a slab (geom, sino, image,
    offset_overlap) with offset_overlap > 0.  All sinograms share one dtype.
    The workspace (uint8 device tensor) is allocated here when not given."""
    lib = load_library()
    if not slabs:
        raise ValueError("no slabs")
    dt = slabs[0][1].dtype
    if any(s[1].dtype != dt for s in slabs):
        raise ValueError("all sinograms of a batch must share one dtype")
    arr, keep = _slab_array(slabs)
    need = int(lib.xct_fbp_workspace_bytes(arr, len(slabs), DTYPES[filtered_dtype]))
    if need == 0:
        raise ValueError("xct_fbp_workspace_bytes rejected the slabs")
    dev = slabs[0][1].device
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    rc = lib.xct_fbp_batch(arr, len(slabs), DTYPES[dt], WINDOWS[window], DTYPES[filtered_dtype],
                           _dev(workspace, "workspace"), workspace.numel(), _stream(slabs[0][1]))
    _check("xct_fbp_batch", rc)


def _reduce(name: str, a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    lib = load_library()
    if a.shape != b.shape:
        raise ValueError("operands differ in shape")
    n = a.numel()
    pa = _dev(a, "a", (torch.float32,))
    pb = _dev(b, "b", (torch.float32,))
    out = torch.empty((), dtype=torch.float64, device=a.device)
    nbytes = int(lib.xct_reduce_workspace_bytes(n))
    ws = torch.empty(max(nbytes // 8, 1), dtype=torch.float64, device=a.device)
    rc = getattr(lib, name)(pa, pb, n, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                            nbytes, _stream(a))
    _check(name, rc)
    return out


def xct_dot_f64(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """sum (double)a * (double)b, as a 0-d float64 device tensor."""
    return _reduce("xct_dot_f64", a, b)


def xct_dot_f64_noalloc(a: torch.Tensor, b: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
    """xct_dot_f64 into the caller's 0-d float64 device tensor `out`, with no
    workspace (the library's per-device scratch array holds the partials)."""
    lib = load_library()
    if a.shape != b.shape:
        raise ValueError("operands differ in shape")
    pa = _dev(a, "a", (torch.float32,))
    pb = _dev(b, "b", (torch.float32,))
    po = _dev(out, "out", (torch.float64,))
    if out.numel() != 1:
        raise ValueError("out must hold one float64")
    rc = lib.xct_dot_f64_noalloc(pa, pb, a.numel(), po, _stream(a))
    _check("xct_dot_f64_noalloc", rc)
    return out


def xct_sqdist_f64(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """sum ((double)a - (double)b)^2, as a 0-d float64 device tensor."""
    return _reduce("xct_sqdist_f64", a, b)


def xct_version() -> int:
    return int(load_library().xct_version())


def xct_cache_clear() -> None:
    load_library().xct_cache_clear()


# ---------------------------------------------------------------- conveniences

def filter(sino: torch.Tensor, geom, window: str, out_dtype=torch.float32) -> torch.Tensor:
    out = torch.empty(sino.shape, dtype=out_dtype, device=sino.device)
    xct_filter(geom, sino, out, window)
    return out


def backproject(sino: torch.Tensor, geom, scale: float = 1.0) -> torch.Tensor:
    """scale * A^T sino (the plain back-projector; any storage dtype)."""
    img = torch.empty((sino.shape[0], geom.ny, geom.nx), dtype=torch.float32, device=sino.device)
    xct_backproject(geom, sino, img, scale, False)
    return img


def forward_project(image: torch.Tensor, geom) -> torch.Tensor:
    """P image for image (S, N_y, N_x)."""
    out = torch.empty((image.shape[0], geom.n_angles, geom.n_det), dtype=torch.float32,
                      device=image.device)
    xct_forward_project(geom, image, out)
    return out


def project_adjoint(sino: torch.Tensor, geom) -> torch.Tensor:
    """P^T sino for an FP32 sinogram (S, N_p, N_c)."""
    img = torch.empty((sino.shape[0], geom.ny, geom.nx), dtype=torch.float32, device=sino.device)
    xct_project_adjoint(geom, sino, img)
    return img


def fbp(sino: torch.Tensor, geom, window: str, filtered_dtype=torch.float32,
        workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Filtered back-projection of a half-turn scan (S, N_p, N_c) through
    xct_fbp_batch."""
    img = torch.empty((sino.shape[0], geom.ny, geom.nx), dtype=torch.float32, device=sino.device)
    xct_fbp_batch([(geom, sino, img)], window, filtered_dtype, workspace)
    return img
