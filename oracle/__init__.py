"""FP64 CPU oracle for per-slice parallel-beam filtered back-projection.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``, never by the library.  It shares no
code with the HIP path.

The arithmetic lives in ``xct_oracle.c`` (plain double-precision loops, built
into ``liboracle.so`` by ``oracle.build``); this module marshals numpy arrays
and adds the one step that uses a library primitive: ``filter_fft``, the same
linear convolution as ``filter_direct`` evaluated through scipy's FP64 FFT,
for detector widths where the direct O(N_c^2) sum is too slow.

Definitions (the paper describes FBP only in words, Section IV-B and Section
V-A c; the conventions below are the readings this repository takes):

* geometry: pixel centres x_j = (j - (N_x-1)/2) pix, y_i = (i - (N_y-1)/2) pix;
  detector coordinate u = (x cos th + y sin th)/pitch + center, bin n at u = n;
* filter:  q = (1/pitch) h_W * p, linear convolution along the detector, zero
  outside it; h_W the inverse DTFT of |nu| W(nu) on |nu| <= 1/2;
* back-projection: f = w A^T q with A[(k,n),(i,j)] = max(0, 1 - |u_k(x_j,y_i) - n|);
  FBP uses w = pi / N_p;
* forward projector: P = (pix^2/pitch) A;
* least squares: L(x) = ||P x - y||^2, grad L = 2 P^T (P x - y).
"""

from __future__ import annotations

import ctypes
import math
import os

import numpy as np
import scipy.fft

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

WINDOWS = {"ram_lak": 0, "shepp_logan": 1, "hann": 2}

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b

        _b.build()
    lib = ctypes.CDLL(LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    i32, i64, d = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.oracle_kernel_tap.argtypes = [ctypes.c_int, ctypes.c_long]
    lib.oracle_kernel_tap.restype = d
    lib.oracle_filter.argtypes = [dp, i64, i32, d, ctypes.c_int, dp]
    lib.oracle_filter.restype = ctypes.c_int
    geo = [i32, i32, i32, i32, d, d, d, dp, i32]
    lib.oracle_backproject.argtypes = geo + [dp, d, dp]
    lib.oracle_backproject.restype = ctypes.c_int
    lib.oracle_backproject_pixels.argtypes = geo + [dp, ctypes.POINTER(ctypes.c_int64), i64, d, dp]
    lib.oracle_backproject_pixels.restype = ctypes.c_int
    lib.oracle_forward.argtypes = geo + [dp, dp]
    lib.oracle_forward.restype = ctypes.c_int
    lib.oracle_threads.argtypes = []
    lib.oracle_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def threads() -> int:
    """OpenMP threads the oracle's loops run on."""
    return int(_load().oracle_threads())


def _f64(a) -> np.ndarray:
    if hasattr(a, "detach"):  # torch tensor
        a = a.detach().cpu().to(dtype=__import__("torch").float64).numpy()
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _geo_args(g):
    ang = _f64(g.angles)
    return ang, (g.n_angles, g.n_det, g.nx, g.ny, float(g.det_pitch), float(g.pixel_size),
                 float(g.center), _ptr(ang))


def _workers() -> int:
    """Threads for scipy's FFT: the CPUs this process may run on, capped by
    OMP_NUM_THREADS when it is set (the share of a shared host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS", "")
    if omp.isdigit() and int(omp) > 0:
        n = min(n, int(omp))
    return max(n, 1)


def kernel_taps(window: str, n: int) -> np.ndarray:
    """h_W[d] for d = -(n-1) .. n-1 (length 2n-1)."""
    lib = _load()
    w = WINDOWS[window]
    return np.array([lib.oracle_kernel_tap(w, d) for d in range(-(n - 1), n)], dtype=np.float64)


def filter_direct(p, det_pitch: float, window: str) -> np.ndarray:
    """(1/pitch) h_W * p along the last axis, direct double sum.  p: (..., N_c)."""
    p = _f64(p)
    nc = p.shape[-1]
    rows = int(np.prod(p.shape[:-1])) if p.ndim > 1 else 1
    q = np.empty_like(p)
    rc = _load().oracle_filter(_ptr(p), rows, nc, float(det_pitch), WINDOWS[window], _ptr(q))
    if rc:
        raise ValueError("oracle_filter rejected its arguments")
    return q


def filter_fft(p, det_pitch: float, window: str) -> np.ndarray:
    """The same linear convolution as ``filter_direct``, through scipy's FP64
    FFT: zero-pad each row to L >= 2 N_c - 1, place h_W circularly
    (h[d] at index d mod L), multiply spectra, invert, keep [0, N_c)."""
    p = _f64(p)
    nc = p.shape[-1]
    L = 1 << int(math.ceil(math.log2(max(2 * nc - 1, 2))))
    h = kernel_taps(window, nc)
    hc = np.zeros(L)
    d = np.arange(-(nc - 1), nc)
    hc[d % L] = h
    H = scipy.fft.rfft(hc) / det_pitch
    out = np.empty_like(p)
    flat_in = p.reshape(-1, nc)
    flat_out = out.reshape(-1, nc)
    workers = _workers()
    for b in range(0, flat_in.shape[0], 256):
        P = scipy.fft.rfft(flat_in[b:b + 256], n=L, axis=-1, workers=workers)
        P *= H
        flat_out[b:b + 256] = scipy.fft.irfft(P, n=L, axis=-1, workers=workers)[:, :nc]
    return out


def filter(p, det_pitch: float, window: str) -> np.ndarray:
    """Filter with the direct sum for short rows, the FFT route otherwise."""
    p = _f64(p)
    if p.shape[-1] <= 1024 and p.size <= 4_000_000:
        return filter_direct(p, det_pitch, window)
    return filter_fft(p, det_pitch, window)


def backproject(q, geom, weight: float = 1.0) -> np.ndarray:
    """weight * A^T q.  q: (N_p, N_c) or (S, N_p, N_c) -> (N_y, N_x) or (S, N_y, N_x)."""
    q = _f64(q)
    squeeze = q.ndim == 2
    q3 = q[None] if squeeze else q
    if q3.shape[1:] != (geom.n_angles, geom.n_det):
        raise ValueError("sinogram shape does not match the geometry")
    ang, ga = _geo_args(geom)
    out = np.empty((q3.shape[0], geom.ny, geom.nx))
    rc = _load().oracle_backproject(*ga, q3.shape[0], _ptr(q3), float(weight), _ptr(out))
    if rc:
        raise ValueError("oracle_backproject rejected its arguments")
    return out[0] if squeeze else out


def backproject_pixels(q, geom, pixels, weight: float = 1.0) -> np.ndarray:
    """weight * (A^T q) at the (slice, row, col) triples in ``pixels`` (M, 3)."""
    q = _f64(q)
    q3 = q[None] if q.ndim == 2 else q
    pix = np.ascontiguousarray(pixels, dtype=np.int64).reshape(-1, 3)
    ang, ga = _geo_args(geom)
    out = np.empty(pix.shape[0])
    rc = _load().oracle_backproject_pixels(
        *ga, q3.shape[0], _ptr(q3), pix.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        pix.shape[0], float(weight), _ptr(out))
    if rc:
        raise ValueError("oracle_backproject_pixels rejected its arguments")
    return out


def forward(x, geom) -> np.ndarray:
    """P x = (pix^2/pitch) A x.  x: (N_y, N_x) or (S, N_y, N_x)."""
    x = _f64(x)
    squeeze = x.ndim == 2
    x3 = x[None] if squeeze else x
    if x3.shape[1:] != (geom.ny, geom.nx):
        raise ValueError("image shape does not match the geometry")
    ang, ga = _geo_args(geom)
    out = np.empty((x3.shape[0], geom.n_angles, geom.n_det))
    rc = _load().oracle_forward(*ga, x3.shape[0], _ptr(x3), _ptr(out))
    if rc:
        raise ValueError("oracle_forward rejected its arguments")
    return out[0] if squeeze else out


def fbp_weight(geom) -> float:
    """Angular quadrature weight of FBP over a half turn: pi / N_p."""
    return math.pi / geom.n_angles


def fbp(p, geom, window: str) -> np.ndarray:
    """Filtered back-projection: (pi/N_p) A^T ((1/pitch) h_W * p)."""
    return backproject(filter(p, geom.det_pitch, window), geom, fbp_weight(geom))


def offset_weights(n_det: int, center: float, overlap: float) -> np.ndarray:
    """Redundancy weights w[n] of a full-turn scan whose rotation axis sits at
    bin ``center`` (offset scan, Section V-A b): a ray measured at angle th and
    bin n is measured again at th + pi and bin 2c - n, and the two weights sum
    to one.  Reading (the paper gives no weighting): with t = (n - c)/overlap,
    signed so that t > 0 on the longer side of the detector,
    w = 0 for t <= -1, sin^2(pi (1 + t) / 4) for |t| < 1, 1 for t >= 1."""
    n = np.arange(n_det, dtype=np.float64)
    side = 1.0 if (n_det - 1 - center) >= center else -1.0
    t = side * (n - center) / overlap
    return np.where(t <= -1.0, 0.0, np.where(t >= 1.0, 1.0, np.sin(0.25 * math.pi * (1.0 + t)) ** 2))


def offset_virtual_detector(n_det: int, center: float) -> tuple[int, float, int]:
    """(N_v, c_v, first): the detector of a full-turn scan mirrored about the
    axis, bins 2c - (N_c - 1) .. N_c - 1 when the longer side is to the right
    (else 0 .. 2c), renumbered from 0; `first` is the virtual bin of physical
    bin 0.  Needs 2c integral."""
    two_c = int(round(2.0 * center))
    if (n_det - 1 - center) >= center:
        lo = two_c - (n_det - 1)
        return n_det - lo, center - lo, -lo
    return two_c + 1, center, 0


def offset_rows(p, n_det: int, center: float, overlap: float) -> np.ndarray:
    """Rows of an offset scan weighted by offset_weights and placed on the
    virtual detector (zero on the bins the physical detector does not see)."""
    p = _f64(p)
    nv, _, first = offset_virtual_detector(n_det, center)
    out = np.zeros(p.shape[:-1] + (nv,))
    out[..., first:first + n_det] = p * offset_weights(n_det, center, overlap)
    return out


def fbp_offset(p, geom, window: str, overlap: float) -> np.ndarray:
    """FBP of a full-turn offset scan: weighted rows on the virtual detector,
    filtered there, back-projected over the full turn with weight 2 pi / N_p
    through the virtual detector geometry."""
    nv, cv, _ = offset_virtual_detector(geom.n_det, geom.center)
    q = filter(offset_rows(p, geom.n_det, geom.center, overlap), geom.det_pitch, window)
    return backproject(q, geom.replace(n_det=nv, center=cv), 2.0 * math.pi / geom.n_angles)


def fbp_pixels(p, geom, window: str, pixels) -> np.ndarray:
    """FBP at the listed (slice, row, col) pixels; the filter runs on every row."""
    return backproject_pixels(filter(p, geom.det_pitch, window), geom, pixels, fbp_weight(geom))


def adjoint_scale(geom) -> float:
    """P = adjoint_scale * A, so P^T = adjoint_scale * A^T."""
    return geom.pixel_size ** 2 / geom.det_pitch


def ls_loss(x, y, geom) -> float:
    """||P x - y||^2 in FP64."""
    r = forward(x, geom) - _f64(y)
    return float(np.sum(r * r))


def ls_grad(x, y, geom) -> np.ndarray:
    """2 P^T (P x - y) in FP64."""
    r = forward(x, geom) - _f64(y)
    return 2.0 * backproject(r, geom, adjoint_scale(geom))
