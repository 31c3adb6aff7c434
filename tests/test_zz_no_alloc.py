"""The allocation-free dot product: xct_dot_f64_noalloc, called through the C
ABI, returns what xct_dot_f64 returns (same kernels, bit for bit) on two calls
in a row, the second with a smaller input, so leftover partial sums in the
library's scratch array cannot leak into a result."""

import ctypes

import numpy as np
import pytest
import torch

from paper_2505_13955_amd import xct as X
from tests.gpu_util import say


@pytest.mark.gpu
def test_dot_f64_noalloc_equals_workspace_form():
    lib = X.load_library()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rng = np.random.default_rng(20250513)
    for n in (3_000_017, 1_001):  # full partial grid, then a single partial
        say("xct_dot_f64_noalloc vs xct_dot_f64, n =", n)
        a_h = rng.standard_normal(n).astype(np.float32)
        b_h = rng.standard_normal(n).astype(np.float32)
        a = torch.from_numpy(a_h).cuda()
        b = torch.from_numpy(b_h).cuda()
        ref = torch.zeros(1, dtype=torch.float64, device="cuda")
        got = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        nbytes = int(lib.xct_reduce_workspace_bytes(n))
        ws = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
        assert lib.xct_dot_f64(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), n,
                               ctypes.c_void_p(ref.data_ptr()), ctypes.c_void_p(ws.data_ptr()), nbytes,
                               stream) == 0
        assert lib.xct_dot_f64_noalloc(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), n,
                                       ctypes.c_void_p(got.data_ptr()), stream) == 0
        torch.cuda.synchronize()
        r, g = float(ref.item()), float(got.item())
        assert g == r, (n, g, r)
        exact = float(np.dot(a_h.astype(np.float64), b_h.astype(np.float64)))
        assert abs(g - exact) <= 1e-12 * float(np.dot(np.abs(a_h).astype(np.float64), np.abs(b_h)))
