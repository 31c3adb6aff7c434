"""MI355X-native parallel-beam filtered back-projection.

The computation lives in ``libxct.so`` (hand-written HIP kernels for gfx950
behind the C ABI declared in ``include/xct.h``); this package is its Python
binding plus the differentiable projector pair.  PyTorch provides device
memory and streams only.
"""

from .xct import (  # noqa: F401
    EXPORTS,
    LIB_PATH,
    WINDOWS,
    XCT_BF16,
    XCT_F16,
    XCT_F32,
    XCT_U16,
    XctError,
    backproject,
    fbp,
    fbp_offset,
    filter,
    forward_project,
    project_adjoint,
    load_library,
    make_geometry,
    xct_backproject,
    xct_backproject_u16,
    xct_cache_clear,
    xct_dot_f64,
    xct_fbp_batch,
    xct_fbp_workspace_bytes,
    xct_filter,
    xct_filter_offset,
    xct_forward_project,
    xct_forward_residual,
    xct_project_adjoint,
    xct_offset_detector,
    xct_preprocess_filter,
    xct_sqdist_f64,
    xct_version,
)
from .autograd import XctProject, ls_loss_and_grad, project  # noqa: F401
