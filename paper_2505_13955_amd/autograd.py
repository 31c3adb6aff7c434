"""Differentiable projector pair: the pixel-driven forward projector P and its
exact transpose, the back-projector, as a torch.autograd.Function.

    y = project(x, geom)            # P x       (xct_forward_project)
    y.backward(g)  ->  x.grad = P^T g            (xct_project_adjoint)

Slices are processed ``chunk`` at a time so that the launches of one call stay
bounded; ``ls_loss_and_grad`` goes further and streams the least-squares loss
||P x - y||^2 and its gradient 2 P^T (P x - y) slice chunk by slice chunk,
holding only one chunk's projections at a time.  Loss sums are FP64.  The
default chunk holds as many slices as keep one chunk's projections within
CHUNK_BYTES (1 GiB: 128 slices of 1440 x 1449 bins), so a stack that fits
runs as one launch per operator and larger stacks stream.
"""

from __future__ import annotations

import torch

from . import xct

CHUNK_BYTES = 1 << 30


def default_chunk(geom) -> int:
    """Slices per chunk whose FP32 projections fit CHUNK_BYTES (at least one)."""
    return max(1, CHUNK_BYTES // (4 * geom.n_angles * geom.n_det))


class XctProject(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x: torch.Tensor, geom, chunk: int | None = None):
        chunk = chunk or default_chunk(geom)
        x = x.contiguous()
        ctx.geom = geom
        ctx.chunk = chunk
        S = x.shape[0]
        y = torch.empty((S, geom.n_angles, geom.n_det), dtype=torch.float32, device=x.device)
        for s0 in range(0, S, chunk):
            xct.xct_forward_project(geom, x[s0:s0 + chunk], y[s0:s0 + chunk])
        return y

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        geom, chunk = ctx.geom, ctx.chunk
        g = g.contiguous().to(torch.float32)
        S = g.shape[0]
        gx = torch.empty((S, geom.ny, geom.nx), dtype=torch.float32, device=g.device)
        for s0 in range(0, S, chunk):
            xct.xct_project_adjoint(geom, g[s0:s0 + chunk], gx[s0:s0 + chunk])
        return gx, None, None


def project(x: torch.Tensor, geom, chunk: int | None = None) -> torch.Tensor:
    """P x for x of shape (S, N_y, N_x), differentiable in x."""
    return XctProject.apply(x, geom, chunk)


def ls_loss_and_grad(x: torch.Tensor, y: torch.Tensor, geom, chunk: int | None = None):
    """(||P x - y||^2 as a float64 device scalar, 2 P^T (P x - y) as FP32),
    computed chunk by chunk of slices, holding one chunk's residual at a time.
    The residual r = y - P x is formed inside the forward projector's store
    (one multiply-add per element, y read once); the loss is an FP64
    reduction of r and the gradient one back-projection, -2 P^T r."""
    chunk = chunk or default_chunk(geom)
    x = x.contiguous()
    y = y.contiguous()
    S = x.shape[0]
    loss = torch.zeros((), dtype=torch.float64, device=x.device)
    grad = torch.empty_like(x)
    res = torch.empty((min(chunk, S), geom.n_angles, geom.n_det), dtype=torch.float32, device=x.device)
    for s0 in range(0, S, chunk):
        s1 = min(s0 + chunk, S)
        r = res[: s1 - s0]
        xct.xct_forward_residual(geom, x[s0:s1], y[s0:s1], r, -1.0)
        loss += xct.xct_dot_f64(r, r)
        xct.xct_project_adjoint(geom, r, grad[s0:s1], -2.0)
    return loss, grad
