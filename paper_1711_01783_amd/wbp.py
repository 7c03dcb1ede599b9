"""Weighted BP: learnable FP32 scales per (edge type, iteration) on
check-to-variable messages, with gradients from hand-written adjoint kernels.

``weighted_bp(weights, code, llr, syn, ckpt_every)`` returns the posteriors
[B, N] after ``weights.shape[1]`` iterations and is differentiable with respect
to ``weights`` (a [n_edge_types, L] float32 CUDA tensor).  The forward pass
keeps the message state of every ``ckpt_every``-th iteration; the backward pass
recomputes the others segment by segment.  Both run entirely in the library's
HIP kernels; this module only marshals arguments.
"""
from __future__ import annotations

import ctypes
import math

from ._lib import check, lib


def default_checkpoint_interval(iterations: int) -> int:
    """About sqrt(L): checkpoints plus one recomputed segment cost ~2 sqrt(L) states."""
    return max(1, int(math.ceil(math.sqrt(iterations))))


def workspace_bytes(code, frames: int, iterations: int, ckpt_every: int) -> int:
    n = ctypes.c_size_t()
    check(lib.met_wbp_workspace_bytes(code.handle, int(frames), int(iterations), int(ckpt_every), ctypes.byref(n)))
    return int(n.value)


def _stream(stream):
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _aligned(ws):
    off = (-ws.data_ptr()) % 256
    return ctypes.c_void_p(ws.data_ptr() + off), ws.numel() - off


def _check_weights(code, weights):
    import torch

    if not (isinstance(weights, torch.Tensor) and weights.is_cuda and weights.dtype == torch.float32):
        raise TypeError("weights must be a float32 CUDA tensor")
    t = code.info()["n_edge_types"]
    if weights.dim() != 2 or weights.shape[0] != t or not weights.is_contiguous():
        raise ValueError("weights must be contiguous [n_edge_types=%d, iterations]" % t)


def forward(code, llr, syn, weights, ckpt_every: int = 0, workspace=None, stream=None):
    """(posterior f32 [B, N], bits u8 [B, N], converged u8 [B], workspace)."""
    import torch

    _check_weights(code, weights)
    b, iters = int(llr.shape[0]), int(weights.shape[1])
    k = ckpt_every or default_checkpoint_interval(iters)
    need = workspace_bytes(code, b, iters, k)
    if workspace is None or workspace.numel() < need + 256:
        workspace = torch.empty(need + 256, dtype=torch.uint8, device=llr.device)
    ws, wsl = _aligned(workspace)
    post = torch.empty((b, code.N), dtype=torch.float32, device=llr.device)
    bits = torch.empty((b, code.N), dtype=torch.uint8, device=llr.device)
    conv = torch.empty(b, dtype=torch.uint8, device=llr.device)
    check(lib.met_wbp_forward(code.handle, llr.data_ptr(), syn.data_ptr(), b, iters, weights.data_ptr(), k,
                              post.data_ptr(), bits.data_ptr(), conv.data_ptr(), ws, wsl, _stream(stream)))
    return post, bits, conv, workspace


def backward(code, grad_posterior, weights, ckpt_every: int, workspace, stream=None):
    """dLoss/dweights [T, L] from dLoss/dposterior [B, N] (same workspace as forward)."""
    import torch

    _check_weights(code, weights)
    b, iters = int(grad_posterior.shape[0]), int(weights.shape[1])
    k = ckpt_every or default_checkpoint_interval(iters)
    g = grad_posterior.contiguous().float()
    out = torch.empty_like(weights)
    ws, wsl = _aligned(workspace)
    check(lib.met_wbp_backward(code.handle, g.data_ptr(), b, iters, weights.data_ptr(), k, out.data_ptr(), ws, wsl,
                               _stream(stream)))
    return out


def _function():
    import torch

    class WeightedBP(torch.autograd.Function):
        @staticmethod
        def forward(ctx, weights, code, llr, syn, ckpt_every):
            w = weights.detach().contiguous()
            post, _bits, _conv, ws = forward(code, llr, syn, w, ckpt_every)
            ctx.code, ctx.ws, ctx.k = code, ws, ckpt_every
            ctx.save_for_backward(w)
            return post

        @staticmethod
        def backward(ctx, grad_post):
            (w,) = ctx.saved_tensors
            return backward(ctx.code, grad_post, w, ctx.k, ctx.ws), None, None, None, None

    return WeightedBP


_FN = None


def weighted_bp(weights, code, llr, syn, ckpt_every: int = 0):
    """Differentiable posteriors of weighted BP (see module docstring)."""
    global _FN
    if _FN is None:
        _FN = _function()
    return _FN.apply(weights, code, llr, syn, ckpt_every)
