"""Oracle: weighted BP (learnable scales on check-to-variable messages), FP64.

TEST INFRASTRUCTURE ONLY (see the package header).

Weighted BP is the flooding decoder of `oracle.bp` (Methods, Steps 2-4, eq.
(1)-(4)) with one change: the check-to-variable message of every edge of type t
produced in iteration l is multiplied by a scale w[t, l] after the syndrome
sign and before the variable update,

    c2v_e^l = w[t(e), l] * (1 - 2 s_j) * 2 artanh( prod_{e' != e} tanh(x_e'/2) ).

It runs a fixed number L of iterations and returns the posteriors after the
last one (eq. (5)).  The training loss is the mean binary cross-entropy of the
posteriors against the sent bits, with p(bit = 1) = sigmoid(-P):

    loss = mean_{b,i} softplus(-(1 - 2 x_i) P_i^L).

The gradient with respect to w comes from float64 reverse-mode automatic
differentiation (torch on the CPU) over this plain re-implementation; no
gradient flows through an active clamp (the derivative of clamp outside its
range is 0).  w = 1 reproduces `oracle.bp` exactly in arithmetic (pinned).
"""
from __future__ import annotations

import numpy as np

LLR_MAX = 30.0


def _torch():
    import torch

    return torch


class _Graph:
    def __init__(self, code):
        torch = _torch()
        self.n, self.m, self.e = code.n, code.m, code.e
        self.v = torch.as_tensor(code.v, dtype=torch.long)
        self.c = torch.as_tensor(code.c, dtype=torch.long)
        self.t = torch.as_tensor(code.t, dtype=torch.long)
        deg = np.bincount(code.c, minlength=code.m)
        first = np.concatenate([[0], np.cumsum(deg)])
        self.groups = []
        for d in np.unique(deg):
            if d == 0:
                continue
            chk = np.nonzero(deg == d)[0]
            eidx = first[chk][:, None] + np.arange(d)[None, :]
            self.groups.append((torch.as_tensor(chk), torch.as_tensor(eidx)))


def forward(code, llr, syn, weights, iters: int):
    """Posteriors after `iters` weighted iterations.

    llr float64 tensor [B, N]; syn uint8 array [B, M]; weights float64 tensor
    [T, iters] (may require grad).  Returns float64 tensor [B, N]."""
    torch = _torch()
    g = _Graph(code)
    sgn = torch.as_tensor(1.0 - 2.0 * np.asarray(syn, dtype=np.float64))
    v2c = llr[:, g.v]  # Step 2
    post = llr
    for it in range(iters):
        x = torch.clamp(v2c, -LLR_MAX, LLR_MAX)
        th = torch.tanh(x / 2.0)
        c2v = torch.zeros_like(v2c)
        for chk, eidx in g.groups:
            t = th[:, eidx]  # [B, n_d, d]
            ones = torch.ones_like(t[..., :1])
            prefix = torch.cumprod(torch.cat([ones, t[..., :-1]], dim=-1), dim=-1)
            suffix = torch.flip(torch.cumprod(torch.cat([ones, torch.flip(t[..., 1:], [-1])], dim=-1), dim=-1), [-1])
            r = sgn[:, chk][..., None] * 2.0 * torch.atanh(prefix * suffix)
            c2v[:, eidx] = r
        c2v = c2v * weights[g.t, it][None, :]          # the learnable scale
        post = llr.index_add(1, g.v, c2v)                # Step 4 / eq. (4)-(5)
        v2c = post[:, g.v] - c2v
    return post


def bce_loss(post, bits):
    torch = _torch()
    s = torch.as_tensor(1.0 - 2.0 * np.asarray(bits, dtype=np.float64))
    return torch.nn.functional.softplus(-s * post).mean()


def loss_and_grad(code, llr, syn, bits, weights, iters: int):
    """(loss, d loss / d weights) in float64; weights numpy [T, iters]."""
    torch = _torch()
    w = torch.tensor(np.asarray(weights, dtype=np.float64), requires_grad=True)
    l64 = torch.as_tensor(np.asarray(llr, dtype=np.float64))
    post = forward(code, l64, syn, w, iters)
    loss = bce_loss(post, bits)
    loss.backward()
    return float(loss.detach()), w.grad.numpy().copy()


def posteriors(code, llr, syn, weights, iters: int) -> np.ndarray:
    torch = _torch()
    with torch.no_grad():
        w = torch.as_tensor(np.asarray(weights, dtype=np.float64))
        return forward(code, torch.as_tensor(np.asarray(llr, dtype=np.float64)), syn, w, iters).numpy()
