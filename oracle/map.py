"""Oracle: exhaustive MAP decoding against a syndrome (tiny codes only).

TEST INFRASTRUCTURE ONLY (see the package header).

For a code with n <= 22 variable nodes, enumerate every word x in {0,1}^n with
H x = s (mod 2).  With channel LLRs L (ln p(0)/p(1)), the likelihood of x is
proportional to exp(sum_k L_k (1 - 2 x_k) / 2).  The bitwise MAP posterior is

    P_i = ln sum_{x: Hx=s, x_i=0} w(x)  -  ln sum_{x: Hx=s, x_i=1} w(x).

On a code whose Tanner graph is a tree, sum-product BP reaches exactly these
posteriors after as many iterations as the graph's diameter, which is what pins
the check rule, its syndrome sign, the variable rule and the LLR convention of
the BP oracle.
"""
from __future__ import annotations

import numpy as np


def _logsumexp(a: np.ndarray, axis=None):
    mx = np.max(a, axis=axis, keepdims=True)
    out = mx + np.log(np.sum(np.exp(a - mx), axis=axis, keepdims=True))
    return np.squeeze(out, axis=axis)


def posteriors(code, llr, syn) -> np.ndarray:
    """Bitwise MAP log-ratios for one frame: llr [N], syn [M] -> float64 [N]."""
    n, m = code.n, code.m
    if n > 22:
        raise ValueError("exhaustive MAP is limited to n <= 22")
    llr = np.asarray(llr, dtype=np.float64)
    syn = np.asarray(syn, dtype=np.int64)
    words = ((np.arange(1 << n)[:, None] >> np.arange(n)[None, :]) & 1).astype(np.int64)  # [2^n, n]
    h = np.zeros((m, n), dtype=np.int64)
    h[code.c, code.v] = 1
    ok = np.all((words @ h.T) % 2 == syn[None, :], axis=1)
    words = words[ok]
    if words.shape[0] == 0:
        raise ValueError("syndrome not reachable")
    logw = (llr[None, :] * (1 - 2 * words) / 2.0).sum(axis=1)
    out = np.empty(n)
    for i in range(n):
        z = words[:, i] == 0
        a = _logsumexp(logw[z]) if np.any(z) else -np.inf
        b = _logsumexp(logw[~z]) if np.any(~z) else -np.inf
        out[i] = a - b
    return out
