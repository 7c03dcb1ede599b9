"""Oracle: flooding sum-product decoding against a syndrome, FP64, LLR domain.

TEST INFRASTRUCTURE ONLY (see the package header).

What it computes (paper, Methods, Steps 2-5, eq. (1)-(5)), written in
log-likelihood ratios L = ln p(0)/p(1) = -ln q0 (the paper works with the
ratio q = p(1)/p(0) and mentions the LLR form in its last Methods paragraph):

* Step 2 / eq. (1): every variable-to-check message starts at the channel LLR
  of its variable node, v2c_e = L_v(e).
* Step 3 / eq. (2)-(3), check update, with the syndrome bit of the check:
  c2v_e = (1 - 2 s_j) * 2 artanh( prod_{e' in E(j), e' != e} tanh(x_e' / 2) ),
  where x = v2c clipped to [-30, 30].  In ratios, (1-q)/(1+q) = tanh(L/2) and
  r = (1-t)/(1+t) is the same as L_out = 2 artanh(t); a check whose syndrome bit
  is 1 flips the sign (reading: Bob's syndrome S_B is the target of Step 5).
  The leave-one-out product is formed from prefix and suffix products, never by
  division.
* Step 4 / eq. (4), variable update (flooding: every check used the messages of
  the previous iteration): P_i = L_i + sum_{e in E(i)} c2v_e and
  v2c_e = P_i - c2v_e, which is eq. (4) in logarithms.
* Step 5 / eq. (5): posterior P_i; hard decision c_i = 1 iff P_i < 0 (q > 1),
  a tie P_i = 0 gives 0; stop when H c = S_B (early-exit mode) or after
  max_iter iterations.  The test runs after each full iteration l >= 1.

Pins (tests/test_oracle_*.py): exhaustive MAP on tree codes, the closed-form
two-input check, sign symmetry, the all-zero syndrome textbook case, noiseless
frames.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

LLR_MAX = 30.0


@dataclass
class DecodeResult:
    bits: np.ndarray        # uint8 [B, N]
    iterations: np.ndarray  # int32 [B]
    converged: np.ndarray   # uint8 [B]
    posterior: np.ndarray   # float64 [B, N] at the stopping iteration
    trace: dict             # iteration -> posterior float64 [B, N]


class _Graph:
    """Index structures of a code for the vectorised update."""

    def __init__(self, code):
        self.n, self.m, self.e = code.n, code.m, code.e
        self.v = code.v
        self.c = code.c
        # checks grouped by degree: for degree d, matrix of edge indices [n_d, d]
        deg = np.bincount(code.c, minlength=code.m)
        first = np.concatenate([[0], np.cumsum(deg)])
        self.groups = []
        for d in np.unique(deg):
            if d == 0:
                continue
            chk = np.nonzero(deg == d)[0]
            eidx = first[chk][:, None] + np.arange(d)[None, :]
            self.groups.append((chk, eidx))
        ones = np.ones(code.e)
        # incidence edge -> variable node (E x N) and check -> variable (M x N)
        self.e2v = sp.csr_matrix((ones, (np.arange(code.e), code.v)), shape=(code.e, code.n))
        self.h = sp.csr_matrix((np.ones(code.e, dtype=np.int64), (code.c, code.v)), shape=(code.m, code.n))


def check_update(g: _Graph, v2c: np.ndarray, sgn: np.ndarray) -> np.ndarray:
    """eq. (2)-(3) with the syndrome sign; v2c [B, E], sgn = 1 - 2 s  [B, M]."""
    x = np.clip(v2c, -LLR_MAX, LLR_MAX)
    th = np.tanh(x / 2.0)
    c2v = np.empty_like(v2c)
    for chk, eidx in g.groups:
        t = th[:, eidx]  # [B, n_d, d]
        ones = np.ones_like(t[..., :1])
        prefix = np.cumprod(np.concatenate([ones, t[..., :-1]], axis=-1), axis=-1)
        suffix = np.cumprod(np.concatenate([ones, t[..., :0:-1]], axis=-1), axis=-1)[..., ::-1]
        loo = prefix * suffix
        c2v[:, eidx] = sgn[:, chk][..., None] * 2.0 * np.arctanh(loo)
    return c2v


def variable_update(g: _Graph, llr: np.ndarray, c2v: np.ndarray):
    """eq. (4)-(5): posteriors P [B, N] and extrinsic v2c [B, E]."""
    post = llr + np.asarray((g.e2v.T @ c2v.T).T)
    v2c = post[:, g.v] - c2v
    return post, v2c


def hard_decision(post: np.ndarray) -> np.ndarray:
    """Step 5: c = 1 iff P < 0 (q > 1); P = 0 gives 0."""
    return (post < 0).astype(np.uint8)


def syndrome_of(g: _Graph, bits: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(((g.h @ bits.astype(np.int64).T) % 2).T, dtype=np.uint8))


def decode(code, llr, syn, max_iter: int, early_exit: bool = True, trace_iters=()) -> DecodeResult:
    """Decode frames llr [B, N] (any float, promoted to FP64) against syn [B, M].

    Frames are independent; in early-exit mode a frame stops at the first
    iteration whose hard decision satisfies its syndrome.  In fixed mode every
    frame runs max_iter iterations and `converged` reports the final test.
    `trace_iters` lists iterations whose posteriors are recorded for all frames
    (frames that stopped earlier record their final posterior).
    """
    g = _Graph(code)
    llr = np.atleast_2d(np.asarray(llr, dtype=np.float64))
    syn = np.atleast_2d(np.asarray(syn, dtype=np.uint8))
    b = llr.shape[0]
    sgn = 1.0 - 2.0 * syn.astype(np.float64)
    bits = np.zeros((b, code.n), dtype=np.uint8)
    post_out = llr.copy()
    iters = np.full(b, max_iter, dtype=np.int32)
    conv = np.zeros(b, dtype=np.uint8)
    trace = {}
    act = np.arange(b)
    v2c = llr[:, g.v]  # Step 2
    for it in range(1, max_iter + 1):
        c2v = check_update(g, v2c, sgn[act])             # Step 3
        post, v2c = variable_update(g, llr[act], c2v)     # Step 4
        hard = hard_decision(post)                        # Step 5
        ok = np.all(syndrome_of(g, hard) == syn[act], axis=1)
        bits[act] = hard
        post_out[act] = post
        if it in trace_iters:
            trace[it] = post_out.copy()
        if early_exit:
            done = ok
            conv[act[done]] = 1
            iters[act[done]] = it
            keep = ~done
            act = act[keep]
            v2c = v2c[keep]
            if act.size == 0:
                for later in trace_iters:
                    if later > it:
                        trace[later] = post_out.copy()
                break
        elif it == max_iter:
            conv[act] = ok.astype(np.uint8)
    return DecodeResult(bits, iters, conv, post_out, trace)
