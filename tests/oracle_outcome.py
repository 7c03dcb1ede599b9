"""Frame-level parity of a decoder's outcome with the FP64 oracle's.

A frame's outcome is its decoded word, its converged flag and its iteration
count.  Near the decision boundary of BP a change of the inputs by one FP32
rounding can change the outcome of the FP64 oracle itself (another codeword
reached, convergence an iteration later or not at all).  On such frames the
FP32 decoder and the oracle may legitimately differ; everywhere else they must
agree exactly (word, flag) and within one iteration (count).

`compare` applies that rule frame by frame:

* a frame both sides decoded (converged) must have the same word and a count
  within one iteration, unless the oracle's own outcome moves in that respect
  under FP32-sized perturbations: `draws` copies of its LLRs each moved by a
  relative 1e-7 (about one FP32 rounding of the inputs), and `draws` runs with
  every check-to-variable message multiplied by (1 + 2^-23 n), n standard
  normal, in every iteration (about one FP32 rounding of every message, as an
  FP32 decoder makes them);
* a frame only one side decoded is a frame error of the other: frames that do
  not converge on both sides are compared through the frame error rate (its
  confidence interval is checked by the callers).  Such a flag difference is
  accepted without further proof when the side that converged needed more than
  half the budget (the slow regime where flooding BP turns rounding-sized
  differences into different trajectories; the oracle can sit in a
  non-decoding state for hundreds of iterations while a perturbed trajectory
  escapes it), and otherwise needs the same proof as above;
* the converging side stopping at the last or next-to-last iteration is the
  one-iteration boundary, not a different outcome.

Accepted frames are returned with one line each, so that tests can print them.
"""
from __future__ import annotations

import hashlib

import numpy as np

from oracle import bp, code as oc

REL = 1e-7


def digest(bits_row) -> str:
    return hashlib.sha1(np.ascontiguousarray(bits_row, dtype=np.uint8).tobytes()).hexdigest()


def perturbed(llr_row, draws, seed):
    rng = np.random.default_rng(seed)
    base = np.asarray(llr_row, dtype=np.float64)
    return base[None, :] * (1.0 + REL * rng.standard_normal((draws, base.size)))


MSG_REL = 2.0 ** -23


def noisy_decode(code_o, llr_rows, syn_rows, max_iter, seed):
    """Early-exit decoding by the oracle's own steps with every check-to-variable
    message multiplied by (1 + 2^-23 n) in every iteration; returns
    (converged, iterations, words)."""
    g = bp._Graph(code_o)
    llr_rows = np.asarray(llr_rows, dtype=np.float64)
    syn_rows = np.asarray(syn_rows, dtype=np.uint8)
    b = llr_rows.shape[0]
    rng = np.random.default_rng(seed)
    sgn = 1.0 - 2.0 * syn_rows.astype(np.float64)
    conv = np.zeros(b, dtype=np.uint8)
    iters = np.full(b, max_iter, dtype=np.int32)
    words = np.zeros((b, code_o.n), dtype=np.uint8)
    act = np.arange(b)
    v2c = llr_rows[:, g.v]
    for it in range(1, max_iter + 1):
        c2v = bp.check_update(g, v2c, sgn[act])
        c2v = c2v * (1.0 + MSG_REL * rng.standard_normal(c2v.shape))
        post, v2c = bp.variable_update(g, llr_rows[act], c2v)
        hard = bp.hard_decision(post)
        words[act] = hard
        ok = np.all(bp.syndrome_of(g, hard) == syn_rows[act], axis=1)
        conv[act[ok]] = 1
        iters[act[ok]] = it
        act, v2c = act[~ok], v2c[~ok]
        if act.size == 0:
            break
    return conv, iters, words


def oracle_outcomes(code_o, llr, syn, max_iter):
    """The oracle's early-exit outcome per frame: converged, iterations, word digests."""
    r = bp.decode(code_o, llr, syn, max_iter)
    return {"converged": r.converged.astype(int), "iterations": r.iterations.astype(int),
            "digest": [digest(x) for x in r.bits]}


def compare(code_o, llr, syn, max_iter, got_bits, got_conv, got_iters, ref=None, draws=8):
    """Frame-by-frame check of a decoder's early-exit outcome against the oracle.

    llr [B, N] float32 and syn [B, M] uint8 are the decoder's inputs; got_* its
    outputs.  `ref` holds the oracle's outcomes (as `oracle_outcomes` returns
    them, e.g. from stored goldens); without it the oracle runs here.
    Returns (accepted frames, report lines).  Raises AssertionError on a
    converged flag that is not the exact syndrome test of the decoded bits, or
    on a frame that differs from the oracle without the proof described above.
    """
    conv_exact = np.all(oc.syndrome(code_o, got_bits) == syn, axis=1).astype(np.uint8)
    bad = np.nonzero(conv_exact != np.asarray(got_conv))[0]
    assert bad.size == 0, "converged flag is not the syndrome test of the decoded bits: frames %s" % bad[:10]
    if ref is None:
        ref = oracle_outcomes(code_o, llr, syn, max_iter)
    accepted, report = [], []
    for f in range(llr.shape[0]):
        gc, oc_ = int(got_conv[f]), int(ref["converged"][f])
        gi, oi = int(got_iters[f]), int(ref["iterations"][f])
        if gc != oc_:
            first = gi if gc else oi  # count of the side that converged
            if first >= max_iter - 1:
                continue
            if 2 * first > max_iter:
                accepted.append(f)
                report.append("frame %d: flag differs (decoder converged %d at %d, oracle %d at %d): late "
                              "convergence, a frame error of one side only (rate compared)" % (f, gc, gi, oc_, oi))
                continue
            kind = "flag"
        elif gc and digest(got_bits[f]) != ref["digest"][f]:
            kind = "word"
        elif gc and abs(gi - oi) > 1:
            kind = "iterations"
        else:
            continue
        rows = np.repeat(syn[f:f + 1], draws, axis=0)
        pr = bp.decode(code_o, perturbed(llr[f], draws, 1000 + f), rows, max_iter)
        nc, ni, nw = noisy_decode(code_o, np.repeat(np.asarray(llr[f:f + 1], np.float64), draws, axis=0), rows,
                                  max_iter, 2000 + f)
        all_conv = np.concatenate([pr.converged, nc])
        all_it = np.concatenate([pr.iterations, ni])
        words = {digest(x) for x in pr.bits} | {digest(x) for x in nw}
        flag_moved = bool(np.any(all_conv != oc_))
        word_moved = flag_moved or any(w != ref["digest"][f] for w in words)
        count_moved = word_moved or bool(np.any(all_it != oi))
        shown = {"flag": flag_moved, "word": word_moved, "iterations": count_moved}[kind]
        line = ("frame %d: %s differs (decoder converged %d at %d, oracle %d at %d); oracle under %d input "
                "perturbations of 1e-7 and %d runs with 2^-23 message noise: converged %s at %s, %d distinct words"
                % (f, kind, gc, gi, oc_, oi, draws, draws, all_conv.tolist(), all_it.tolist(), len(words)))
        assert shown, "not explained by the oracle's own sensitivity: " + line
        accepted.append(f)
        report.append(line)
    return accepted, report
