"""Frame-level parity of a decoder's outcome with the FP64 oracle's.

A frame's outcome is its decoded word, its converged flag and its iteration
count.  Near the decision boundary of BP a change of the inputs by one FP32
rounding can change the outcome of the FP64 oracle itself (another codeword
reached, convergence an iteration later or not at all).  On such frames the
FP32 decoder and the oracle may legitimately differ; everywhere else they must
agree exactly (word, flag) and within one iteration (count).

`compare` applies that rule frame by frame: every frame whose outcome differs
from the oracle's is decoded again by the oracle on `draws` copies of its LLRs,
each moved by a relative 1e-7 (about one FP32 rounding), and the difference is
accepted only if at least one copy changes the oracle's own outcome in the same
respect: its word (for a different word), its flag (for a different flag), its
count or more (for counts more than one apart).  Accepted frames are returned
with one line each, so that tests can print the list.
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
            # the converging side stopping at the last or next-to-last iteration
            # is the one-iteration boundary, not a different outcome
            if (gi if gc else oi) >= max_iter - 1:
                continue
            kind = "flag"
        elif gc and digest(got_bits[f]) != ref["digest"][f]:
            kind = "word"
        elif gc and abs(gi - oi) > 1:
            kind = "iterations"
        else:
            continue
        pr = bp.decode(code_o, perturbed(llr[f], draws, 1000 + f), np.repeat(syn[f:f + 1], draws, axis=0),
                       max_iter)
        flag_moved = bool(np.any(pr.converged != oc_))
        word_moved = flag_moved or any(digest(x) != ref["digest"][f] for x in pr.bits)
        count_moved = word_moved or bool(np.any(pr.iterations != oi))
        shown = {"flag": flag_moved, "word": word_moved, "iterations": count_moved}[kind]
        line = ("frame %d: %s differs (decoder converged %d at %d, oracle %d at %d); oracle under %d "
                "perturbations of 1e-7: converged %s at %s, %d distinct words"
                % (f, kind, gc, gi, oc_, oi, draws, pr.converged.tolist(), pr.iterations.tolist(),
                   len({digest(x) for x in pr.bits})))
        assert shown, "not explained by the oracle's own sensitivity: " + line
        accepted.append(f)
        report.append(line)
    return accepted, report
