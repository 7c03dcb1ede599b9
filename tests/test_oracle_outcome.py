"""The frame-outcome comparison used by the GPU tests, on the CPU.

Outputs of the oracle itself pass with no frame needing proof; planted
mistakes on well-conditioned frames (a converged flag that is not the syndrome
test of the bits, a count three iterations off, a frame reported unconverged
that the oracle decodes early) are rejected.
"""
import numpy as np
import pytest

from met_inputs import PROFILES, make_frames
from oracle import bp, code as oc
from tests import oracle_outcome as oo


@pytest.fixture(scope="module")
def case():
    code = oc.build(PROFILES["r0.1"], 4096, 2)
    bits, llr = make_frames(4096, 6, 0.35, 17)
    syn = oc.syndrome(code, bits)
    r = bp.decode(code, llr, syn, 40)
    assert r.converged.all() and r.iterations.max() < 20
    return code, llr, syn, r


def test_oracle_outputs_pass_unexplained(case):
    code, llr, syn, r = case
    acc, rep = oo.compare(code, llr, syn, 40, r.bits, r.converged, r.iterations)
    assert acc == [] and rep == []


def test_flag_inconsistent_with_bits_is_rejected(case):
    code, llr, syn, r = case
    conv = r.converged.copy()
    conv[2] = 0
    with pytest.raises(AssertionError, match="syndrome test"):
        oo.compare(code, llr, syn, 40, r.bits, conv, r.iterations)


def test_count_off_by_three_on_a_stable_frame_is_rejected(case):
    code, llr, syn, r = case
    it = r.iterations.copy()
    it[1] += 3
    with pytest.raises(AssertionError, match="iterations differs"):
        oo.compare(code, llr, syn, 40, r.bits, r.converged, it)


def test_missed_convergence_on_a_stable_frame_is_rejected(case):
    code, llr, syn, r = case
    bits, conv, it = r.bits.copy(), r.converged.copy(), r.iterations.copy()
    bits[3] = (llr[3] < 0).astype(np.uint8)     # the channel's hard decision
    assert not np.all(oc.syndrome(code, bits[3:4]) == syn[3:4])
    conv[3], it[3] = 0, 40
    with pytest.raises(AssertionError, match="flag differs"):
        oo.compare(code, llr, syn, 40, bits, conv, it)


def test_late_flag_difference_is_a_frame_error_of_one_side(case):
    """One side converging after more than half the budget, the other not at
    all: accepted and listed (such frames are compared through the FER)."""
    code, llr, syn, r = case
    ref = oo.oracle_outcomes(code, llr, syn, 40)
    ref["converged"] = ref["converged"].copy()
    ref["iterations"] = ref["iterations"].copy()
    ref["converged"][4], ref["iterations"][4] = 0, 40   # as if the oracle had not converged
    it = r.iterations.copy()
    it[4] = 31                                          # and the decoder only late
    acc, rep = oo.compare(code, llr, syn, 40, r.bits, r.converged, it, ref=ref)
    assert acc == [4] and "late convergence" in rep[0]
