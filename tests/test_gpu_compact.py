"""Compaction of running frames (early exit, groups of 64 frames).

Every few iterations the decoder writes out frames that stopped and packs the
frames still running into as few groups of 64 as hold them.  A frame's
arithmetic does not depend on its lane, so every output must be identical to
the decode without compaction, and (where both converge) to the FP64 oracle's
bits (Methods, Step 5).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_1711_01783_amd as met  # noqa: E402
from met_inputs import PROFILES, make_frames  # noqa: E402
from oracle import bp, code as oc  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run(code, llr, syn, max_iter, compact):
    out = met.decode(code, llr, syn, max_iter, compact=compact)
    torch.cuda.synchronize()
    return out.bits.cpu().numpy(), out.iterations.cpu().numpy(), out.converged.cpu().numpy()


def _same(a, b):
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("prof,n,b,snr,max_iter", [("r0.1", 16384, 768, 0.19, 60), ("r0.05", 12000, 700, 0.10, 64),
                                                   ("r0.02", 9000, 130, 0.065, 80)])
def test_compaction_changes_nothing_at_waterfall(prof, n, b, snr, max_iter):
    code = met.Code.build(PROFILES[prof], n, 21)
    bits, llr = make_frames(n, b, snr, 4000)
    syn = met.syndrome(code, torch.from_numpy(bits).to(DEV))
    d_llr = torch.from_numpy(llr).to(DEV)
    print("compaction", prof, n, b, snr, max_iter, flush=True)
    on = _run(code, d_llr, syn, max_iter, True)
    off = _run(code, d_llr, syn, max_iter, False)
    _same(on, off)
    it, conv = on[1], on[2]
    # a spread of exit iterations, so that compaction points saw partial groups
    assert 0.2 < conv.mean() < 0.98 and np.unique(it[conv == 1]).size > 5
    # 16 frames spread over the groups against the FP64 oracle: identical bits
    # where both converged, counts within one, and every converged flag equal
    # to the exact syndrome test of the decoded bits
    code_o = oc.build(PROFILES[prof], n, 21)
    pick = np.linspace(0, b - 1, 16).astype(int)
    ref = bp.decode(code_o, llr[pick], oc.syndrome(code_o, bits[pick]), max_iter)
    both = (conv[pick] == 1) & (ref.converged == 1)
    np.testing.assert_array_equal(on[0][pick][both], ref.bits[both])
    assert np.all(np.abs(it[pick][both].astype(int) - ref.iterations[both]) <= 1)
    np.testing.assert_array_equal(conv, np.all(oc.syndrome(code_o, on[0]) == syn.cpu().numpy(), axis=1))


def test_forced_moves_between_groups():
    """Two groups whose few slow frames fit in one: after the first compaction
    point the second group's running frames move into the first."""
    n = 8192
    code = met.Code.build(PROFILES["r0.1"], n, 5)
    b = 128
    bits, llr_hi = make_frames(n, b, 3.0, 77)     # converge at once
    bits_lo, llr_lo = make_frames(n, b, 0.02, 78)  # never converge
    slow = np.zeros(b, dtype=bool)
    slow[50:64] = True                            # 14 slow frames in group 0
    slow[64:74] = True                            # 10 slow frames in group 1
    x = np.where(slow[:, None], bits_lo, bits)
    llr = np.where(slow[:, None], llr_lo, llr_hi).astype(np.float32)
    syn = met.syndrome(code, torch.from_numpy(np.ascontiguousarray(x)).to(DEV))
    d_llr = torch.from_numpy(np.ascontiguousarray(llr)).to(DEV)
    on = _run(code, d_llr, syn, 40, True)
    off = _run(code, d_llr, syn, 40, False)
    _same(on, off)
    assert np.all(on[2][~slow] == 1) and np.all(on[1][~slow] <= 2)
    assert np.all(on[2][slow] == 0) and np.all(on[1][slow] == 40)
    np.testing.assert_array_equal(on[0][~slow], x[~slow])


def test_every_frame_written_once_with_ragged_last_group():
    n = 6000
    code = met.Code.build(PROFILES["r0.05"], n, 8)
    b = 64 * 5 + 17
    bits, llr = make_frames(n, b, 0.12, 99)
    syn = met.syndrome(code, torch.from_numpy(bits).to(DEV))
    d_llr = torch.from_numpy(llr).to(DEV)
    on = _run(code, d_llr, syn, 48, True)
    off = _run(code, d_llr, syn, 48, False)
    _same(on, off)
    # converged frames satisfy their syndrome
    conv = on[2] == 1
    got = met.syndrome(code, torch.from_numpy(on[0]).to(DEV)).cpu().numpy()
    np.testing.assert_array_equal(got[conv], syn.cpu().numpy()[conv])
