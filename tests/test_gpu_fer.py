"""FER parity: the GPU decoder against stored oracle outcomes on 1024 frames.

The golden files hold, per frame, what the FP64 oracle decoded (converged flag,
iterations, frame error, SHA-1 of the decoded bits); they were written by
tests/golden/make_fer_golden.py, which calls only the oracle.  The GPU decodes
the same seeded frames with the same seeded code in one batch of 1024 frames.

Codes: the seeded random construction and progressive edge growth; the
library's graph must hash to the edge list the oracle's construction produced
for the golden file.

Gates: each side's FER inside the other's 95 % Wilson interval; every converged
flag equal to the exact syndrome test of the decoded bits; on every frame both
sides decoded, the oracle's word and count (within one iteration), except
where the oracle itself changes that outcome under FP32-sized perturbations;
frames only one side decoded are frame errors of the other, compared through
the FER, and need the same proof unless the converging side took more than
half the budget (tests/oracle_outcome.py; accepted frames are listed in the
output).
"""
import hashlib
import json
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_1711_01783_amd as met  # noqa: E402
from met_inputs import PROFILES, make_frames  # noqa: E402
from oracle import code as oc  # noqa: E402
from tests import oracle_outcome as oo  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def wilson(k, n, z=1.96):
    p = k / n
    d = 1 + z * z / n
    c = (p + z * z / (2 * n)) / d
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / d
    return c - h, c + h


@pytest.mark.parametrize("construction", ["random", "peg"])
@pytest.mark.parametrize("prof", ["r0.1", "r0.05", "r0.02"])
def test_fer_within_oracle_confidence_interval(prof, construction):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    stem = "fer_peg_%s_N65536.json" if construction == "peg" else "fer_%s_N65536.json"
    with open(os.path.join(GOLDEN, stem % prof)) as f:
        gold = json.load(f)
    frames = gold["frames"]
    n, b = gold["N"], len(frames)
    if construction == "peg":
        code = met.Code.build_peg(PROFILES[prof], n, gold["code_seed"], gold["peg_depth"])
    else:
        code = met.Code.build(PROFILES[prof], n, gold["code_seed"])
    bits, llr = make_frames(n, b, gold["snr"], gold["frame_seed"])
    dev = "cuda:0"
    d_bits = torch.from_numpy(bits).to(dev)
    syn = met.syndrome(code, d_bits)
    print("FER", construction, prof, n, b, gold["snr"], flush=True)
    out = met.decode(code, torch.from_numpy(llr).to(dev), syn, gold["max_iter"])
    torch.cuda.synchronize()
    got = out.bits.cpu().numpy()
    it = out.iterations.cpu().numpy()
    conv = out.converged.cpu().numpy()
    err = np.any(got != bits, axis=1)
    o_err = np.array([x["frame_error"] for x in frames])
    o_conv = np.array([x["converged"] for x in frames])
    o_it = np.array([x["iterations"] for x in frames])
    k_g, k_o = int(err.sum()), int(o_err.sum())
    lo, hi = wilson(k_o, b)
    print("  FER gpu %.4f oracle %.4f (95%% CI %.4f-%.4f)" % (k_g / b, k_o / b, lo, hi), flush=True)
    assert lo <= k_g / b <= hi
    lo_g, hi_g = wilson(k_g, b)
    assert lo_g <= k_o / b <= hi_g
    # frame by frame: the exact syndrome test behind every converged flag, and
    # the oracle's word, flag and count (within one) on every frame except
    # those whose oracle outcome itself moves under 1e-7 input perturbations
    # the oracle's graph: the library's, once its edge list is shown to hash to
    # what the oracle's construction gave when the golden file was written
    vn, cn, et = code.export()
    h = hashlib.sha1()
    for a in (vn, cn, et):
        h.update(np.ascontiguousarray(a, dtype=np.int64).tobytes())
    assert h.hexdigest() == gold["code_sha1"], "the library built another graph than the oracle's construction"
    code_o = oc.from_edges(n, code.M, vn, cn, et, n_edge_types=len(PROFILES[prof].vn_types[0][1]))
    ref = {"converged": o_conv, "iterations": o_it, "digest": [x["bits_sha1"] for x in frames]}
    differ = np.nonzero((conv != o_conv) | (np.abs(it.astype(int) - o_it) > 1)
                        | np.array([conv[f] == 1 and oo.digest(got[f]) != frames[f]["bits_sha1"]
                                    for f in range(b)]))[0]
    print("  %d frames differ from the oracle in word, flag or count (%s)" % (differ.size, differ.tolist()),
          flush=True)
    assert differ.size <= b // 50, "too many frames differ to prove each one"
    acc, rep = oo.compare(code_o, llr, syn.cpu().numpy(), gold["max_iter"], got, conv, it, ref=ref)
    for line in rep:
        print("   ", line, flush=True)
