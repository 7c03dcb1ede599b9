"""FER parity: the GPU decoder against stored oracle outcomes on 1024 frames.

The golden files hold, per frame, what the FP64 oracle decoded (converged flag,
iterations, frame error, SHA-1 of the decoded bits); they were written by
tests/golden/make_fer_golden.py, which calls only the oracle.  The GPU decodes
the same seeded frames with the same seeded code in one batch of 1024 frames.
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

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def wilson(k, n, z=1.96):
    p = k / n
    d = 1 + z * z / n
    c = (p + z * z / (2 * n)) / d
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / d
    return c - h, c + h


@pytest.mark.parametrize("prof", ["r0.1", "r0.05", "r0.02"])
def test_fer_within_oracle_confidence_interval(prof):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    with open(os.path.join(GOLDEN, "fer_%s_N65536.json" % prof)) as f:
        gold = json.load(f)
    frames = gold["frames"]
    n, b = gold["N"], len(frames)
    code = met.Code.build(PROFILES[prof], n, gold["code_seed"])
    bits, llr = make_frames(n, b, gold["snr"], gold["frame_seed"])
    dev = "cuda:0"
    d_bits = torch.from_numpy(bits).to(dev)
    syn = met.syndrome(code, d_bits)
    print("FER", prof, n, b, gold["snr"], flush=True)
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
    agree = np.mean(conv == o_conv)
    both = (conv == 1) & (o_conv == 1)
    same_bits = np.mean([hashlib.sha1(got[f].tobytes()).hexdigest() == frames[f]["bits_sha1"]
                         for f in np.nonzero(both)[0]])
    it_close = np.mean(np.abs(it[both].astype(int) - o_it[both]) <= 1)
    print("  converged agreement %.4f, identical bits on both-converged %.4f, iterations within 1: %.4f"
          % (agree, same_bits, it_close), flush=True)
    assert agree >= 0.97
    assert same_bits >= 0.99
    assert it_close >= 0.97
