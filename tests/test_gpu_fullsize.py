"""Parity at the benchmark's full size, in the benchmark's launch configuration.

N = 10^6 with 64 frames per code (one group of 64 frames, the check kernels'
default steps per wave), as `bench.py` decodes them.  The FP64 oracle cannot
decode 64 frames of 10^6 bits in test time, so it decodes sampled frames for a
few iterations (the posteriors of eq. (5) after 6 fixed iterations, Methods,
Steps 2-4), compared element by element; every frame is checked through
properties that hold at any size: converged frames satisfy their syndrome
(Step 5) bit-exactly, the batched form reproduces the plain form bit for bit,
and the syndrome kernel equals the oracle's H x.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_1711_01783_amd as met  # noqa: E402
from oracle import bp, code as oc  # noqa: E402
from met_inputs import BJ_SNR, PROFILES, WATERFALL_SNR, make_frames  # noqa: E402

DEV = "cuda:0"
N, B = 10**6, 64
SEED = {"r0.1": 101, "r0.05": 102, "r0.02": 103}   # the benchmark's codes
SAMPLE = (0, 37, 63)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("prof", ["r0.1", "r0.02"])
def test_sampled_frames_match_oracle_at_full_size(prof):
    code_o = oc.build(PROFILES[prof], N, SEED[prof])
    code_g = met.Code.build(PROFILES[prof], N, SEED[prof])
    bits, llr = make_frames(N, B, BJ_SNR[prof], 5000)
    syn = oc.syndrome(code_o, bits)
    d_syn = torch.from_numpy(syn).to(DEV)
    np.testing.assert_array_equal(met.syndrome(code_g, torch.from_numpy(bits).to(DEV)).cpu().numpy(), syn)
    it = 6
    out = met.decode(code_g, torch.from_numpy(llr).to(DEV), d_syn, it, fixed_iters=True, posterior=True)
    torch.cuda.synchronize()
    post = out.posterior.cpu().numpy()
    for f in SAMPLE:
        print("full size", prof, "frame", f, flush=True)
        ref = bp.decode(code_o, llr[f:f + 1], syn[f:f + 1], it, early_exit=False).posterior[0]
        err = np.abs(post[f] - ref)
        bad = err > 1e-3 * np.abs(ref) + 1e-4
        assert not bad.any(), (f, int(bad.sum()), float(err.max()))


def test_full_size_properties_at_waterfall():
    """Rate 0.1 at SNR 0.19, where about half the frames converge: every
    converged frame's bits satisfy its syndrome; batched and plain forms agree
    bit for bit."""
    prof = "r0.1"
    code = met.Code.build(PROFILES[prof], N, SEED[prof])
    bits, llr = make_frames(N, B, WATERFALL_SNR[prof], 6000)
    d_bits = torch.from_numpy(bits).to(DEV)
    syn = met.syndrome(code, d_bits)
    d_llr = torch.from_numpy(llr).to(DEV)
    plain = met.decode(code, d_llr, syn, 100)
    batched = met.decode_batched([met.Job(code, d_llr, syn, 100)])[0]
    torch.cuda.synchronize()
    conv = plain.converged.cpu().numpy() == 1
    print("converged", int(conv.sum()), "of", B, flush=True)
    assert conv.sum() >= B // 4
    got = met.syndrome(code, plain.bits).cpu().numpy()
    np.testing.assert_array_equal(got[conv], syn.cpu().numpy()[conv])
    # a converged frame that differs from the sent bits differs by a codeword of
    # the code (these random codes have low-weight ones: short cycles among the
    # degree-24 nodes' two type-1 edges); counted, not gated
    wrong = ~np.all(plain.bits.cpu().numpy()[conv] == bits[conv], axis=1)
    print("undetected errors among converged frames:", int(wrong.sum()), flush=True)
    for a, b in ((plain.bits, batched.bits), (plain.iterations, batched.iterations),
                 (plain.converged, batched.converged)):
        np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
