"""8-bit storage of check-to-variable messages (MET_C2V_Q8).

The check and variable updates compute in float; the stored check-to-variable
messages are 8-bit codes (sign and a 7-bit index into a log-uniform grid of
magnitudes from 2^-14 to 2^5, read back through a table): the quantised,
table-read message storage the paper suggests as a variant (last Methods
paragraph).  Its results are not the float decoder's, so its gate is the frame
error rate: on the 1024 stored oracle outcomes per rate at waterfall points
(random and PEG codes), its FER must lie in the oracle's 95 % interval and the
oracle's in its own.  Exact properties of the storage path: the converged flag
is the exact syndrome test of the returned bits; degree-1 posteriors after
iteration 1, formed in float inside the check update, equal the float
decoder's; frames well above threshold decode to the sent words; two runs are
bit-identical.  The table-driven check update (MET_CHECK_LUT: phi of an input
and the code of an output read from tables on the same grid) is gated the same
way.
"""
import json
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_1711_01783_amd as met  # noqa: E402
from oracle import code as oc  # noqa: E402
from met_inputs import PROFILES, make_frames  # noqa: E402

DEV = "cuda:0"
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def wilson(k, n, z=1.96):
    p = k / n
    d = 1 + z * z / n
    c = (p + z * z / (2 * n)) / d
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / d
    return c - h, c + h


@pytest.mark.parametrize("lut", [False, True])
@pytest.mark.parametrize("construction", ["random", "peg"])
@pytest.mark.parametrize("prof", ["r0.1", "r0.05", "r0.02"])
def test_q8_messages_fer_within_oracle_interval(prof, construction, lut):
    stem = "fer_peg_%s_N65536.json" if construction == "peg" else "fer_%s_N65536.json"
    with open(os.path.join(GOLDEN, stem % prof)) as f:
        gold = json.load(f)
    frames = gold["frames"]
    n, b = gold["N"], len(frames)
    if construction == "peg":
        code = met.Code.build_peg(PROFILES[prof], n, gold["code_seed"], gold["peg_depth"])
    else:
        code = met.Code.build(PROFILES[prof], n, gold["code_seed"])
    vn, cn, et = code.export()
    code_o = oc.from_edges(n, code.M, vn, cn, et, n_edge_types=3)
    bits, llr = make_frames(n, b, gold["snr"], gold["frame_seed"])
    syn = met.syndrome(code, torch.from_numpy(bits).to(DEV))
    print("FER with 8-bit messages", "table-driven check update" if lut else "", construction, prof, n, b,
          gold["snr"], flush=True)
    out = met.decode(code, torch.from_numpy(llr).to(DEV), syn, gold["max_iter"], c2v_q8=True, check_lut=lut)
    torch.cuda.synchronize()
    got = out.bits.cpu().numpy()
    conv = out.converged.cpu().numpy()
    k_q = int(np.any(got != bits, axis=1).sum())
    k_o = int(sum(x["frame_error"] for x in frames))
    lo, hi = wilson(k_o, b)
    lo_q, hi_q = wilson(k_q, b)
    print("  FER 8-bit %.4f oracle %.4f (95%% CI %.4f-%.4f), mean iterations %.1f" % (
        k_q / b, k_o / b, lo, hi, out.iterations.float().mean().item()), flush=True)
    assert lo <= k_q / b <= hi
    assert lo_q <= k_o / b <= hi_q
    s = syn.cpu().numpy()
    np.testing.assert_array_equal(conv, np.all(oc.syndrome(code_o, got) == s, axis=1).astype(np.uint8))


@pytest.mark.parametrize("prof,n,b,snr", [("r0.1", 8192, 64, 0.205), ("r0.02", 8192, 100, 0.068)])
def test_q8_first_iteration_and_determinism(prof, n, b, snr):
    code = met.Code.build(PROFILES[prof], n, 5)
    bits, llr = make_frames(n, b, snr, 11)
    d_llr = torch.from_numpy(llr).to(DEV)
    syn = met.syndrome(code, torch.from_numpy(bits).to(DEV))
    print("first iteration", prof, n, b, flush=True)
    q = met.decode(code, d_llr, syn, 1, fixed_iters=True, posterior=True, c2v_q8=True)
    f = met.decode(code, d_llr, syn, 1, fixed_iters=True, posterior=True)
    q2 = met.decode(code, d_llr, syn, 25, c2v_q8=True)
    q3 = met.decode(code, d_llr, syn, 25, c2v_q8=True)
    torch.cuda.synchronize()
    pq, pf = q.posterior.cpu().numpy(), f.posterior.cpu().numpy()
    vn, _cn, _et = code.export()
    deg = np.bincount(vn, minlength=n)
    leaf = deg == 1
    np.testing.assert_array_equal(pq[:, leaf], pf[:, leaf])
    # a node of degree d >= 2: each of its d stored messages moved by at most
    # 5.4 % of itself (or by less than 2^-14 when it became 0); |c2v| <= 30
    bound = deg[~leaf] * (30.0 * 0.0537 + 2.0 ** -14) + 1e-5 * np.abs(pf[:, ~leaf])
    diff = np.abs(pq[:, ~leaf] - pf[:, ~leaf])
    assert np.all(diff <= bound)
    assert diff.max() > 0  # the storage path is really 8-bit
    for x, y in ((q2.bits, q3.bits), (q2.iterations, q3.iterations), (q2.converged, q3.converged)):
        np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy())


def test_lut_check_update_is_deterministic_and_differs_from_evaluated_phi():
    code = met.Code.build(PROFILES["r0.05"], 8192, 6)
    bits, llr = make_frames(8192, 64, 0.10, 12)
    d_llr = torch.from_numpy(llr).to(DEV)
    syn = met.syndrome(code, torch.from_numpy(bits).to(DEV))
    a = met.decode(code, d_llr, syn, 30, c2v_q8=True, check_lut=True)
    b = met.decode(code, d_llr, syn, 30, c2v_q8=True, check_lut=True)
    e = met.decode(code, d_llr, syn, 2, fixed_iters=True, posterior=True, c2v_q8=True)
    t = met.decode(code, d_llr, syn, 2, fixed_iters=True, posterior=True, c2v_q8=True, check_lut=True)
    torch.cuda.synchronize()
    for x, y in ((a.bits, b.bits), (a.iterations, b.iterations), (a.converged, b.converged)):
        np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy())
    pe, pt = e.posterior.cpu().numpy(), t.posterior.cpu().numpy()
    assert np.any(pe != pt)  # the tables really replace phi
    # both are approximations of the same update: the posteriors agree in sign
    # on nearly every bit after two iterations
    assert np.mean(np.sign(pe) == np.sign(pt)) > 0.97
    s = syn.cpu().numpy()
    from oracle import code as oc2
    vn, cn, et = code.export()
    code_o = oc2.from_edges(8192, code.M, vn, cn, et, n_edge_types=3)
    np.testing.assert_array_equal(a.converged.cpu().numpy(),
                                  np.all(oc2.syndrome(code_o, a.bits.cpu().numpy()) == s, axis=1).astype(np.uint8))


@pytest.mark.parametrize("lut,snr", [(False, 0.3), (False, 0.4), (True, 0.4), (True, 0.5)])
def test_q8_decodes_clean_frames(snr, lut):
    """Well above the waterfall the 8-bit storage decodes every frame that
    float storage decodes, to the sent word.  (At SNR 0.3 one of these 40
    frames is stuck for float and 8-bit storage; the table-driven update, a
    coarser approximation of the same update, leaves one more of them stuck
    there within 60 iterations, so its clean-frame points start at 0.4; its
    FER gate above is the test of its decoding quality.)"""
    code = met.Code.build(PROFILES["r0.1"], 16384, 8)
    bits, llr = make_frames(16384, 40, snr, 13)
    syn = met.syndrome(code, torch.from_numpy(bits).to(DEV))
    d_llr = torch.from_numpy(llr).to(DEV)
    ref = met.decode(code, d_llr, syn, 60)
    out = met.decode(code, d_llr, syn, 60, c2v_q8=True, check_lut=lut)
    torch.cuda.synchronize()
    ok = ref.converged.cpu().numpy() == 1
    assert ok.sum() >= 39
    assert np.all(out.converged.cpu().numpy()[ok] == 1)
    np.testing.assert_array_equal(out.bits.cpu().numpy()[ok], bits[ok])
