"""Pins of the oracle's code construction, its generator and the input module."""
import json
import math
import os

import numpy as np
import pytest

from oracle import code as oc
from met_inputs import PROFILES, beta_efficiency, make_frames

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_splitmix64_published_vector():
    g = _golden("splitmix64.json")
    rng = oc.SplitMix64(g["seed"])
    assert [str(rng.next()) for _ in range(len(g["outputs"]))] == g["outputs"]


def test_uniform_is_multiply_shift():
    rng = oc.SplitMix64(99)
    raw = oc.SplitMix64(99)
    for n in (1, 2, 3, 1000, 2**31 - 1):
        assert rng.uniform(n) == (raw.next() * n) >> 64


@pytest.mark.parametrize("name", list(PROFILES))
def test_degree_histograms_follow_profile(name):
    prof = PROFILES[name]
    n = 20000
    code = oc.build(prof, n, 5)
    vdeg = code.vn_degree()
    n2 = int(math.floor(prof.vn_types[0][0] * n + 1e-6))
    assert np.all(vdeg[:n2] == sum(prof.vn_types[0][1]))
    assert np.all(vdeg[n2:] == 1)
    # per-type VN degrees
    for t in range(3):
        per = np.bincount(code.v[code.t == t], minlength=n)
        assert np.all(per[:n2] == prof.vn_types[0][1][t])
        assert np.all(per[n2:] == prof.vn_types[1][1][t])
    # checks: type sizes and degrees up to the stated balancing of +-1
    m1 = code.cn_count_per_type[0]
    cdeg = code.cn_degree()
    d1 = sum(prof.cn_types[0][1])
    assert np.all(np.abs(cdeg[:m1] - d1) <= 1)
    assert np.all(np.abs(cdeg[m1:] - 4) <= 1)
    assert code.cn_count_per_type[1] == n - n2  # leaf pairing exact
    # each leaf VN sits on exactly one check with one type-3 edge
    assert np.all(np.bincount(code.c[code.t == 2], minlength=code.m)[m1:] == 1)


def test_no_multi_edges_and_deterministic():
    prof = PROFILES["r0.02"]
    a = oc.build(prof, 5000, 17)
    b = oc.build(prof, 5000, 17)
    c = oc.build(prof, 5000, 18)
    keys = a.v * a.m + a.c
    assert np.unique(keys).size == keys.size
    np.testing.assert_array_equal(a.v, b.v)
    np.testing.assert_array_equal(a.c, b.c)
    assert not np.array_equal(a.v, c.v)


def test_repair_removes_forced_collisions():
    """A dense small profile forces repeated pairs; the repair must remove them."""
    from met_inputs import Profile

    prof = Profile("dense", 0.5, vn_types=((1.0, (3,)),), cn_types=((0.5, (6,)),))
    code = oc.build(prof, 40, 3)
    keys = code.v * code.m + code.c
    assert np.unique(keys).size == keys.size
    assert np.all(code.vn_degree() == 3)
    assert np.all(code.cn_degree() == 6)


def test_edges_sorted_in_check_order():
    code = oc.build(PROFILES["r0.1"], 3000, 1)
    key = (code.c * 3 + code.t) * code.n + code.v
    assert np.all(np.diff(key) > 0)


def test_table1_bookkeeping_at_full_length():
    """Table 1 identities on the rate-0.1 profile at N = 10^6 (counts of this profile)."""
    t1 = _golden("paper_table1.json")
    # the paper's own codes satisfy: updated CNs = (1-R) N, VNs split into
    # updated + ignored = N, edges to pass = total edges - ignored VNs
    for r, m, n2, n1, e, ep in zip(t1["rates"], t1["updated_cns"], t1["updated_vns_deg_gt1"],
                                   t1["ignored_vns_deg1"], t1["total_edges"], t1["edges_to_pass_deg1_skipped"]):
        assert m == round((1 - r) * t1["block_length"])
        assert n2 + n1 == t1["block_length"]
        assert e - n1 == ep
    code = oc.build(PROFILES["r0.1"], 10**6, 2024)
    st = code.stats()
    assert st["M"] == 900000
    assert st["E"] == 3760000
    assert st["n_deg1"] == 880000
    assert st["edges_to_pass"] == 2880000
    assert st["E_type"] == [240000, 2640000, 880000]
    assert st["M"] == round((1 - 0.1) * st["N"])


def test_beta_reproduces_table1():
    """SNR convention: beta = R / (0.5 log2(1+SNR)) gives Table 1's efficiencies."""
    t1 = _golden("paper_table1.json")
    for r, snr, beta in zip(t1["rates"], t1["snr"], t1["beta_percent"]):
        assert abs(100 * beta_efficiency(r, snr) - beta) < 0.01


def test_speed_definition_reproduces_table1():
    """Speed counts N bits per frame: N / (iterations * per-codeword latency)."""
    t1 = _golden("paper_table1.json")
    for it, lat, sp in zip(t1["iterations"], t1["latency_ms_per_iteration_deg1_skipped"], t1["speed_mbit_s_deg1_skipped"]):
        mbit = t1["block_length"] / (it * lat * 1e-3) / 1e6
        assert abs(mbit - sp) / sp < 0.005


def test_channel_llrs_are_consistent():
    """BIAWGN LLRs satisfy E[exp(-L) | x = 0] = 1 only with L = 2 y / sigma^2."""
    n = 400000
    bits, llr = make_frames(n, 1, 0.3, 77)
    l0 = llr[0][bits[0] == 0].astype(np.float64)
    assert abs(np.mean(np.exp(-l0)) - 1.0) < 0.01
    assert abs(np.mean(l0) - 2 * 0.3) < 0.01          # mean 2 SNR
    assert abs(np.var(l0) - 4 * 0.3) < 0.02           # variance 4 SNR


def test_frames_independent_of_batch():
    b1, l1 = make_frames(1000, 5, 0.2, 10)
    b2, l2 = make_frames(1000, 2, 0.2, 10, first_frame=3)
    np.testing.assert_array_equal(b1[3:], b2)
    np.testing.assert_array_equal(l1[3:], l2)
