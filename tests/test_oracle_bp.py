"""Pins of the FP64 BP oracle against exact inference, closed forms and invariants."""
import numpy as np
import pytest

from oracle import bp, code as oc, map as omap
from met_inputs import PROFILES, make_frames
from tests.trees import random_tree


def _tree_code(seed, n_vn):
    rng = np.random.default_rng(seed)
    n, m, v, c, t = random_tree(n_vn, rng)
    return oc.from_edges(n, m, v, c, t, n_edge_types=3), rng


@pytest.mark.parametrize("seed", range(12))
def test_bp_equals_exhaustive_map_on_trees(seed):
    """On a tree BP is exact: posteriors equal brute-force MAP to 1e-10."""
    code, rng = _tree_code(seed, 6 + seed % 10)
    x = rng.integers(0, 2, code.n).astype(np.uint8)
    s = oc.syndrome(code, x)[0]
    # flip some syndrome bits too: any reachable syndrome is a valid target
    llr = rng.normal(0.0, 2.0, code.n)
    res = bp.decode(code, llr[None], s[None], max_iter=2 * code.n + 2, early_exit=False)
    ref = omap.posteriors(code, llr, s)
    np.testing.assert_allclose(res.posterior[0], ref, rtol=0, atol=1e-10)


@pytest.mark.parametrize("seed", range(4))
def test_bp_map_with_random_reachable_syndrome(seed):
    """Syndrome sign (reading: factor 1 - 2 s_j on the check rule) against MAP."""
    code, rng = _tree_code(100 + seed, 12)
    for _ in range(3):
        x = rng.integers(0, 2, code.n).astype(np.uint8)
        s = oc.syndrome(code, x)[0]
        llr = rng.normal(0.5, 1.5, code.n)
        res = bp.decode(code, llr[None], s[None], max_iter=30, early_exit=False)
        np.testing.assert_allclose(res.posterior[0], omap.posteriors(code, llr, s), atol=1e-10)


def test_map_closed_forms():
    """The MAP pin itself: two-VN parity and a single degree-3 check."""
    code = oc.from_edges(2, 1, [0, 1], [0, 0])
    for s in (0, 1):
        p = omap.posteriors(code, np.array([0.7, -1.3]), np.array([s]))
        np.testing.assert_allclose(p, [0.7 + (1 - 2 * s) * -1.3, -1.3 + (1 - 2 * s) * 0.7], atol=1e-12)
    code3 = oc.from_edges(3, 1, [0, 1, 2], [0, 0, 0])
    a, b, c = 0.4, -2.1, 1.7
    for s in (0, 1):
        p = omap.posteriors(code3, np.array([a, b, c]), np.array([s]))
        boxplus = np.log((1 + np.exp(a + b)) / (np.exp(a) + np.exp(b)))
        np.testing.assert_allclose(p[2], c + (1 - 2 * s) * boxplus, atol=1e-12)


@pytest.mark.parametrize("s", [0, 1])
def test_two_input_check_closed_form(s):
    """A degree-3 check: c2v = (1-2s) ln((1 + e^(a+b)) / (e^a + e^b))."""
    code = oc.from_edges(3, 1, [0, 1, 2], [0, 0, 0])
    g = bp._Graph(code)
    rng = np.random.default_rng(5)
    v2c = rng.normal(0, 4, (50, 3))
    out = bp.check_update(g, v2c, np.full((50, 1), 1.0 - 2 * s))
    for k in range(3):
        a, b = v2c[:, (k + 1) % 3], v2c[:, (k + 2) % 3]
        ref = (1 - 2 * s) * np.log((1 + np.exp(a + b)) / (np.exp(a) + np.exp(b)))
        np.testing.assert_allclose(out[:, k], ref, rtol=1e-12, atol=1e-12)


def test_check_update_clamps_inputs():
    """Inputs beyond +-30 act as +-30 (the shared clamp); outputs stay finite."""
    code = oc.from_edges(3, 1, [0, 1, 2], [0, 0, 0])
    g = bp._Graph(code)
    out_big = bp.check_update(g, np.array([[500.0, 400.0, -1e9]]), np.ones((1, 1)))
    out_cl = bp.check_update(g, np.array([[30.0, 30.0, -30.0]]), np.ones((1, 1)))
    np.testing.assert_array_equal(out_big, out_cl)
    assert np.all(np.isfinite(out_big))
    assert abs(out_big[0, 2] - 29.3068528) < 1e-3  # 30 boxplus 30 = 30 - ln 2 + O(e^-30)


def test_sign_symmetry_invariant():
    """decode(L, H x) equals decode((1-2x) L, 0) with posteriors times (1-2x)."""
    code = oc.build(PROFILES["r0.1"], 2000, 9)
    bits, llr = make_frames(code.n, 3, 0.2, 42)
    s = oc.syndrome(code, bits)
    flip = 1.0 - 2.0 * bits
    a = bp.decode(code, llr, s, 15, early_exit=False)
    b = bp.decode(code, flip * llr.astype(np.float64), np.zeros_like(s), 15, early_exit=False)
    np.testing.assert_array_equal(a.posterior, flip * b.posterior)
    np.testing.assert_array_equal(a.converged, b.converged)
    nz = a.posterior != 0
    np.testing.assert_array_equal(a.bits[nz], (b.bits ^ bits)[nz])


def test_noiseless_frames_converge_at_first_iteration():
    code = oc.build(PROFILES["r0.05"], 3000, 3)
    rng = np.random.default_rng(1)
    x = rng.integers(0, 2, (4, code.n)).astype(np.uint8)
    s = oc.syndrome(code, x)
    llr = 2 * 0.5 * (1.0 - 2.0 * x)
    r = bp.decode(code, llr, s, 50)
    np.testing.assert_array_equal(r.iterations, 1)
    np.testing.assert_array_equal(r.converged, 1)
    np.testing.assert_array_equal(r.bits, x)


def test_converged_implies_syndrome_and_early_exit_counts():
    """converged => H c = s; the count is the first iteration at which it holds."""
    code = oc.build(PROFILES["r0.1"], 8192, 2)
    bits, llr = make_frames(code.n, 6, 0.24, 11)
    s = oc.syndrome(code, bits)
    r = bp.decode(code, llr, s, 60)
    assert r.converged.sum() >= 3
    for f in range(6):
        if r.converged[f]:
            np.testing.assert_array_equal(oc.syndrome(code, r.bits[f:f + 1])[0], s[f])
    # fixed-iteration runs one short of each stop must not satisfy the syndrome
    for f in np.nonzero(r.converged)[0]:
        it = int(r.iterations[f])
        if it > 1:
            q = bp.decode(code, llr[f:f + 1], s[f:f + 1], it - 1, early_exit=False)
            assert q.converged[0] == 0
        q = bp.decode(code, llr[f:f + 1], s[f:f + 1], it, early_exit=False)
        assert q.converged[0] == 1
        np.testing.assert_array_equal(q.bits[0], r.bits[f])


def test_hard_decision_tie_goes_to_zero():
    """Step 5: c = 1 iff q > 1, i.e. P < 0; P = 0 gives 0."""
    np.testing.assert_array_equal(bp.hard_decision(np.array([[-1e-300, 0.0, -0.0, 1e-300]])), [[1, 0, 0, 0]])


def test_far_below_threshold_never_converges():
    code = oc.build(PROFILES["r0.1"], 4096, 4)
    bits, llr = make_frames(code.n, 3, 0.05, 3)
    r = bp.decode(code, llr, oc.syndrome(code, bits), 20)
    np.testing.assert_array_equal(r.converged, 0)
    np.testing.assert_array_equal(r.iterations, 20)
