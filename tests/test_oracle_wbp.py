"""Pins of the weighted-BP oracle and its FP64 gradient."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import bp, code as oc, wbp  # noqa: E402
from met_inputs import PROFILES, make_frames  # noqa: E402


def _case(n=1500, b=3, snr=0.2, seed=3, prof="r0.1"):
    code = oc.build(PROFILES[prof], n, seed)
    bits, llr = make_frames(n, b, snr, 100 + seed)
    return code, bits, llr, oc.syndrome(code, bits)


def test_unit_weights_equal_plain_bp():
    code, bits, llr, syn = _case()
    it = 8
    w = np.ones((3, it))
    post = wbp.posteriors(code, llr, syn, w, it)
    ref = bp.decode(code, llr, syn, it, early_exit=False).posterior
    np.testing.assert_allclose(post, ref, rtol=1e-12, atol=1e-12)


def test_gradient_matches_central_differences():
    code, bits, llr, syn = _case(n=600, b=2)
    it = 5
    rng = np.random.default_rng(0)
    w = 1.0 + 0.2 * rng.standard_normal((3, it))
    loss, g = wbp.loss_and_grad(code, llr, syn, bits, w, it)
    h = 1e-6
    for (t, l) in [(0, 0), (1, 2), (1, 4), (2, 4), (0, 3)]:
        wp, wm = w.copy(), w.copy()
        wp[t, l] += h
        wm[t, l] -= h
        lp, _ = wbp.loss_and_grad(code, llr, syn, bits, wp, it)
        lm, _ = wbp.loss_and_grad(code, llr, syn, bits, wm, it)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[t, l]) <= 1e-6 * max(1e-3, abs(g[t, l])), (t, l, fd, g[t, l])


def test_leaf_edge_weights_only_matter_in_last_iteration():
    """Degree-1 VNs always send their channel LLR, so the scales of their edge
    type (type 3) reach the loss only through the final posteriors."""
    code, bits, llr, syn = _case()
    it = 6
    _, g = wbp.loss_and_grad(code, llr, syn, bits, np.ones((3, it)), it)
    assert np.all(g[2, :-1] == 0.0)
    assert g[2, -1] != 0.0
    assert np.all(g[:2] != 0.0)


def test_posteriors_are_affine_in_last_iteration_weights():
    """P^L = L + sum_e w[t(e), L] r_e: doubling the last scales doubles the messages."""
    code, bits, llr, syn = _case()
    it = 4
    w1 = np.ones((3, it))
    w2 = w1.copy()
    w2[:, -1] = 2.0
    w0 = w1.copy()
    w0[:, -1] = 0.0
    p1 = wbp.posteriors(code, llr, syn, w1, it)
    p2 = wbp.posteriors(code, llr, syn, w2, it)
    p0 = wbp.posteriors(code, llr, syn, w0, it)
    np.testing.assert_allclose(p0, llr.astype(np.float64), atol=0)
    np.testing.assert_allclose(p2 - p0, 2 * (p1 - p0), rtol=1e-12, atol=1e-12)
