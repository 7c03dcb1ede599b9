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


def test_bce_loss_closed_forms():
    """The loss against the binary cross-entropy written with probabilities.

    With L = ln p(0)/p(1) (the LLR sign convention of eq. (1), read as a ratio
    of bit probabilities), a posterior P means p(bit = 1) = 1 / (1 + e^P), and
    the cross-entropy of a sent bit x is -ln p(x).  P = ln 3 gives
    p(1) = 1/4: cost ln(4/3) for a sent 0 and ln 4 for a sent 1; P = 0 costs
    ln 2 either way.  A swapped sign convention would exchange the first two.
    """
    post = torch.tensor([[np.log(3.0), np.log(3.0)], [0.0, 0.0]], dtype=torch.float64)
    bits = np.array([[0, 1], [0, 1]], dtype=np.uint8)
    per_bit = [np.log(4.0 / 3.0), np.log(4.0), np.log(2.0), np.log(2.0)]
    assert abs(float(wbp.bce_loss(post, bits)) - np.mean(per_bit)) <= 1e-15
    # one element at a time, against -ln p(x) with p from the posterior ratio
    rng = np.random.default_rng(5)
    p = rng.normal(0.0, 4.0, (3, 7))
    x = rng.integers(0, 2, (3, 7)).astype(np.uint8)
    p1 = 1.0 / (1.0 + np.exp(p))
    direct = -np.mean(np.where(x == 1, np.log(p1), np.log1p(-p1)))
    assert abs(float(wbp.bce_loss(torch.as_tensor(p), x)) - direct) <= 1e-13


def test_bce_loss_gradient_is_probability_minus_bit():
    """d(-ln p(x))/dP = x - p(1): the gradient the adjoint sweep starts from,
    divided by the number of bits averaged."""
    rng = np.random.default_rng(6)
    p = torch.tensor(rng.normal(0.0, 3.0, (2, 5)), requires_grad=True)
    x = rng.integers(0, 2, (2, 5)).astype(np.uint8)
    wbp.bce_loss(p, x).backward()
    p1 = 1.0 / (1.0 + np.exp(p.detach().numpy()))
    np.testing.assert_allclose(p.grad.numpy(), (x - p1) / x.size, rtol=1e-12, atol=1e-15)
