"""Weighted BP on the GPU against the FP64 oracle (forward and gradient)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

import paper_1711_01783_amd as met  # noqa: E402
from paper_1711_01783_amd import wbp  # noqa: E402
from oracle import code as oc, wbp as owbp  # noqa: E402
from met_inputs import PROFILES, make_frames  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _case(prof, n, b, snr, seed=4):
    code_o = oc.build(PROFILES[prof], n, seed)
    code_g = met.Code.build(PROFILES[prof], n, seed)
    bits, llr = make_frames(n, b, snr, 300 + seed)
    syn = oc.syndrome(code_o, bits)
    return code_o, code_g, bits, llr, syn


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _loss_grad_gpu(code_g, llr, syn, bits, w, k):
    wt = _t(w.astype(np.float32)).requires_grad_(True)
    post = wbp.weighted_bp(wt, code_g, _t(llr), _t(syn), k)
    s = _t(1.0 - 2.0 * bits.astype(np.float32))
    loss = torch.nn.functional.softplus(-s * post).mean()
    loss.backward()
    torch.cuda.synchronize()
    return float(loss.detach()), wt.grad.cpu().numpy(), post.detach().cpu().numpy()


def test_unit_weights_bit_identical_to_plain_decode():
    code_o, code_g, bits, llr, syn = _case("r0.1", 8192, 64, 0.2)
    it = 12
    post, b1, c1, _ = wbp.forward(code_g, _t(llr), _t(syn), torch.ones(3, it, device=DEV), 4)
    out = met.decode(code_g, _t(llr), _t(syn), it, fixed_iters=True, posterior=True)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(post.cpu().numpy(), out.posterior.cpu().numpy())
    np.testing.assert_array_equal(b1.cpu().numpy(), out.bits.cpu().numpy())
    np.testing.assert_array_equal(c1.cpu().numpy(), out.converged.cpu().numpy())


# frame counts 8 and 5 run in groups of 16 frames (four checks per wave), 1 in
# groups of one, 24 in groups of 32 (two checks per wave) and 40 in groups of
# 64 (one check per wave); odd lengths leave a partly filled last wave
@pytest.mark.parametrize("prof,n,b,snr,it", [("r0.1", 4096, 8, 0.2, 10), ("r0.02", 4096, 5, 0.07, 8),
                                             ("r0.05", 3000, 1, 0.12, 6), ("r0.1", 2010, 24, 0.2, 6),
                                             ("r0.02", 2550, 40, 0.07, 5)])
def test_forward_and_gradient_match_fp64_oracle(prof, n, b, snr, it):
    code_o, code_g, bits, llr, syn = _case(prof, n, b, snr)
    rng = np.random.default_rng(1)
    w = (1.0 + 0.15 * rng.standard_normal((3, it))).astype(np.float32)
    print("wbp", prof, n, b, snr, it, flush=True)
    loss_g, grad_g, post_g = _loss_grad_gpu(code_g, llr, syn, bits, w, 3)
    loss_r, grad_r = owbp.loss_and_grad(code_o, llr, syn, bits, w.astype(np.float64), it)
    post_r = owbp.posteriors(code_o, llr, syn, w.astype(np.float64), it)
    err = np.abs(post_g - post_r)
    assert np.all(err <= 1e-3 * np.abs(post_r) + 1e-4), err.max()
    assert abs(loss_g - loss_r) <= 1e-5 * abs(loss_r)
    scale = np.abs(grad_r).max()
    np.testing.assert_allclose(grad_g, grad_r, rtol=2e-3, atol=2e-4 * scale)
    assert np.linalg.norm(grad_g - grad_r) <= 1e-3 * np.linalg.norm(grad_r)
    # leaf-edge scales reach the loss only through the final posteriors
    assert np.all(grad_g[2, :-1] == 0.0)


def test_gradient_independent_of_checkpoint_interval_and_deterministic():
    code_o, code_g, bits, llr, syn = _case("r0.1", 4096, 16, 0.19)
    it = 9
    w = (1.0 + 0.1 * np.random.default_rng(2).standard_normal((3, it))).astype(np.float32)
    ref = _loss_grad_gpu(code_g, llr, syn, bits, w, 1)[1]
    for k in (2, 4, 9, 1):
        print("checkpoint interval", k, flush=True)
        np.testing.assert_array_equal(_loss_grad_gpu(code_g, llr, syn, bits, w, k)[1], ref)


def test_gradient_against_finite_differences_on_the_gpu():
    """Central differences of the FP32 GPU forward (step 1e-2) agree with the
    adjoint to the precision such differences allow."""
    code_o, code_g, bits, llr, syn = _case("r0.1", 4096, 32, 0.2)
    it = 6
    w = np.ones((3, it), dtype=np.float32)
    _, g, _ = _loss_grad_gpu(code_g, llr, syn, bits, w, 2)
    h = 1e-2
    for (t, l) in [(0, 1), (1, 3), (1, 5), (2, 5)]:
        wp, wm = w.copy(), w.copy()
        wp[t, l] += h
        wm[t, l] -= h
        lp = _loss_grad_gpu(code_g, llr, syn, bits, wp, 2)[0]
        lm = _loss_grad_gpu(code_g, llr, syn, bits, wm, 2)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[t, l]) <= 0.02 * abs(g[t, l]) + 1e-6, (t, l, fd, g[t, l])


def test_tree_code_gradient_generic_shapes():
    """Run-time-degree check shapes (tree codes) through the adjoint."""
    from tests.trees import random_tree

    rng = np.random.default_rng(7)
    n, m, v, c, t = random_tree(12, rng)
    code_o = oc.from_edges(n, m, v, c, t, n_edge_types=3)
    code_g = met.Code.from_edges(n, m, v, c, t)
    x = rng.integers(0, 2, (3, n)).astype(np.uint8)
    s = oc.syndrome(code_o, x)
    llr = rng.normal(0.4, 1.2, (3, n)).astype(np.float32)
    it = 5
    w = (1.0 + 0.2 * rng.standard_normal((3, it))).astype(np.float32)
    _, grad_g, _ = _loss_grad_gpu(code_g, llr, s, x, w, 2)
    _, grad_r = owbp.loss_and_grad(code_o, llr, s, x, w.astype(np.float64), it)
    np.testing.assert_allclose(grad_g, grad_r, rtol=2e-3, atol=1e-5 * np.abs(grad_r).max())


def test_gradient_at_fifty_iterations_with_checkpoints_every_ten():
    """The training configuration's depth (50 unrolled iterations, message state
    kept every 10th) and operating point (rate 0.1, SNR 0.157) at N = 4096.

    Over 50 iterations the FP64 oracle's own gradient moves by about 3e-5 (norm,
    relative) when its inputs move by one FP32 rounding (relative 1e-7), so the
    FP32 adjoint is held to the same bounds as at 10 iterations: 1e-3 of the
    gradient's norm, and 2e-3 element-wise with a floor of 2e-4 of its largest
    element."""
    code_o, code_g, bits, llr, syn = _case("r0.1", 4096, 8, 0.157)
    it = 50
    w = (1.0 + 0.1 * np.random.default_rng(1).standard_normal((3, it))).astype(np.float32)
    print("wbp L=50 k=10", flush=True)
    loss_g, grad_g, post_g = _loss_grad_gpu(code_g, llr, syn, bits, w, 10)
    loss_r, grad_r = owbp.loss_and_grad(code_o, llr, syn, bits, w.astype(np.float64), it)
    assert abs(loss_g - loss_r) <= 1e-5 * abs(loss_r), (loss_g, loss_r)
    rel = np.linalg.norm(grad_g - grad_r) / np.linalg.norm(grad_r)
    print("  loss %.8f / %.8f, gradient norm error %.3g" % (loss_g, loss_r, rel), flush=True)
    assert rel <= 1e-3
    np.testing.assert_allclose(grad_g, grad_r, rtol=2e-3, atol=2e-4 * np.abs(grad_r).max())
    assert np.all(grad_g[2, :-1] == 0.0)
    # the same gradient with every iteration kept
    np.testing.assert_array_equal(_loss_grad_gpu(code_g, llr, syn, bits, w, 1)[1], grad_g)
