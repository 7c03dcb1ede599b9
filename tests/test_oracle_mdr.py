"""Pins of the multidimensional-reconciliation oracle (oracle/mdr.py)."""
import numpy as np
import pytest

from met_inputs import gaussian_raw_keys
from oracle import mdr


def hamilton(a, b):
    """The quaternion product in the basis (1, i, j, k), i^2 = j^2 = k^2 = ijk = -1."""
    a0, a1, a2, a3 = a
    b0, b1, b2, b3 = b
    return np.array([a0 * b0 - a1 * b1 - a2 * b2 - a3 * b3,
                     a0 * b1 + a1 * b0 + a2 * b3 - a3 * b2,
                     a0 * b2 - a1 * b3 + a2 * b0 + a3 * b1,
                     a0 * b3 + a1 * b2 - a2 * b1 + a3 * b0])


def test_table_is_complex_and_quaternion_multiplication():
    rng = np.random.default_rng(1)
    for _ in range(20):
        p, q = rng.standard_normal(2), rng.standard_normal(2)
        z = complex(*p) * complex(*q)
        np.testing.assert_allclose(mdr.mul(p, q), [z.real, z.imag], rtol=0, atol=1e-14)
        p, q = rng.standard_normal(4), rng.standard_normal(4)
        np.testing.assert_allclose(mdr.mul(p, q), hamilton(p, q), rtol=0, atol=1e-14)


def test_octonions_compose_norms_and_are_alternative_not_associative():
    rng = np.random.default_rng(2)
    nonassoc = 0.0
    for _ in range(50):
        p, q, r = rng.standard_normal((3, 8))
        assert abs(np.linalg.norm(mdr.mul(p, q)) - np.linalg.norm(p) * np.linalg.norm(q)) < 1e-12
        np.testing.assert_allclose(mdr.mul(mdr.mul(p, p), q), mdr.mul(p, mdr.mul(p, q)), atol=1e-12)
        np.testing.assert_allclose(mdr.mul(mdr.mul(p, q), q), mdr.mul(p, mdr.mul(q, q)), atol=1e-12)
        nonassoc = max(nonassoc, np.abs(mdr.mul(mdr.mul(p, q), r) - mdr.mul(p, mdr.mul(q, r))).max())
    assert nonassoc > 1e-3   # octonions, not an associative algebra


@pytest.mark.parametrize("d", [1, 2, 4, 8])
def test_rotation_is_orthogonal_and_maps_y_onto_u(d):
    rng = np.random.default_rng(3)
    y = rng.standard_normal((2, 8 * d))
    bits = rng.integers(0, 2, (2, 8 * d)).astype(np.uint8)
    alpha, norm = mdr.bob(y, bits, d)
    for f in range(2):
        for k in range(8):
            blk = slice(k * d, (k + 1) * d)
            M = mdr.rotation(alpha[f, blk], d)
            np.testing.assert_allclose(M.T @ M, np.eye(d), atol=1e-12)
            u = (1.0 - 2.0 * bits[f, blk]) / np.sqrt(d)
            np.testing.assert_allclose(M @ (y[f, blk] / norm[f, k]), u, atol=1e-12)


def test_noiseless_keys_give_u_exactly():
    """x = y: Alice's v is Bob's u, and the LLRs are 2 |y|^2 s / (d sigma^2)."""
    x, y, u = gaussian_raw_keys(64, 3, 0.3, 8)
    alpha, norm = mdr.bob(y, u)
    v, llr = mdr.alice(y, alpha, norm, 0.5)
    s = 1.0 - 2.0 * u
    np.testing.assert_allclose(v, s / np.sqrt(8), atol=1e-12)
    expect = 2.0 * np.repeat(norm, 8, axis=1) ** 2 * s / (8 * 0.5)
    np.testing.assert_allclose(llr, expect, rtol=1e-12)


def test_dimension_one_is_sign_reconciliation():
    """d = 1: M = +-1 and L = 2 (1 - 2b) x y / sigma^2, the BIAWGN LLR of the sign channel."""
    x, y, u = gaussian_raw_keys(200, 2, 0.2, 9)
    alpha, norm = mdr.bob(y, u, 1)
    np.testing.assert_array_equal(np.abs(alpha), 1.0)
    _, llr = mdr.alice(x, alpha, norm, 1.0, 1)
    np.testing.assert_allclose(llr, 2.0 * (1.0 - 2.0 * u) * x.astype(np.float64) * y, rtol=1e-12, atol=1e-15)


def test_noise_norm_identity():
    """w = sqrt(d) |x| v / |y| equals s - sqrt(d) M z / |y|, so |w - s| = sqrt(d) |z| / |y| per block."""
    x, y, u = gaussian_raw_keys(128, 2, 0.25, 10)
    z = y.astype(np.float64) - x.astype(np.float64)
    alpha, norm = mdr.bob(y, u)
    v, _ = mdr.alice(x, alpha, norm, 1.0)
    xb = np.linalg.norm(x.astype(np.float64).reshape(2, -1, 8), axis=-1)
    w = np.sqrt(8) * v.reshape(2, -1, 8) * (xb / norm)[..., None]
    s = (1.0 - 2.0 * u).reshape(2, -1, 8)
    lhs = np.linalg.norm(w - s, axis=-1)
    rhs = np.sqrt(8) * np.linalg.norm(z.reshape(2, -1, 8), axis=-1) / norm
    np.testing.assert_allclose(lhs, rhs, rtol=1e-6)


def test_virtual_channel_matches_its_noise_model():
    """Over many blocks, the scaled noise w - s has the variance d sigma_Z^2 / |y|^2
    the LLR assumes: the normalised residual (w - s) |y| / sqrt(d) has unit variance."""
    x, y, u = gaussian_raw_keys(8 * 4096, 4, 0.2, 11)
    alpha, norm = mdr.bob(y, u)
    v, _ = mdr.alice(x, alpha, norm, 1.0)
    xb = np.linalg.norm(x.astype(np.float64).reshape(4, -1, 8), axis=-1)
    w = np.sqrt(8) * v.reshape(4, -1, 8) * (xb / norm)[..., None]
    r = (w - (1.0 - 2.0 * u).reshape(4, -1, 8)) * norm[..., None] / np.sqrt(8)
    assert abs(r.var() - 1.0) < 0.02 and abs(r.mean()) < 0.01


def test_zero_blocks():
    y = np.zeros((1, 16))
    y[0, 8:] = 1.0
    u = np.zeros((1, 16), dtype=np.uint8)
    alpha, norm = mdr.bob(y, u)
    assert norm[0, 0] == 0.0
    np.testing.assert_allclose(alpha[0, :8], mdr.mul(np.full(8, 1 / np.sqrt(8)), mdr.conj(np.eye(8)[0])))
    v, llr = mdr.alice(np.zeros((1, 16)), alpha, norm, 1.0)
    np.testing.assert_array_equal(v, 0.0)
    np.testing.assert_array_equal(llr, 0.0)
