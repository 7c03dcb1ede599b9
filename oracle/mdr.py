"""Oracle: multidimensional reconciliation (the front end of the decoder), FP64.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper turns the correlated Gaussian raw keys of Alice (X) and Bob
(Y = X + Z) into a binary string U on Bob's side and a noisy version V of it on
Alice's side by rotating blocks of d Gaussian values (Results, "Information
reconciliation for CV-QKD system"; the rotation itself is the method of its
reference [MD], used in reverse reconciliation: Bob's string is the key, Bob
sends its syndrome, Step 1).  This module writes that method out plainly:

* Algebra.  R^d for d in {1, 2, 4, 8} with the Cayley-Dickson product: an
  element of dimension 2h is a pair (a, b) of elements of dimension h,
  (a, b)(c, d) = (a c - conj(d) b, d a + b conj(c)), conj((a, b)) = (conj(a), -b),
  starting from the reals.  d = 2, 4, 8 give the complex numbers, the
  quaternions and the octonions, composition algebras: |p q| = |p| |q|.  The
  basis products e_i e_j = +-e_k form a table; L_i is the matrix of
  left multiplication by e_i (column j holds e_i e_j).
* Bob, per block of d components: y' = y / |y|, u the block of his bits mapped
  to (1 - 2 b) / sqrt(d) (a unit vector).  The vectors L_i y' (i < d) are an
  orthonormal basis, so alpha_i = <u, L_i y'> gives u = sum_i alpha_i L_i y',
  i.e. M y' = u for M = sum_i alpha_i L_i, an orthogonal matrix.  Bob
  publishes alpha and |y|: for a direction y' uniform on the sphere, alpha is
  uniform on the sphere whatever u is.
* Alice: x' = x / |x|, v = M x'.  Since M x = |y| u - M Z, the scaled
  w = sqrt(d) |x| v / |y| is the sign s = 1 - 2b plus noise of variance
  d sigma_Z^2 / |y|^2 (M is orthogonal), so her log-likelihood ratios are
  L = 2 w / (d sigma_Z^2 / |y|^2) = 2 |x| |y| v / (sqrt(d) sigma_Z^2).
* A block with |y| = 0 takes y' = e_0; a block with |x| = 0 gives v = 0.

Pins (tests/test_oracle_mdr.py): the table against complex multiplication
(d = 2) and the Hamilton product (d = 4), |p q| = |p| |q| and alternativity
for octonions, M orthogonal and M y' = u, noiseless keys giving v = u exactly,
d = 1 reducing to sign reconciliation, the noise norm identity.
"""
from __future__ import annotations

import numpy as np

DIMS = (1, 2, 4, 8)


def _cd_mul(p, q):
    """Cayley-Dickson product of two coefficient vectors of equal length 2^k."""
    n = len(p)
    if n == 1:
        return np.array([p[0] * q[0]])
    h = n // 2
    a, b, c, d = p[:h], p[h:], q[:h], q[h:]
    return np.concatenate([_cd_mul(a, c) - _cd_mul(conj(d), b), _cd_mul(d, a) + _cd_mul(b, conj(c))])


def conj(p):
    """Conjugate: (a, b)* = (a*, -b), the reals self-conjugate."""
    p = np.asarray(p, dtype=np.float64)
    if len(p) == 1:
        return p.copy()
    h = len(p) // 2
    return np.concatenate([conj(p[:h]), -p[h:]])


def mul(p, q):
    """The product of two elements given as length-d coefficient vectors."""
    return _cd_mul(np.asarray(p, dtype=np.float64), np.asarray(q, dtype=np.float64))


def left_matrices(d: int) -> np.ndarray:
    """L[i] (d x d): column j holds the coefficients of e_i e_j."""
    assert d in DIMS
    eye = np.eye(d)
    out = np.zeros((d, d, d))
    for i in range(d):
        for j in range(d):
            out[i][:, j] = mul(eye[i], eye[j])
    return out


def _blocks(a, d):
    a = np.asarray(a, dtype=np.float64)
    assert a.shape[-1] % d == 0
    return a.reshape(a.shape[:-1] + (a.shape[-1] // d, d))


def bob(y, u_bits, d: int = 8):
    """Bob's side: (alpha [B, N] float64, |y| [B, N/d] float64) for y [B, N], bits [B, N]."""
    L = left_matrices(d)
    yb = _blocks(np.atleast_2d(y), d)
    ub = (1.0 - 2.0 * _blocks(np.atleast_2d(u_bits), d)) / np.sqrt(d)
    norm = np.linalg.norm(yb, axis=-1)
    unit = np.zeros(d)
    unit[0] = 1.0
    safe = np.where(norm[..., None] > 0, yb / np.where(norm > 0, norm, 1.0)[..., None], unit)
    # alpha_i = <u, L_i y'>
    basis = np.einsum("ikj,...j->...ik", L, safe)       # [..., i, k] = (L_i y')_k
    alpha = np.einsum("...ik,...k->...i", basis, ub)
    return alpha.reshape(np.atleast_2d(y).shape), norm


def rotation(alpha_block, d: int = 8) -> np.ndarray:
    """M = sum_i alpha_i L_i for one block."""
    return np.einsum("i,ijk->jk", np.asarray(alpha_block, dtype=np.float64), left_matrices(d))


def alice(x, alpha, ynorm, sigma_z2: float, d: int = 8):
    """Alice's side: (v [B, N], llr [B, N]) from her x, Bob's alpha and |y|."""
    L = left_matrices(d)
    xb = _blocks(np.atleast_2d(x), d)
    ab = _blocks(np.atleast_2d(alpha), d)
    xn = np.linalg.norm(xb, axis=-1)
    xs = np.where(xn[..., None] > 0, xb / np.where(xn > 0, xn, 1.0)[..., None], 0.0)
    M = np.einsum("...i,ijk->...jk", ab, L)
    v = np.einsum("...jk,...k->...j", M, xs)
    scale = 2.0 * xn * np.asarray(ynorm, dtype=np.float64) / (np.sqrt(d) * sigma_z2)
    llr = v * scale[..., None]
    shape = np.atleast_2d(x).shape
    return v.reshape(shape), llr.reshape(shape)
