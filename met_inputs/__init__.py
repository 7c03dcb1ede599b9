"""Seeded synthetic inputs shared by the decoder's tests, its benchmark and the oracle.

This module holds no decoding arithmetic.  It supplies only what both sides are
given as input:

* the multi-edge-type degree profiles of the three code rates (data, not code);
* per-frame random information bits;
* the channel: BPSK over AWGN, turned into FP32 log-likelihood ratios.

The paper's workloads are raw keys of a CV-QKD system after multidimensional
reconciliation, which by construction behave as a binary-input AWGN channel
(Results, "Information reconciliation for CV-QKD system").  Those keys and the
paper's own degree distributions are not available, so the frames here are
synthetic stand-ins with the same channel model.

Conventions
-----------
* SNR is the ratio for unit-energy BPSK: noise variance sigma^2 = 1 / SNR.  With
  this reading the efficiency beta = R / (0.5 * log2(1 + SNR)) reproduces the
  paper's Table 1 (93.40 / 95.84 / 96.99 %).
* bit x in {0, 1} is sent as 1 - 2x; y = (1 - 2x) + n,  n ~ N(0, 1/SNR).
* LLR L = ln p(y | x=0) / p(y | x=1) = 2 y / sigma^2 = 2 * SNR * y, cast to FP32.
  (The paper's Step 2 uses the inverse ratio q0 = p(1)/p(0), so L = -ln q0.)
* frame f of a batch drawn with base seed s uses numpy PCG64(s + f): a frame's
  content does not depend on the batch it is drawn in.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Profile",
    "PROFILES",
    "BJ_SNR",
    "WATERFALL_SNR",
    "ITER_BUDGET",
    "frame_bits",
    "channel_llr",
    "make_frames",
    "beta_efficiency",
    "gaussian_raw_keys",
]


@dataclass(frozen=True)
class Profile:
    """A multi-edge-type degree profile.

    ``vn_types`` rows are (fraction of N, degrees per edge type); ``cn_types`` rows
    are (fraction of N, degrees per edge type).  Edge types are numbered from 0.
    """

    name: str
    rate: float
    vn_types: tuple  # ((frac, (d_t0, d_t1, ...)), ...)
    cn_types: tuple

    @property
    def n_edge_types(self) -> int:
        return len(self.vn_types[0][1])


# Rate 0.1: 12 % variable nodes of degree 24 (2 type-1 + 22 type-2 edges), 88 %
# degree-1 variable nodes (one type-3 edge); checks 0.02 N of degree 12 (type-1)
# plus 0.88 N with three type-2 edges and one type-3 edge.
# Rate 0.05: 6 % degree-49 (2 + 47), checks 0.01 N degree-12 + 0.94 N (3 + 1).
# Rate 0.02: 3 % degree-99 (2 + 97), checks 0.01 N degree-6 + 0.97 N (3 + 1).
# (Type numbering in the comments is 1-based; in the tuples it is 0-based.)
PROFILES = {
    "r0.1": Profile(
        "r0.1", 0.1,
        vn_types=((0.12, (2, 22, 0)), (0.88, (0, 0, 1))),
        cn_types=((0.02, (12, 0, 0)), (0.88, (0, 3, 1))),
    ),
    "r0.05": Profile(
        "r0.05", 0.05,
        vn_types=((0.06, (2, 47, 0)), (0.94, (0, 0, 1))),
        cn_types=((0.01, (12, 0, 0)), (0.94, (0, 3, 1))),
    ),
    "r0.02": Profile(
        "r0.02", 0.02,
        vn_types=((0.03, (2, 97, 0)), (0.97, (0, 0, 1))),
        cn_types=((0.01, (6, 0, 0)), (0.97, (0, 3, 1))),
    ),
}

# Operating points of the benchmark workloads (about 95 % of capacity).
BJ_SNR = {"r0.1": 0.157, "r0.05": 0.0757, "r0.02": 0.0296}
# Iteration budgets per rate (paper Table 1: 100 / 150 / 200).
ITER_BUDGET = {"r0.1": 100, "r0.05": 150, "r0.02": 200}
# Points in the waterfall region of these profiles at moderate length, where the
# frame error rate is strictly between 0 and 1 (chosen with the oracle).
WATERFALL_SNR = {"r0.1": 0.19, "r0.05": 0.10, "r0.02": 0.065}


def beta_efficiency(rate: float, snr: float) -> float:
    """Reconciliation efficiency beta = R / C with C = 0.5 log2(1 + SNR)."""
    return rate / (0.5 * math.log2(1.0 + snr))


def _rng(seed: int, frame: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed) + int(frame)))


def frame_bits(n: int, frames: int, seed: int, first_frame: int = 0) -> np.ndarray:
    """Uniform random bits, uint8 [frames, n]; frame f uses PCG64(seed + f)."""
    out = np.empty((frames, n), dtype=np.uint8)
    for i in range(frames):
        g = _rng(seed, first_frame + i)
        out[i] = g.integers(0, 2, size=n, dtype=np.uint8)
    return out


def channel_llr(bits: np.ndarray, snr: float, seed: int, first_frame: int = 0) -> np.ndarray:
    """BPSK + AWGN at the given SNR; returns FP32 LLRs [frames, n].

    The noise of frame f comes from the same PCG64(seed + f) stream as its bits,
    drawn after them, so (bits, llr) of a frame depend only on (seed, f).
    """
    frames, n = bits.shape
    out = np.empty((frames, n), dtype=np.float32)
    sigma = 1.0 / math.sqrt(snr)
    for i in range(frames):
        g = _rng(seed, first_frame + i)
        g.integers(0, 2, size=n, dtype=np.uint8)  # skip the bit draws
        noise = g.standard_normal(n)
        y = (1.0 - 2.0 * bits[i].astype(np.float64)) + sigma * noise
        out[i] = (2.0 * snr * y).astype(np.float32)
    return out


def make_frames(n: int, frames: int, snr: float, seed: int, first_frame: int = 0):
    """(bits uint8 [frames, n], llr float32 [frames, n]) for one seed."""
    bits = frame_bits(n, frames, seed, first_frame)
    llr = channel_llr(bits, snr, seed, first_frame)
    return bits, llr


def gaussian_raw_keys(n: int, frames: int, snr: float, seed: int, first_frame: int = 0):
    """Correlated Gaussian raw keys of a CV-QKD run and Bob's random string.

    Returns (x, y, u): x float32 [frames, n] Alice's variables, X ~ N(0, SNR)
    (unit noise, so that SNR = sigma_X^2 / sigma_Z^2); y float32 Bob's,
    Y = X + Z with Z ~ N(0, 1) (Results, "Information reconciliation for CV-QKD
    system"); u uint8 [frames, n] the uniform bits Bob maps his variables onto.
    Frame f draws x, then z, then u from PCG64(seed + f), in that order.
    """
    x = np.empty((frames, n), dtype=np.float32)
    y = np.empty((frames, n), dtype=np.float32)
    u = np.empty((frames, n), dtype=np.uint8)
    sx = math.sqrt(snr)
    for i in range(frames):
        g = _rng(seed, first_frame + i)
        xf = sx * g.standard_normal(n)
        zf = g.standard_normal(n)
        x[i] = xf.astype(np.float32)
        y[i] = (xf + zf).astype(np.float32)
        u[i] = g.integers(0, 2, size=n, dtype=np.uint8)
    return x, y, u
