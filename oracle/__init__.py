"""CPU FP64 oracle for syndrome-based sum-product decoding of MET-LDPC codes.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, calls or
links this code; only the test suite, the package smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP decoder:
the only common module is ``met_inputs`` (seeded bits, channel LLRs, degree
profiles), which holds no decoding arithmetic.

Contents
--------
code      seeded multi-edge-type code construction (SplitMix64, Fisher-Yates per
          edge type, multi-edge repair) and the syndrome H x mod 2.
bp        flooding belief propagation in the LLR domain, FP64, following the
          paper's Methods section, Steps 2-5 and eq. (1)-(5).
map       exhaustive maximum-a-posteriori decoding for tiny codes (pin for bp).
wbp       weighted BP (learnable scale per edge type and iteration on
          check-to-variable messages) with an FP64 reverse-mode gradient.
mdr       multidimensional reconciliation (the decoder's front end): Bob's
          rotation coefficients and Alice's virtual-channel LLRs from Gaussian
          raw keys, with explicit Cayley-Dickson multiplication matrices.

Every function is pinned by tests under ``tests/`` against something other than
itself (brute-force MAP on tree codes, closed-form boxplus, invariants, the
paper's Table 1 bookkeeping); see each module's header.
"""
from . import code, bp, map  # noqa: F401
