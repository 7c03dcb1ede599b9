"""Oracle: seeded MET-LDPC code construction and syndrome (FP-free, exact).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper builds its parity-check matrices with progressive edge growth from
degree distributions that are not available (Methods, first paragraph).  The
construction here is the one this project fixes instead: a random socket
permutation per edge type, drawn from a seed.  It is specified exactly so that
the product's C++ builder and this independent re-implementation produce the
same graph bit for bit.

Specification
-------------
1. Variable-node counts: VN types in profile order; every type but the last gets
   floor(frac * N + 1e-6) nodes, the last gets the remainder.  VNs are numbered
   type by type.
2. VN sockets of edge type t: total S_t = sum over VN types of count * degree.
3. Check-node counts: each edge type with sockets must belong to exactly one CN
   type.  For CN type k, its anchor edge type is the one with the smallest
   non-zero check degree d (lowest type index on ties); the count is
   m_k = round_half_up(S_anchor / d) = (2 S + d) // (2 d).  Checks are numbered
   type by type.
4. Socket balance: for every edge type t of CN type k with degree d, the excess
   D = m_k d - S_t is spread over the first |D| checks of that type, which get
   degree d - 1 (D > 0) or d + 1 (D < 0).  Every check keeps degree >= 2.
5. Random stream of edge type t: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014)
   with state0 = mix(seed ^ mix(t + 1)); next() adds the golden gamma to the
   state and returns mix(state); uniform(n) = (next() * n) >> 64.
6. Socket lists in node order: VN sockets of type t (node v repeated by its
   type-t degree) and CN sockets likewise.  The CN list is shuffled by
   Fisher-Yates (i from n-1 down to 1, j = uniform(i + 1), swap), and edge i of
   type t joins VN socket i with shuffled CN socket i.
7. Multi-edge repair, so that H is a 0/1 matrix: for t in order and edge i of
   type t in socket order, while the pair (v_i, c_i) occurs more than once in the
   whole graph: j = uniform(E_t) from the same stream; if j != i and neither
   (v_i, c_j) nor (v_j, c_i) exists yet, swap the check ends of edges i and j.
   More than 100000 draws for one edge is an error.
8. Edge order of the result: sorted by (check, edge type, variable node).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

M64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
MAX_REPAIR_DRAWS = 100000


def mix64(z: int) -> int:
    """SplitMix64 output function (a bijection on 64-bit words)."""
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


class SplitMix64:
    def __init__(self, state: int):
        self.state = state & M64

    def next(self) -> int:
        self.state = (self.state + GAMMA) & M64
        return mix64(self.state)

    def uniform(self, n: int) -> int:
        return (self.next() * n) >> 64


def edge_type_stream(seed: int, t: int) -> SplitMix64:
    return SplitMix64(mix64((seed & M64) ^ mix64(t + 1)))


@dataclass
class Code:
    """A parity-check graph; edges are listed in (check, type, VN) order."""

    n: int
    m: int
    v: np.ndarray  # int64 [E]  variable node of each edge
    c: np.ndarray  # int64 [E]  check node of each edge
    t: np.ndarray  # int64 [E]  edge type
    n_edge_types: int = 1
    vn_count_per_type: tuple = field(default=())
    cn_count_per_type: tuple = field(default=())

    @property
    def e(self) -> int:
        return int(self.v.size)

    def vn_degree(self) -> np.ndarray:
        return np.bincount(self.v, minlength=self.n)

    def cn_degree(self) -> np.ndarray:
        return np.bincount(self.c, minlength=self.m)

    def stats(self) -> dict:
        """Bookkeeping in the terms of the paper's Table 1."""
        vdeg = self.vn_degree()
        e_type = np.bincount(self.t, minlength=self.n_edge_types)
        n_deg1 = int(np.count_nonzero(vdeg == 1))
        return {
            "N": self.n,
            "M": self.m,
            "E": self.e,
            "E_type": [int(x) for x in e_type],
            "n_deg1": n_deg1,
            # Table 1 note 2: leaf VNs drop out of the check-to-variable passes.
            "edges_to_pass": self.e - n_deg1,
        }


def from_edges(n: int, m: int, v, c, t=None, n_edge_types: int | None = None) -> Code:
    """A code from an explicit edge list (any order); sorted into check order."""
    v = np.asarray(v, dtype=np.int64)
    c = np.asarray(c, dtype=np.int64)
    t = np.zeros_like(v) if t is None else np.asarray(t, dtype=np.int64)
    order = np.lexsort((v, t, c))
    ntypes = int(t.max()) + 1 if n_edge_types is None and t.size else (n_edge_types or 1)
    return Code(n, m, v[order], c[order], t[order], ntypes)


def _node_counts(profile, n: int):
    vn_types = profile.vn_types
    cn_types = profile.cn_types
    ntypes = len(vn_types[0][1])
    counts = []
    for k, (frac, _deg) in enumerate(vn_types):
        if k < len(vn_types) - 1:
            counts.append(int(math.floor(frac * n + 1e-6)))
        else:
            counts.append(n - sum(counts))
    if min(counts) < 0:
        raise ValueError("profile fractions exceed 1")
    sockets = [sum(counts[k] * vn_types[k][1][t] for k in range(len(vn_types))) for t in range(ntypes)]
    owner = [-1] * ntypes
    for k, (_frac, deg) in enumerate(cn_types):
        for t in range(ntypes):
            if deg[t] > 0:
                if owner[t] != -1:
                    raise ValueError("edge type %d belongs to two check types" % t)
                owner[t] = k
    for t in range(ntypes):
        if sockets[t] > 0 and owner[t] == -1:
            raise ValueError("edge type %d has no check type" % t)
    m_counts = []
    for k, (_frac, deg) in enumerate(cn_types):
        present = [t for t in range(ntypes) if deg[t] > 0]
        anchor = min(present, key=lambda t: (deg[t], t))
        d = deg[anchor]
        m_counts.append((2 * sockets[anchor] + d) // (2 * d))
    return counts, m_counts, sockets


def build(profile, n: int, seed: int) -> Code:
    """Seeded construction following the module specification."""
    vn_counts, cn_counts, sockets = _node_counts(profile, n)
    ntypes = profile.n_edge_types
    m = sum(cn_counts)
    vn_type_of = np.repeat(np.arange(len(vn_counts)), vn_counts)
    cn_type_of = np.repeat(np.arange(len(cn_counts)), cn_counts)
    vdeg = np.array([d for _f, d in profile.vn_types], dtype=np.int64)  # [nvt, ntypes]
    cdeg_base = np.array([d for _f, d in profile.cn_types], dtype=np.int64)
    cdeg = cdeg_base[cn_type_of].copy()  # [m, ntypes]
    cn_start = np.concatenate([[0], np.cumsum(cn_counts)])
    for k in range(len(cn_counts)):
        for t in range(ntypes):
            d = int(cdeg_base[k, t])
            if d == 0:
                continue
            excess = cn_counts[k] * d - sockets[t]
            if abs(excess) > cn_counts[k]:
                raise ValueError("cannot balance sockets of edge type %d" % t)
            lo = cn_start[k]
            cdeg[lo:lo + abs(excess), t] += -1 if excess > 0 else 1
    if m and cdeg.sum(axis=1).min() < 2:
        raise ValueError("a check would have degree < 2")

    vs_all, cs_all, ts_all = [], [], []
    streams = []
    for t in range(ntypes):
        vsock = np.repeat(np.arange(n, dtype=np.int64), vdeg[vn_type_of, t])
        csock = np.repeat(np.arange(m, dtype=np.int64), cdeg[:, t])
        assert vsock.size == csock.size
        rng = edge_type_stream(seed, t)
        cs = csock.tolist()
        for i in range(len(cs) - 1, 0, -1):
            j = rng.uniform(i + 1)
            cs[i], cs[j] = cs[j], cs[i]
        vs_all.append(vsock)
        cs_all.append(np.array(cs, dtype=np.int64))
        ts_all.append(np.full(vsock.size, t, dtype=np.int64))
        streams.append(rng)

    _repair(vs_all, cs_all, streams, m)
    v = np.concatenate(vs_all)
    c = np.concatenate(cs_all)
    t = np.concatenate(ts_all)
    order = np.lexsort((v, t, c))
    return Code(n, m, v[order], c[order], t[order], ntypes, tuple(vn_counts), tuple(cn_counts))


def _repair(vs_all, cs_all, streams, m):
    """Step 7 of the specification (removes repeated (VN, check) pairs)."""
    keys = np.concatenate([vs * m + cs for vs, cs in zip(vs_all, cs_all)]) if vs_all else np.zeros(0, np.int64)
    if keys.size == 0:
        return
    uniq, counts = np.unique(keys, return_counts=True)
    if counts.max() <= 1:
        return
    # count(key): the multiplicity in the current graph.  Base counts come from
    # the sorted array; changes made by swaps live in a dict on top of it.
    delta: dict = {}

    def count(key: int) -> int:
        if key in delta:
            return delta[key]
        pos = np.searchsorted(uniq, key)
        if pos < uniq.size and uniq[pos] == key:
            return int(counts[pos])
        return 0

    def setc(key: int, val: int):
        delta[key] = val

    dup_keys = set(uniq[counts > 1].tolist())
    for t, (vs, cs) in enumerate(zip(vs_all, cs_all)):
        rng = streams[t]
        e_t = vs.size
        kt = vs * m + cs
        cand = np.nonzero(np.isin(kt, list(dup_keys)))[0]
        for i in cand.tolist():
            draws = 0
            while True:
                ki = int(vs[i]) * m + int(cs[i])
                if count(ki) <= 1:
                    break
                draws += 1
                if draws > MAX_REPAIR_DRAWS:
                    raise ValueError("multi-edge repair failed")
                j = rng.uniform(e_t)
                if j == i:
                    continue
                a = int(vs[i]) * m + int(cs[j])
                b = int(vs[j]) * m + int(cs[i])
                if count(a) != 0 or count(b) != 0:
                    continue
                kj = int(vs[j]) * m + int(cs[j])
                setc(ki, count(ki) - 1)
                setc(kj, count(kj) - 1)
                cs[i], cs[j] = cs[j], cs[i]
                setc(a, 1)
                setc(b, 1)


def parity_matrix(code: Code):
    """H as a scipy CSR matrix of shape (M, N) with 0/1 entries."""
    import scipy.sparse as sp

    data = np.ones(code.e, dtype=np.int64)
    return sp.csr_matrix((data, (code.c, code.v)), shape=(code.m, code.n))


def syndrome(code: Code, bits: np.ndarray) -> np.ndarray:
    """S = H x mod 2 for each frame; bits uint8 [B, N] -> uint8 [B, M]."""
    bits = np.atleast_2d(np.asarray(bits))
    h = parity_matrix(code)
    s = (h @ bits.astype(np.int64).T) % 2
    return np.ascontiguousarray(np.asarray(s.T, dtype=np.uint8))
