"""Oracle: progressive edge growth (PEG) for multi-edge-type codes (exact).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper builds its parity-check matrices with the progressive edge-growth
algorithm (Methods, first paragraph): edges are added one at a time, each from
its variable node to a check as far from that node as the graph built so far
allows, which keeps short cycles out.  This module specifies the variant the
product's C++ builder implements and re-implements it plainly, so that the two
produce the same graph bit for bit.

Specification
-------------
1. Node counts and per-check socket counts cdeg[c][t]: steps 1-4 of the
   random construction (``oracle.code``).
2. Random stream: SplitMix64 stream number T (T = number of edge types; the
   random construction uses streams 0..T-1), one draw per edge.
3. Edges are placed variable node by variable node (v = 0..N-1), and within a
   node edge type by edge type (t = 0..T-1), deg_t(v) edges of each.
4. For edge (v, t): a breadth-first search from v over the edges of type t
   placed so far gives check layers C_1 (the type-t checks of v), C_2 (the
   type-t checks of the nodes reached from C_1, not in earlier layers), ...,
   C_K, stopping early when a layer comes out empty.  K = depth[t].
5. Candidates: checks with a free type-t socket (fill_t(c) < cdeg[c][t]) that
   are not yet neighbours of v (any type).  For k = (number of layers) down to
   1, take the candidates outside C_1 .. C_k; the first k that leaves any
   decides: among them, those with the smallest fill_t form the tie set, and
   the edge goes to its r-th check in increasing check order, r = uniform(size
   of the tie set) from the stream.  No candidate outside C_1 is an error.
6. Result: the edge list sorted by (check, edge type, variable node).

A new edge between v and a check of layer C_k closes a cycle of length 2k;
the choice outside C_1 .. C_K therefore leaves no cycle of length <= 2K in the
type-t subgraph where the graph allows it.

Default depths (``default_depths``): with d_v and d_c the largest type-t
degrees of variable and check nodes, layer k of a full graph holds about
(d_v - 1) g^(k-1) checks, g = (d_v - 1)(d_c - 1); K = 1 when g = 0 (edges of
degree-1 nodes close no cycle), otherwise the largest K (1 <= K <= 16) with
(d_v - 1) g^(K-1) <= 1024, which bounds the work of a search.
"""
from __future__ import annotations

import numpy as np

from .code import Code, _node_counts, edge_type_stream

MAX_DEPTH = 16
LAYER_BUDGET = 1024


def default_depths(profile) -> list:
    """Per-edge-type search depth of the specification's default rule."""
    out = []
    for t in range(profile.n_edge_types):
        dv = max(d[t] for _f, d in profile.vn_types)
        dc = max(d[t] for _f, d in profile.cn_types)
        g = max(dv - 1, 0) * max(dc - 1, 0)
        if g == 0:
            out.append(1)
            continue
        k = 1
        while k < MAX_DEPTH and (dv - 1) * g ** k <= LAYER_BUDGET:
            k += 1
        out.append(k)
    return out


def _socket_degrees(profile, n):
    vn_counts, cn_counts, sockets = _node_counts(profile, n)
    ntypes = profile.n_edge_types
    cn_type_of = np.repeat(np.arange(len(cn_counts)), cn_counts)
    cdeg_base = np.array([d for _f, d in profile.cn_types], dtype=np.int64)
    cdeg = cdeg_base[cn_type_of].copy()
    cn_start = np.concatenate([[0], np.cumsum(cn_counts)]).astype(np.int64)
    for k in range(len(cn_counts)):
        for t in range(ntypes):
            d = int(cdeg_base[k, t])
            if d == 0:
                continue
            excess = cn_counts[k] * d - sockets[t]
            if abs(excess) > cn_counts[k]:
                raise ValueError("cannot balance sockets of edge type %d" % t)
            lo = int(cn_start[k])
            cdeg[lo:lo + abs(excess), t] += -1 if excess > 0 else 1
    if cdeg.shape[0] and cdeg.sum(axis=1).min() < 2:
        raise ValueError("a check would have degree < 2")
    vn_type_of = np.repeat(np.arange(len(vn_counts)), vn_counts)
    vdeg = np.array([d for _f, d in profile.vn_types], dtype=np.int64)[vn_type_of]
    return vn_counts, cn_counts, vdeg, cdeg


def build(profile, n: int, seed: int, depth=None) -> Code:
    """PEG construction following the module specification."""
    ntypes = profile.n_edge_types
    depth = list(default_depths(profile) if depth is None else depth)
    if len(depth) != ntypes or min(depth) < 1 or max(depth) > MAX_DEPTH:
        raise ValueError("depth needs one value in 1..%d per edge type" % MAX_DEPTH)
    vn_counts, cn_counts, vdeg, cdeg = _socket_degrees(profile, n)
    m = int(sum(cn_counts))
    rng = edge_type_stream(seed, ntypes)
    fill = np.zeros((m, ntypes), dtype=np.int64)
    vadj = [[[] for _ in range(n)] for _ in range(ntypes)]  # type-t checks of each VN
    cadj = [[[] for _ in range(m)] for _ in range(ntypes)]  # type-t VNs of each check
    nbrs = [set() for _ in range(n)]                        # all checks of each VN
    owners = [np.nonzero(cdeg[:, t] > 0)[0] for t in range(ntypes)]
    pos = []  # position of a check in owners[t], -1 if it has no type-t socket
    for t in range(ntypes):
        p = np.full(m, -1, dtype=np.int64)
        p[owners[t]] = np.arange(owners[t].size)
        pos.append(p.tolist())
    ev, ec, et = [], [], []
    for v in range(n):
        for t in range(ntypes):
            for _ in range(int(vdeg[v, t])):
                # step 4: layers of the search over type-t edges
                layers = [set(vadj[t][v])]
                seen_c, seen_v = set(layers[0]), {v}
                while len(layers) < depth[t]:
                    nodes = {u for c in layers[-1] for u in cadj[t][c]} - seen_v
                    seen_v |= nodes
                    nxt = {c for u in nodes for c in vadj[t][u]} - seen_c
                    if not nxt:
                        break
                    layers.append(nxt)
                    seen_c |= nxt
                # step 5: the deepest level that leaves a candidate decides;
                # only checks that own type-t sockets can be candidates
                own = owners[t]
                free = cdeg[own, t] - fill[own, t] > 0
                for c in nbrs[v]:
                    if pos[t][c] >= 0:
                        free[pos[t][c]] = False
                chosen = -1
                excluded = set()
                cum = []
                for layer in layers:
                    excluded |= layer
                    cum.append(set(excluded))
                for k in range(len(layers), 0, -1):
                    mask = free.copy()
                    for c in cum[k - 1]:
                        mask[pos[t][c]] = False
                    idx = own[mask]
                    if idx.size:
                        f = fill[idx, t]
                        tied = idx[f == f.min()]  # the least filled, in check order
                        chosen = int(tied[rng.uniform(tied.size)])
                        break
                if chosen < 0:
                    raise ValueError("no check left for an edge of type %d of node %d" % (t, v))
                fill[chosen, t] += 1
                vadj[t][v].append(chosen)
                cadj[t][chosen].append(v)
                nbrs[v].add(chosen)
                ev.append(v)
                ec.append(chosen)
                et.append(t)
    v = np.array(ev, dtype=np.int64)
    c = np.array(ec, dtype=np.int64)
    t = np.array(et, dtype=np.int64)
    if not np.array_equal(np.bincount(c, minlength=m), cdeg.sum(axis=1)):
        raise ValueError("sockets left unfilled")
    order = np.lexsort((v, t, c))
    return Code(n, m, v[order], c[order], t[order], ntypes, tuple(vn_counts), tuple(cn_counts))


def girth_type_subgraph(code: Code, t: int, limit: int = 24) -> int:
    """Length of the shortest cycle (up to `limit`) in the bipartite subgraph of
    type-t edges, by breadth-first search from every variable node; 0 if none
    up to the limit.  Plain and slow: for small codes."""
    sel = code.t == t
    v, c = code.v[sel], code.c[sel]
    n, m = code.n, code.m
    adj = [[] for _ in range(n + m)]  # nodes: VNs 0..n-1, checks n..n+m-1
    for a, b in zip(v.tolist(), c.tolist()):
        adj[a].append(n + b)
        adj[n + b].append(a)
    best = 0
    for s in np.unique(v).tolist():
        dist = {s: 0}
        parent = {s: -1}
        frontier = [s]
        found = 0
        while frontier and not found:
            nxt = []
            for x in frontier:
                for y in adj[x]:
                    if y == parent[x]:
                        continue
                    if y in dist:
                        cyc = dist[x] + dist[y] + 1
                        if cyc <= limit and (found == 0 or cyc < found):
                            found = cyc
                        continue
                    dist[y] = dist[x] + 1
                    parent[y] = x
                    nxt.append(y)
            frontier = nxt
            if frontier and dist[frontier[0]] * 2 > limit:
                break
        if found and (best == 0 or found < best):
            best = found
    return best
