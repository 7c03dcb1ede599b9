"""Pins of the oracle's progressive-edge-growth construction (oracle/peg.py).

* The placement rule against an independent formulation: every edge goes to
  the r-th (r drawn from the stream) of the candidates, in check order, that
  maximise min(d(c), K + 1) and, among those, have the fewest type-t edges; d
  is the graph distance in check layers from the edge's node (scipy's
  breadth-first shortest paths over the whole type-t graph so far).
* Degree histograms and per-check socket counts equal to the random
  construction's (steps 1-4 are shared by specification), no repeated pair.
* Short cycles: far fewer variable nodes on cycles of length <= 2K in the
  searched subgraph than in the random construction.
* The default depths, worked out by hand from the stated rule.
"""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

from met_inputs import PROFILES, Profile
from oracle import code as oc, peg


def test_default_depths_by_hand():
    # r0.1: type 0 d_v = 2, d_c = 12, g = 11: 1 * 11 = 11, 121 <= 1024 < 1331 -> 3
    #       type 1 d_v = 22, d_c = 3, g = 42: 21 * 42 = 882 <= 1024 < 21 * 42^2 -> 2
    #       type 2 d_v = 1: g = 0 -> 1
    assert peg.default_depths(PROFILES["r0.1"]) == [3, 2, 1]
    # r0.05: type 1 d_v = 47, g = 92: 46 * 92 = 4232 > 1024 -> 1
    assert peg.default_depths(PROFILES["r0.05"]) == [3, 1, 1]
    # r0.02: type 0 d_c = 6, g = 5: 5^4 = 625 <= 1024 < 3125 -> 5
    assert peg.default_depths(PROFILES["r0.02"]) == [5, 1, 1]


def _replay_rule(profile, n, seed, depth):
    """Rebuilds the graph edge by edge with the closed-form rule and returns the
    edges in placement order."""
    vn_counts, cn_counts, vdeg, cdeg = peg._socket_degrees(profile, n)
    m = int(sum(cn_counts))
    ntypes = profile.n_edge_types
    rng = oc.edge_type_stream(seed, ntypes)
    fill = np.zeros((m, ntypes), dtype=np.int64)
    edges = []
    for v in range(n):
        for t in range(ntypes):
            for _ in range(int(vdeg[v, t])):
                # bipartite type-t graph so far: VN i -> node i, check j -> node n + j
                tv = [a for a, b, tt in edges if tt == t]
                tc = [n + b for a, b, tt in edges if tt == t]
                g = sp.csr_matrix((np.ones(len(tv)), (tv, tc)), shape=(n + m, n + m))
                dist = shortest_path(g, directed=False, unweighted=True, indices=v)[n:]
                layer = np.full(m, np.inf)  # check layer index; unreachable: inf
                fin = np.isfinite(dist)
                layer[fin] = (dist[fin] + 1) // 2
                score = np.minimum(layer, depth[t] + 1)
                nb = {b for a, b, tt in edges if a == v}
                cand = [c for c in range(m) if fill[c, t] < cdeg[c, t] and c not in nb]
                top = max((score[c], -fill[c, t]) for c in cand)
                tied = [c for c in cand if (score[c], -fill[c, t]) == top]
                best = tied[rng.uniform(len(tied))]
                fill[best, t] += 1
                edges.append((v, best, t))
    return edges


@pytest.mark.parametrize("depth", [[2, 2, 1], [4, 1, 1], [1, 1, 1]])
def test_placement_rule_matches_closed_form(depth):
    # a small MET profile of the same shape: 25 % nodes of degree 2 + 9, leaves
    prof = Profile("small", 0.1, vn_types=((0.25, (2, 9, 0)), (0.75, (0, 0, 1))),
                   cn_types=((0.0833, (6, 0, 0)), (0.75, (0, 3, 1))))
    n, seed = 400, 9
    code = peg.build(prof, n, seed, depth)
    ref = _replay_rule(prof, n, seed, depth)
    rv, rc, rt = (np.array(x, dtype=np.int64) for x in zip(*ref))
    order = np.lexsort((rv, rt, rc))
    np.testing.assert_array_equal(code.v, rv[order])
    np.testing.assert_array_equal(code.c, rc[order])
    np.testing.assert_array_equal(code.t, rt[order])


@pytest.mark.parametrize("name", list(PROFILES))
def test_degrees_sockets_and_no_repeated_pairs(name):
    prof = PROFILES[name]
    n = 4096
    code = peg.build(prof, n, 5)
    rnd = oc.build(prof, n, 5)
    assert code.m == rnd.m and code.e == rnd.e
    np.testing.assert_array_equal(code.vn_degree(), rnd.vn_degree())
    for t in range(prof.n_edge_types):
        np.testing.assert_array_equal(np.bincount(code.c[code.t == t], minlength=code.m),
                                      np.bincount(rnd.c[rnd.t == t], minlength=rnd.m))
        np.testing.assert_array_equal(np.bincount(code.v[code.t == t], minlength=code.n),
                                      np.bincount(rnd.v[rnd.t == t], minlength=rnd.n))
    keys = code.v * code.m + code.c
    assert np.unique(keys).size == keys.size
    # deterministic, and the seed matters
    again = peg.build(prof, n, 5)
    np.testing.assert_array_equal(again.v, code.v)
    other = peg.build(prof, n, 6)
    assert not np.array_equal(other.v, code.v)


def _on_short_cycle(code, t, length):
    """VNs of the type-t subgraph that lie on a cycle of length <= `length`:
    for each VN, a search from each of its type-t checks in the graph without
    the VN must reach another of its checks within length - 2 steps."""
    sel = code.t == t
    v, c = code.v[sel], code.c[sel]
    n = code.n
    adj = {}
    for a, b in zip(v.tolist(), c.tolist()):
        adj.setdefault(a, []).append(n + b)
        adj.setdefault(n + b, []).append(a)
    out = set()
    for x in np.unique(v).tolist():
        mine = adj[x]
        for s in mine:
            targets = set(mine) - {s}
            seen, frontier, steps = {s, x}, [s], 0
            hit = False
            while frontier and steps < length - 2 and not hit:
                steps += 1
                nxt = []
                for y in frontier:
                    for z in adj[y]:
                        if z in seen:
                            continue
                        if z in targets:
                            hit = True
                        seen.add(z)
                        nxt.append(z)
                frontier = nxt
            if hit:
                out.add(x)
                break
    return out


def test_fewer_short_cycles_than_random():
    prof = PROFILES["r0.1"]
    n = 8192
    depth = peg.default_depths(prof)
    p = peg.build(prof, n, 3)
    r = oc.build(prof, n, 3)
    # type 0 searched to 3 layers: no cycles of length <= 6 where avoidable
    on_p = _on_short_cycle(p, 0, 2 * depth[0])
    on_r = _on_short_cycle(r, 0, 2 * depth[0])
    n2 = int(np.count_nonzero(p.vn_degree() > 1))
    print("type-0 VNs on cycles <= %d: PEG %d, random %d of %d" % (2 * depth[0], len(on_p), len(on_r), n2))
    assert len(on_r) > 0.2 * n2
    assert len(on_p) < 0.2 * len(on_r)
    # 4-cycles through type-1 edges
    on_p1 = _on_short_cycle(p, 1, 4)
    on_r1 = _on_short_cycle(r, 1, 4)
    print("type-1 VNs on 4-cycles: PEG %d, random %d" % (len(on_p1), len(on_r1)))
    assert len(on_p1) < 0.1 * max(len(on_r1), 1)
