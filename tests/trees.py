"""Random tree-shaped Tanner graphs for exact-inference pins (test helper).

A factor graph that is a tree makes sum-product BP exact: after as many
iterations as the diameter, BP posteriors equal the bitwise MAP posteriors.
The generator grows a tree from one variable node by repeatedly picking an
existing variable node and hanging a new check with one or two new variable
nodes under it, so every check has degree 2 or 3 and leaves are degree-1
variable nodes.  Edge types are drawn from {0, 1, 2} to exercise typed paths.
"""
from __future__ import annotations

import numpy as np


def random_tree(n_vn: int, rng: np.random.Generator):
    """Returns (n, m, v, c, t) edge arrays of a tree with exactly n_vn VNs."""
    v, c, t = [], [], []
    n, m = 1, 0
    while n < n_vn:
        anchor = int(rng.integers(0, n))
        k = 1 if n + 1 == n_vn else int(rng.integers(1, 3))
        chk = m
        m += 1
        v.append(anchor)
        c.append(chk)
        t.append(int(rng.integers(0, 3)))
        for _ in range(k):
            v.append(n)
            c.append(chk)
            t.append(int(rng.integers(0, 3)))
            n += 1
    return n, m, np.array(v), np.array(c), np.array(t)
