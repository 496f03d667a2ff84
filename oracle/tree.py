"""Cluster tree of section 3.1 (oracle; test infrastructure only).

The root owns all indices.  A node with index range [a, b) is split into the
first ceil((b - a) / 2) indices and the rest; splitting continues level by
level until every node of the newest level has at most ``leaf_max`` indices.
The tree is fully populated: all leaves sit at depth L.  Indices are 0-based
and half-open here, whereas the paper counts from 1.
"""
from __future__ import annotations


def cluster_tree(n: int, leaf_max: int) -> list:
    """Return ``levels`` with ``levels[l]`` the list of (start, stop) ranges of
    the 2**l nodes on level l, left to right (section 3.1).

    The stopping rule reads "below the threshold" as size <= leaf_max, so that
    N = 1024 with threshold 32 gives 32 leaves of 32.
    """
    if n < 1 or leaf_max < 1:
        raise ValueError("need n >= 1 and leaf_max >= 1")
    levels = [[(0, n)]]
    while max(b - a for a, b in levels[-1]) > leaf_max:
        nxt = []
        for a, b in levels[-1]:
            half = -(-(b - a) // 2)  # ceil((b - a) / 2)
            nxt.append((a, a + half))
            nxt.append((a + half, b))
        if any(b <= a for a, b in nxt):
            raise ValueError("tree would contain an empty node")
        levels.append(nxt)
    return levels


def depth(levels: list) -> int:
    """L, the depth of the tree (level of the leaves)."""
    return len(levels) - 1


def leaf_sizes(levels: list) -> list:
    return [b - a for a, b in levels[-1]]
