"""Phase I of the migration of Lagrangian points (Algorithm 2) on one device:
relocation of moved points and their owners under a Morton-range partition
(test infrastructure; only the tests and bench.py's oracle leg use it).

- relocate: the host of every point after it moved is by definition the
  result of Algorithm 1 (``Tree.locate``); the points that left their
  previous host are counted.
- find_owner: the leaves are cut into contiguous Morton ranges, one per
  rank (Sec. 3.1, partitioning); rank r owns keys in [split[r], split[r+1]).
  A point's owner is the rank whose range holds the Morton key of its
  finest-level cell, found by a sorted search over the P + 1 splitters;
  points outside a non-periodic domain (or NaN) get -1.
"""
from __future__ import annotations

import numpy as np


def relocate(tree, pos, prev_ids):
    ids = tree.locate(pos)
    moved = int(np.count_nonzero(ids != np.asarray(prev_ids)))
    return ids, moved


def point_keys(pos, L: int, periodic: bool):
    """Morton key (x lowest, a plain bit loop) of floor(x 2^L) per point; -1
    where the point has no cell."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    M = 1 << L
    with np.errstate(invalid="ignore"):
        v = pos * float(M)
        ok = np.all(np.abs(v) < 2.0 ** 52, axis=1)
        c = np.where(np.isfinite(v), np.floor(np.where(np.isfinite(v), v, 0.0)), 0.0).astype(np.int64)
    if periodic:
        c = np.mod(c, M)
    else:
        ok &= np.all((c >= 0) & (c < M), axis=1)
        c = np.where(ok[:, None], c, 0)
    key = np.zeros(pos.shape[0], dtype=np.uint64)
    for b in range(L):
        for d in range(3):
            key |= ((c[:, d] >> b) & 1).astype(np.uint64) << np.uint64(3 * b + d)
    return np.where(ok, key.astype(np.int64), -1)


def leaf_splitters(sorted_keys, P: int, L: int):
    """Equal leaf counts per rank: split[r] = key of leaf floor(r n / P),
    split[P] = 8^L (one past the last key)."""
    n = len(sorted_keys)
    s = [int(sorted_keys[(r * n) // P]) for r in range(P)]
    s[0] = 0
    return np.array(s + [1 << (3 * L)], dtype=np.int64)


def find_owner(splitters, pos, L: int, periodic: bool):
    key = point_keys(pos, L, periodic)
    own = np.searchsorted(np.asarray(splitters[1:-1], dtype=np.int64), key, side="right")
    return np.where(key >= 0, own, -1).astype(np.int64)
