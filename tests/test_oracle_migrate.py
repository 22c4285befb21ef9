"""Pins of the oracle's migration phase I (Algorithm 2): the owner found from
a point's Morton key must be the rank that owns the point's host leaf, the
leaf Algorithm 1 finds (ranks own contiguous ranges of leaf ids, Sec. 3.1);
a hand case checks the bit order of the key; relocation counts the points
whose host changed.
"""
import numpy as np
import pytest

import synth
from oracle import migrate


def _tree(orc, spec):
    return orc.Tree.from_anchors(spec.anchors, spec.levels, spec.l_min, spec.l_max, spec.periodic)


@pytest.mark.parametrize("seed,P", [(0, 2), (1, 3), (2, 8), (3, 5)])
def test_key_owner_is_host_leaf_owner(orc, seed, P):
    rng = np.random.default_rng(seed)
    spec = synth.random_tree(2, 5, rng, periodic=bool(seed % 2))
    t = _tree(orc, spec)
    pos = rng.random((3000, 3)) * 1.2 - 0.1
    ids = t.locate(pos)
    split = migrate.leaf_splitters(t.keys, P, spec.l_max)
    own = migrate.find_owner(split, pos, spec.l_max, spec.periodic)
    first = np.array([(r * t.n_leaves) // P for r in range(P)] + [t.n_leaves])
    by_id = np.searchsorted(first[1:-1], ids, side="right")
    assert np.array_equal(own, np.where(ids >= 0, by_id, -1))


def test_owner_hand_case():
    # level-1 cells: key bits (z y x); two ranks split at key 4 = the z >= 1/2 half
    split = np.array([0, 4, 8])
    pos = np.array([[0.2, 0.9, 0.4], [0.7, 0.1, 0.6], [0.9, 0.9, 0.49], [0.0, 0.0, 0.5]])
    assert list(migrate.find_owner(split, pos, 1, True)) == [0, 1, 0, 1]
    assert list(migrate.point_keys(pos, 1, True)) == [2, 5, 3, 4]


def test_relocate_counts_movers(orc):
    spec = synth.uniform_tree(3, seed=2)
    t = _tree(orc, spec)
    rng = np.random.default_rng(8)
    pos = rng.random((500, 3))
    prev = t.locate(pos)
    new_pos = np.mod(pos + rng.normal(scale=0.05, size=pos.shape), 1.0)
    ids, moved = migrate.relocate(t, new_pos, prev)
    assert np.array_equal(ids, t.locate(new_pos))
    # a point keeps its host iff its level-3 cell is unchanged on this uniform tree
    same = np.all(np.floor(pos * 8) == np.floor(new_pos * 8), axis=1)
    assert moved == int((~same).sum())
