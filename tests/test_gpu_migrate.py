"""GPU migration phase I (ot_relocate, ot_leaf_splitters, ot_find_owner)
against the oracle (oracle/migrate.py): ids, splitters, owners and counts are
integer results and must match bit for bit."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import as_dtype, gpu_tree, oracle_tree, to_dev
from oracle import migrate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ot():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2605_20565_amd as m
    return m


def _specs():
    rng = np.random.default_rng(21)
    return {"random_periodic": synth.random_tree(2, 6, rng, periodic=True),
            "random_walls": synth.random_tree(2, 6, rng, periodic=False),
            "band": synth.workload(1).tree}


@pytest.mark.parametrize("name", ["random_periodic", "random_walls", "band"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_relocate_matches_locate(ot, name, dtype):
    spec = _specs()[name]
    o, t = oracle_tree(spec), gpu_tree(spec)
    rng = np.random.default_rng(5)
    pos = as_dtype(rng.random((20000, 3)), dtype)
    prev = o.locate(pos)
    step = rng.normal(scale=0.4 / (1 << spec.l_max), size=pos.shape)     # mostly under a cell
    new = pos + step
    if spec.periodic:
        new = np.mod(new, 1.0)
    new = as_dtype(new, dtype)
    want, moved = migrate.relocate(o, new, prev)
    ids = torch.from_numpy(prev.astype(np.int32)).cuda()
    got_moved = t.relocate(to_dev(new, dtype), ids)
    assert np.array_equal(ids.cpu().numpy(), want)
    assert got_moved == moved
    assert 0 < moved < len(pos)


@pytest.mark.parametrize("name", ["random_periodic", "random_walls", "band"])
@pytest.mark.parametrize("P", [1, 3, 8, 64])
def test_owners_match_oracle(ot, name, P):
    spec = _specs()[name]
    o, t = oracle_tree(spec), gpu_tree(spec)
    split = t.leaf_splitters(P)
    want_split = migrate.leaf_splitters(o.keys, P, spec.l_max)
    assert np.array_equal(split.cpu().numpy(), want_split)
    rng = np.random.default_rng(P)
    pos = rng.random((30000, 3)) * 1.1 - 0.05
    own, cnt = t.find_owner(split, to_dev(pos, torch.float64))
    want = migrate.find_owner(want_split, pos, spec.l_max, spec.periodic)
    assert np.array_equal(own.cpu().numpy(), want)
    assert np.array_equal(cnt.cpu().numpy(), np.bincount(want[want >= 0], minlength=P))
