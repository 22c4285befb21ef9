"""Autotuner: candidate generation, signatures and the JSON cache (CPU),
and a tuned plan that reproduces the default plan's results (GPU)."""
import os

import numpy as np
import pytest
import torch


class _FakeTree:
    n_leaves, l_min, l_max, periodic = 1000, 2, 5, True


@pytest.fixture(scope="module")
def tune():
    from paper_2605_20565_amd import tune as t
    return t


def test_candidates_cover_shapes_and_sorting(tune):
    c = tune.default_candidates(10 ** 6)
    assert {x.block for x in c} == {256, 512}
    assert all(x.tile % x.block == 0 for x in c)
    assert {x.sort_points for x in c} == {True, False}
    assert all(not x.sort_points for x in tune.default_candidates(10 ** 6, uniform_ops=False))
    small = tune.default_candidates(300)
    assert all(x.tile <= max(x.block, 300) for x in small)


def test_signature_depends_on_the_workload(tune):
    s1 = tune.signature(_FakeTree, [0, 10, 20], [7, 7], torch.float32, "fixed")
    assert s1 == tune.signature(_FakeTree, [0, 10, 20], [7, 7], torch.float32, "fixed")
    assert s1 != tune.signature(_FakeTree, [0, 10, 21], [7, 7], torch.float32, "fixed")
    assert s1 != tune.signature(_FakeTree, [0, 10, 20], [7, 3], torch.float32, "fixed")
    assert s1 != tune.signature(_FakeTree, [0, 10, 20], [7, 7], torch.float64, "fixed")
    assert s1 != tune.signature(_FakeTree, [0, 10, 20], [7, 7], torch.float32, "atomic")


def test_cache_round_trip(tune, tmp_path):
    p = str(tmp_path / "sub" / "tune.json")
    assert tune.load_cache(p) == {}
    tune.store_cache(p, "k1", {"best": {"block": 256, "tile": 1024, "grid": 0, "sort_points": True}, "ms": 1.0})
    tune.store_cache(p, "k2", {"best": {"block": 512, "tile": 2048, "grid": 0, "sort_points": False}, "ms": 2.0})
    d = tune.load_cache(p)
    assert set(d) == {"k1", "k2"} and d["k2"]["best"]["tile"] == 2048
    with open(p, "w") as f:
        f.write("not json")
    assert tune.load_cache(p) == {}


@pytest.mark.gpu
def test_tuned_plan_reproduces_default(tune, tmp_path):
    import synth
    import paper_2605_20565_amd as ot
    from gpu_util import gpu_tree, to_dev
    w = synth.workload(1)
    t = gpu_tree(w.tree)
    P = to_dev(w.points, torch.float32)
    F = to_dev(w.forces, torch.float32)
    Fd = t.permute_rows(to_dev(w.field, torch.float32))
    off = [int(v) for v in w.instances]
    ops = [7] * (len(off) - 1)
    cache = str(tmp_path / "tune.json")
    best, timings = tune.tune(t, off, ops, P, Fd, F, torch.float32, "fixed", reps=2, cache_path=cache)
    assert len(timings) >= 6 and os.path.exists(cache)
    again, _ = tune.tune(t, off, ops, P, Fd, F, torch.float32, "fixed", reps=2, cache_path=cache)
    assert again == best
    n = P.shape[0]
    outs = []
    for cand in (best, tune.Candidate(256, 1024, 0, False)):
        plan = ot.BatchPlan(t, off, ops, dtype=torch.float32, mode="fixed", block=cand.block, tile=cand.tile,
                            grid=cand.grid, sort_points=cand.sort_points)
        ids = torch.empty(n, dtype=torch.int32, device="cuda")
        vel = torch.empty((n, 3), device="cuda")
        fo = torch.empty((t.n_leaves, 3), device="cuda")
        plan.run(P, field=Fd, force=F, ids=ids, vel=vel, field_out=fo)
        torch.cuda.synchronize()
        outs.append((ids, vel, fo))
        plan.close()
    for a, b in zip(*outs):
        assert torch.equal(a, b)
