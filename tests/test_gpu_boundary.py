"""GPU tests of the boundary's contract: host ids given by the caller
(Algorithm 1's host_cell_id, the input Sec. 3.2 names for interpolation and
spreading) give the same results as the calls' own search, bit for bit; tree
handles are read-only, so fixed-point spreading on one tree from two streams
at once equals the same work done one call after the other."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import (TOL, as_dtype, fixed_point_quantum, gpu_tree, oracle_tree, spread_excess, to_dev)

pytestmark = pytest.mark.gpu

DTYPES = [torch.float64, torch.float32]


@pytest.fixture(scope="module")
def ot():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2605_20565_amd as m
    return m


@pytest.fixture(scope="module")
def cfg1():
    w = synth.workload(1)
    return w, oracle_tree(w.tree), gpu_tree(w.tree)


def _inputs(w, o, dtype, rng):
    pts = np.concatenate([w.points, rng.random((500, 3)), [[np.nan, 0.5, 0.5]]])
    frc = np.concatenate([w.forces, rng.standard_normal((501, 3))])
    return as_dtype(pts, dtype), as_dtype(frc, dtype), as_dtype(o.permute_rows(w.field), dtype)


@pytest.mark.parametrize("dtype", DTYPES)
def test_given_ids_equal_own_search_bitwise(ot, cfg1, dtype):
    w, o, t = cfg1
    rng = np.random.default_rng(11)
    pts, frc, fld = _inputs(w, o, dtype, rng)
    P, F, U = to_dev(pts, dtype), to_dev(frc, dtype), to_dev(fld, dtype)
    ids = t.locate(P)
    assert np.array_equal(ids.cpu().numpy().astype(np.int64), o.locate(pts))
    g = to_dev(as_dtype(rng.standard_normal(pts.shape), dtype), dtype)
    assert torch.equal(t.interpolate(U, P, ids=ids), t.interpolate(U, P))
    for mode in ("fixed", "atomic"):
        a = t.spread(F, P, mode=mode, ids=ids)
        b = t.spread(F, P, mode=mode)
        if mode == "fixed":
            assert torch.equal(a, b)
        else:
            f, S, cnt, A = o.spread(frc, pts, with_scale=True)
            assert spread_excess(a.cpu().numpy(), f, S, A, cnt, dtype) <= 1.0
    for entry in ("ot_grad_pos", "ot_interp_grad_pos", "ot_spread_grad_pos"):
        assert torch.equal(t.grad_pos(U, g, P, ids=ids, entry=entry), t.grad_pos(U, g, P))
    gf1, gx1 = t.interp_backward(U, g, P, mode="fixed", ids=ids)
    gf2, gx2 = t.interp_backward(U, g, P, mode="fixed")
    assert torch.equal(gf1, gf2) and torch.equal(gx1, gx2)
    gF1, gy1 = t.spread_backward(U, F, P, ids=ids)
    gF2, gy2 = t.spread_backward(U, F, P)
    assert torch.equal(gF1, gF2) and torch.equal(gy1, gy2)


def test_given_ids_out_of_range_mean_no_host(ot, cfg1):
    """-1 and ids outside [0, n_leaves) are points without a host: velocity 0,
    nothing spread (and no out-of-bounds access)."""
    w, o, t = cfg1
    dtype = torch.float64
    pts = as_dtype(w.points[:64], dtype)
    frc = as_dtype(w.forces[:64], dtype)
    P, F = to_dev(pts, dtype), to_dev(frc, dtype)
    U = to_dev(as_dtype(o.permute_rows(w.field), dtype), dtype)
    ids = t.locate(P)
    bad = ids.clone()
    bad[0::4] = -1
    bad[1::4] = t.n_leaves
    bad[2::4] = 2 ** 31 - 1
    vel = t.interpolate(U, P, ids=bad)
    keep = (torch.arange(64, device="cuda") % 4) == 3
    assert torch.all(vel[~keep] == 0)
    assert torch.equal(vel[keep], t.interpolate(U, P)[keep])
    got = t.spread(F, P, mode="fixed", ids=bad)
    want = t.spread(F[keep].contiguous(), P[keep].contiguous(), mode="fixed")
    q = fixed_point_quantum(frc)
    # the scale differs (max |F| over all 64 against the 16 kept), so compare with the oracle bound
    f, S, cnt, A = o.spread(frc[keep.cpu().numpy()], pts[keep.cpu().numpy()], with_scale=True)
    assert spread_excess(got.cpu().numpy(), f, S, A, cnt, dtype, q) <= 1.0
    assert spread_excess(want.cpu().numpy(), f, S, A, cnt, dtype, fixed_point_quantum(frc[keep.cpu().numpy()])) <= 1.0


def test_workspace_argument_and_own_allocation_agree(ot, cfg1):
    w, o, t = cfg1
    dtype = torch.float32
    rng = np.random.default_rng(3)
    pts, frc, _ = _inputs(w, o, dtype, rng)
    P, F = to_dev(pts, dtype), to_dev(frc, dtype)
    work = t.workspace()
    assert work.numel() == t.info().workspace_bytes == t.n_leaves * 24 + 256
    a = t.spread(F, P, mode="fixed", work=work)
    # NULL workspace: the library allocates one on the stream for the call
    out = torch.empty((t.n_leaves, 3), dtype=dtype, device="cuda")
    ot._check(ot.lib.ot_spread(t.handle, ot._ptr(F), ot._ptr(P), None, ot.OT_F32, P.shape[0], ot.OT_SPREAD_FIXED, 0,
                               ot._ptr(out), None, ot._stream()))
    assert torch.equal(a, out)
    with pytest.raises(ValueError):
        t.spread(F, P, mode="fixed", work=work[1:])   # misaligned


@pytest.mark.parametrize("sort", [False, True])
def test_two_fixed_plans_on_one_tree_on_two_streams(ot, cfg1, sort):
    """Each FIXED plan owns its accumulators: two plans replayed on two
    streams at once give exactly what they give one after the other."""
    w, o, t = cfg1
    dtype = torch.float32
    rng = np.random.default_rng(5)
    pts, frc, fld = _inputs(w, o, dtype, rng)
    n = pts.shape[0]
    P, F, U = to_dev(pts, dtype), to_dev(frc, dtype), to_dev(fld, dtype)
    F2 = to_dev(as_dtype(rng.standard_normal(pts.shape), dtype), dtype)
    off = [0, 1000, n]
    plans = [ot.BatchPlan(t, off, [7, 7], dtype=dtype, mode="fixed", sort_points=sort) for _ in range(2)]
    outs = [(torch.empty(n, dtype=torch.int32, device="cuda"), torch.empty_like(P),
             torch.empty((t.n_leaves, 3), dtype=dtype, device="cuda")) for _ in range(2)]
    forces = [F, F2]
    # serial
    ref = []
    for p, (ids, vel, fo), f in zip(plans, outs, forces):
        p.run(P, field=U, force=f, ids=ids, vel=vel, field_out=fo)
        torch.cuda.synchronize()
        ref.append(fo.clone())
    # concurrent, several times (each replay overwrites field_out)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for _ in range(5):
        torch.cuda.synchronize()
        with torch.cuda.stream(s1):
            plans[0].run(P, field=U, force=F, ids=outs[0][0], vel=outs[0][1], field_out=outs[0][2])
        with torch.cuda.stream(s2):
            plans[1].run(P, field=U, force=F2, ids=outs[1][0], vel=outs[1][1], field_out=outs[1][2])
        torch.cuda.synchronize()
        assert torch.equal(outs[0][2], ref[0])
        assert torch.equal(outs[1][2], ref[1])
    # and plain FIXED spreads from two streams with their own workspaces
    with torch.cuda.stream(s1):
        a = t.spread(F, P, mode="fixed")
    with torch.cuda.stream(s2):
        b = t.spread(F2, P, mode="fixed")
    torch.cuda.synchronize()
    assert torch.equal(a, t.spread(F, P, mode="fixed"))
    assert torch.equal(b, t.spread(F2, P, mode="fixed"))
    for p in plans:
        p.close()


def test_sorted_plan_refuses_skipped_instances(ot, cfg1):
    """A sorted plan visits every point with the common ops, so an instance
    with ops = 0 and points cannot be honoured: creation is refused."""
    w, o, t = cfg1
    with pytest.raises(ot.OtError) as e:
        ot.BatchPlan(t, [0, 10, 20, 30], [7, 0, 7], dtype=torch.float32, mode="fixed", sort_points=True)
    assert e.value.code == -1
    # empty skipped instances are fine
    ot.BatchPlan(t, [0, 10, 10, 30], [7, 0, 7], dtype=torch.float32, mode="fixed", sort_points=True).close()


@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
def test_non_finite_force(ot, cfg1, bad):
    """A force with a non-finite component: ATOMIC spreading carries it to the
    leaves that point reaches (the oracle's non-finite leaves, and no others);
    FIXED spreading, whose integer sums cannot carry it, returns NaN
    everywhere, plain and batched (sorted or not)."""
    w, o, t = cfg1
    dtype = torch.float32
    rng = np.random.default_rng(19)
    pts = as_dtype(w.points, dtype)
    frc = as_dtype(w.forces, dtype)
    frc[123, 1] = bad
    P, F = to_dev(pts, dtype), to_dev(frc, dtype)
    a = t.spread(F, P, mode="atomic").cpu().numpy()
    f = o.spread(frc, pts)
    assert np.array_equal(~np.isfinite(a), ~np.isfinite(f))
    assert (~np.isfinite(a)).sum() > 0 and np.isfinite(a).sum() > 0.99 * a.size
    assert torch.isnan(t.spread(F, P, mode="fixed")).all()
    n = P.shape[0]
    for sort in (False, True):
        plan = ot.BatchPlan(t, [0, 1000, n], [7, 7], dtype=dtype, mode="fixed", sort_points=sort)
        fo = torch.zeros((t.n_leaves, 3), dtype=dtype, device="cuda")
        plan.run(P, field=torch.zeros_like(fo), force=F, ids=torch.empty(n, dtype=torch.int32, device="cuda"),
                 vel=torch.empty_like(P), field_out=fo)
        torch.cuda.synchronize()
        assert torch.isnan(fo).all()
        plan.close()
    # and a finite force field afterwards is clean again (the flag is per call)
    frc2 = as_dtype(w.forces, dtype)
    assert torch.isfinite(t.spread(to_dev(frc2, dtype), P, mode="fixed")).all()
