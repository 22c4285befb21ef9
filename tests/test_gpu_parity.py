"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Host ids and sorted leaf order must match bit for bit; interpolated
velocities, spread forces and position gradients must match within the
stated tolerance on the magnitude-scaled metric (FP64 1e-12, FP32 1e-5),
measured per component against sum |w| |u| (interpolate, gradient) or per leaf
against sum |w F| (spread; FIXED mode adds its stated quantisation bound of
2^-(s+1) per contribution).
"""
import math

import numpy as np
import pytest
import torch

import synth
from gpu_util import (TOL, as_dtype, fixed_point_quantum, gpu_tree, oracle_tree, scaled_err, spread_excess,
                      to_dev)

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
    return w, oracle_tree(w.tree)


@pytest.fixture(scope="module")
def cfg1_gpu(ot, cfg1):
    w, _ = cfg1
    return gpu_tree(w.tree)


def _extra_points(rng, l_max, n=2000):
    """Points on dyadic faces/edges/corners of the finest level, 0, 1-ulp,
    exactly 1.0 and slightly outside the cube (wrapped when periodic)."""
    g = rng.integers(0, 1 << l_max, (n, 3)) * math.ldexp(1.0, -l_max)
    mix = rng.random((n, 3))
    m = rng.random((n, 3)) < 0.5
    mix[m] = g[m]
    edge = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0], [np.nextafter(1.0, 0.0)] * 3, [0.5, 0.5, 0.5],
                     [-1e-9, 0.5, 0.5], [1.0 + 1e-9, 0.25, 0.75], [-0.25, 1.5, 2.0]])
    return np.concatenate([g, mix, edge])


# ---------------------------------------------------------------------------
# Tree build
# ---------------------------------------------------------------------------
def test_encode_keys_bitexact(ot):
    import oracle
    rng = np.random.default_rng(1)
    for L in (1, 7, 10, 21):
        a = rng.integers(0, 1 << L, (5000, 3)).astype(np.uint32)
        got = ot.encode_keys(torch.from_numpy(a.astype(np.int32)).cuda(), L).cpu().numpy().view(np.uint64)
        assert np.array_equal(got, oracle.encode_keys(a, L))


@pytest.mark.parametrize("which", ["cfg1", "rand_a", "rand_b", "deep", "lmin6"])
def test_build_tree_order_and_perm(ot, which):
    rng = np.random.default_rng(7)
    if which == "cfg1":
        spec = synth.workload(1).tree
    elif which == "rand_a":
        spec = synth.random_tree(1, 4, rng, 0.35)
    elif which == "rand_b":
        spec = synth.random_tree(0, 5, rng, 0.3, periodic=False, balance=False)
    elif which == "deep":   # more than 3 levels below the root: several table levels
        spec = synth.band_tree(2, 9, [synth.Sphere((0.3, 0.6, 0.5), 0.2)], seed=3)
    else:                   # 262k base cells, 4 refined levels
        spec = synth.band_tree(6, 10, [synth.Sphere((0.5, 0.5, 0.5), 0.05)], seed=4)
    t = gpu_tree(spec)
    o = oracle_tree(spec)
    keys, lv = t.leaves()
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), o.keys)
    assert np.array_equal(lv.cpu().numpy(), o.levels)
    assert np.array_equal(t.perm.cpu().numpy().astype(np.int64), o.perm)
    inf = t.info()
    assert inf.n_leaves == spec.n_leaves and inf.table_levels >= 1


def test_build_tree_capacity_is_checked_before_any_work(ot):
    """2^26 leaves is the id field's capacity; a complete tree with l_min = 9
    already has 8^9 leaves, so it is refused up front."""
    spec_n = 8 ** 9
    K = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(ot.OtError) as e:
        import ctypes
        h = ctypes.c_void_p()
        desc = ot.TreeDesc(9, 10, 1)
        ot._check(ot.lib.ot_build_tree(ot._ptr(K), ot._ptr(K), spec_n, ctypes.byref(desc), None, None,
                                       ctypes.byref(h)))
    assert e.value.code == -7


def test_build_tree_rejects_bad_partitions(ot):
    import oracle
    spec = synth.random_tree(1, 3, np.random.default_rng(9), 0.4)
    keys = oracle.encode_keys(spec.anchors, 3)
    K = lambda k: torch.from_numpy(k.view(np.int64).copy()).cuda()
    V = lambda v: torch.from_numpy(v.copy()).cuda()
    with pytest.raises(ot.OtError) as e:
        ot.Tree(K(keys[1:]), V(spec.levels[1:]), 1, 3)
    assert e.value.code == -2
    with pytest.raises(ot.OtError) as e:
        ot.Tree(K(np.append(keys, keys[3])), V(np.append(spec.levels, spec.levels[3])), 1, 3)
    assert e.value.code == -3
    lv = spec.levels.copy()
    lv[0] = 5
    with pytest.raises(ot.OtError) as e:
        ot.Tree(K(keys), V(lv), 1, 3)
    assert e.value.code == -4
    with pytest.raises(ot.OtError) as e:
        ot.Tree(K(keys), V(spec.levels), 1, 22)
    assert e.value.code == -4
    # the library still works after the failures
    t = ot.Tree(K(keys), V(spec.levels), 1, 3)
    assert t.n_leaves == spec.n_leaves


# ---------------------------------------------------------------------------
# Host-cell search
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", DTYPES)
def test_locate_bitexact_cfg1(ot, cfg1, cfg1_gpu, dtype):
    w, o = cfg1
    rng = np.random.default_rng(11)
    pts = as_dtype(np.concatenate([w.points, _extra_points(rng, 6)]), dtype)
    ids = cfg1_gpu.locate(to_dev(pts, dtype)).cpu().numpy()
    assert np.array_equal(ids.astype(np.int64), o.locate(pts))


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("dtype", DTYPES)
def test_locate_bitexact_random_trees(ot, seed, dtype):
    rng = np.random.default_rng(200 + seed)
    l_min = int(rng.integers(0, 3))
    l_max = l_min + int(rng.integers(1, 5))
    spec = synth.random_tree(l_min, l_max, rng, 0.3, periodic=bool(seed % 2), balance=seed < 2)
    t, o = gpu_tree(spec), oracle_tree(spec)
    pts = as_dtype(np.concatenate([rng.random((3000, 3)), _extra_points(rng, l_max)]), dtype)
    ids = t.locate(to_dev(pts, dtype)).cpu().numpy().astype(np.int64)
    assert np.array_equal(ids, o.locate(pts))
    if not spec.periodic:
        assert (ids == -1).any()


def test_locate_nan_and_huge(ot, cfg1_gpu, cfg1):
    _, o = cfg1
    pts = np.array([[np.nan, 0.1, 0.1], [0.1, np.inf, 0.2], [1e300, 0.5, 0.5], [-1e300, 0.5, 0.5],
                    [0.3, 0.3, 0.3]])
    ids = cfg1_gpu.locate(to_dev(pts, torch.float64)).cpu().numpy()
    assert list(ids[:4]) == [-1, -1, -1, -1]
    assert ids[4] == o.locate(pts[4:])[0]


# ---------------------------------------------------------------------------
# Interpolation / spreading / fused pass
# ---------------------------------------------------------------------------
def _inputs(w, o, dtype, extra=True):
    rng = np.random.default_rng(5)
    pts = w.points if not extra else np.concatenate([w.points, _extra_points(rng, w.tree.l_max, 500)])
    frc = np.concatenate([w.forces, rng.standard_normal((pts.shape[0] - w.forces.shape[0], 3))])
    pts, frc = as_dtype(pts, dtype), as_dtype(frc, dtype)
    fld = as_dtype(o.permute_rows(w.field), dtype)
    return pts, frc, fld


@pytest.mark.parametrize("dtype", DTYPES)
def test_interpolate_parity_cfg1(ot, cfg1, cfg1_gpu, dtype):
    w, o = cfg1
    pts, _, fld = _inputs(w, o, dtype)
    U, S = o.interpolate(fld, pts, with_scale=True)
    got = cfg1_gpu.interpolate(to_dev(fld, dtype), to_dev(pts, dtype)).cpu().numpy()
    assert scaled_err(got, U, S) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_spread_atomic_parity_cfg1(ot, cfg1, cfg1_gpu, dtype):
    w, o = cfg1
    pts, frc, _ = _inputs(w, o, dtype)
    f, S, cnt, A = o.spread(frc, pts, with_scale=True)
    got = cfg1_gpu.spread(to_dev(frc, dtype), to_dev(pts, dtype), mode="atomic").cpu().numpy()
    assert spread_excess(got, f, S, A, cnt, dtype) <= 1.0


@pytest.mark.parametrize("dtype", DTYPES)
def test_spread_fixed_parity_cfg1(ot, cfg1, cfg1_gpu, dtype):
    w, o = cfg1
    pts, frc, _ = _inputs(w, o, dtype)
    f, S, cnt, A = o.spread(frc, pts, with_scale=True)
    got = cfg1_gpu.spread(to_dev(frc, dtype), to_dev(pts, dtype), mode="fixed").cpu().numpy()
    # the quantisation term dominates in FP64; FP32 adds its own rounding
    assert spread_excess(got, f, S, A, cnt, dtype, fixed_point_quantum(frc)) <= 1.0


def test_fixed_point_is_bitwise_reproducible(ot, cfg1, cfg1_gpu):
    w, o = cfg1
    pts, frc, _ = _inputs(w, o, torch.float32)
    P, F = to_dev(pts, torch.float32), to_dev(frc, torch.float32)
    ref = cfg1_gpu.spread(F, P, mode="fixed")
    perm = torch.randperm(P.shape[0], device=P.device)
    for r in range(5):
        a = cfg1_gpu.spread(F, P, mode="fixed")
        assert torch.equal(a, ref)
    # and independent of point order
    b = cfg1_gpu.spread(F[perm].contiguous(), P[perm].contiguous(), mode="fixed")
    assert torch.equal(b, ref)


@pytest.mark.parametrize("dtype", DTYPES)
def test_spread_accumulate_adds(ot, cfg1, cfg1_gpu, dtype):
    w, o = cfg1
    pts, frc, fld = _inputs(w, o, dtype)
    P, F = to_dev(pts, dtype), to_dev(frc, dtype)
    base = to_dev(fld, dtype)
    for mode in ("atomic", "fixed"):
        one = cfg1_gpu.spread(F, P, mode=mode)
        acc = cfg1_gpu.spread(F, P, mode=mode, out=base.clone(), accumulate=True)
        assert torch.allclose(acc, base + one, rtol=0, atol=1e-5 if dtype == torch.float32 else 1e-12)


@pytest.mark.parametrize("dtype", DTYPES)
def test_track_fused_matches_separate_ops(ot, cfg1, cfg1_gpu, dtype):
    w, o = cfg1
    pts, frc, fld = _inputs(w, o, dtype)
    P, F, Fd = to_dev(pts, dtype), to_dev(frc, dtype), to_dev(fld, dtype)
    ids, vel, fo = cfg1_gpu.track(P, field=Fd, force=F, mode="fixed")
    assert torch.equal(ids, cfg1_gpu.locate(P))
    assert torch.equal(vel, cfg1_gpu.interpolate(Fd, P))
    assert torch.equal(fo, cfg1_gpu.spread(F, P, mode="fixed"))
    U, S = o.interpolate(fld, pts, with_scale=True)
    assert scaled_err(vel.cpu().numpy(), U, S) <= TOL[dtype]
    assert np.array_equal(ids.cpu().numpy().astype(np.int64), o.locate(pts))


@pytest.mark.parametrize("dtype", DTYPES)
def test_nonperiodic_and_deep_tree_parity(ot, dtype):
    """Non-periodic walls (nodes dropped) and a 7-level tree (3 table levels)."""
    spec = synth.band_tree(2, 9, [synth.Sphere((0.3, 0.6, 0.5), 0.2), synth.Sphere((0.8, 0.2, 0.15), 0.1)],
                           periodic=False, seed=5)
    t, o = gpu_tree(spec), oracle_tree(spec)
    rng = np.random.default_rng(6)
    s = synth.Sphere((0.3, 0.6, 0.5), 0.2)
    pts = as_dtype(np.concatenate([synth.fibonacci_sphere(s, 3000, wrap=False), rng.random((3000, 3)),
                                   _extra_points(rng, 9, 300)]), dtype)
    frc = as_dtype(rng.standard_normal(pts.shape), dtype)
    fld = as_dtype(rng.standard_normal((spec.n_leaves, 3)), dtype)
    ids, vel, fo = t.track(to_dev(pts, dtype), field=to_dev(fld, dtype), force=to_dev(frc, dtype), mode="atomic")
    assert np.array_equal(ids.cpu().numpy().astype(np.int64), o.locate(pts))
    U, S = o.interpolate(fld, pts, with_scale=True)
    assert scaled_err(vel.cpu().numpy(), U, S) <= TOL[dtype]
    f, Sf, cnt, A = o.spread(frc, pts, with_scale=True)
    assert spread_excess(fo.cpu().numpy(), f, Sf, A, cnt, dtype) <= 1.0


def test_empty_input(ot, cfg1_gpu):
    P = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    assert cfg1_gpu.locate(P).numel() == 0
    fo = cfg1_gpu.spread(P, P, mode="fixed")
    assert torch.count_nonzero(fo) == 0
    fo = cfg1_gpu.spread(P, P, mode="atomic")
    assert torch.count_nonzero(fo) == 0


def test_single_leaf_tree(ot):
    spec = synth.uniform_tree(0, seed=None)
    t, o = gpu_tree(spec), oracle_tree(spec)
    pts = np.random.default_rng(3).random((100, 3))
    fld = np.array([[1.0, 2.0, 3.0]])
    ids, vel, fo = t.track(to_dev(pts, torch.float64), field=to_dev(fld, torch.float64),
                           force=to_dev(np.ones_like(pts), torch.float64))
    assert (ids.cpu().numpy() == 0).all()
    assert np.allclose(vel.cpu().numpy(), o.interpolate(fld, pts), rtol=0, atol=1e-14)
    assert np.allclose(fo.cpu().numpy(), o.spread(np.ones_like(pts), pts), rtol=1e-14)


# ---------------------------------------------------------------------------
# Position gradient
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", DTYPES)
def test_grad_pos_parity_cfg1(ot, cfg1, cfg1_gpu, dtype):
    w, o = cfg1
    pts, frc, fld = _inputs(w, o, dtype)
    g, S = o.grad_pos(fld, frc, pts, with_scale=True)
    got = cfg1_gpu.grad_pos(to_dev(fld, dtype), to_dev(frc, dtype), to_dev(pts, dtype)).cpu().numpy()
    assert scaled_err(got, g, S) <= TOL[dtype]


@pytest.mark.parametrize("dtype", DTYPES)
def test_interp_backward_one_pass_cfg1(ot, cfg1, cfg1_gpu, dtype):
    """Backward of interpolation in one pass: the field's gradient is the
    spreading of the upstream gradient, the positions' the phi' contraction.
    The per-point arithmetic is that of the separate passes (FIXED spreading
    is order independent), so both outputs match them bit for bit."""
    w, o = cfg1
    pts, g, fld = _inputs(w, o, dtype)
    P, G, Fd = to_dev(pts, dtype), to_dev(g, dtype), to_dev(fld, dtype)
    gf, gx = cfg1_gpu.interp_backward(Fd, G, P, mode="fixed")
    assert torch.equal(gf, cfg1_gpu.spread(G, P, mode="fixed"))
    assert torch.equal(gx, cfg1_gpu.grad_pos(Fd, G, P))
    want, S = o.grad_pos(fld, g, pts, with_scale=True)
    assert scaled_err(gx.cpu().numpy(), want, S) <= TOL[dtype]
    f, Sf, cnt, A = o.spread(g, pts, with_scale=True)
    assert spread_excess(gf.cpu().numpy(), f, Sf, A, cnt, dtype, fixed_point_quantum(g)) <= 1.0
    # one output at a time, and accumulation into the field's gradient
    gf1, none = cfg1_gpu.interp_backward(Fd, G, P, mode="fixed", need_pos=False)
    assert none is None and torch.equal(gf1, gf)
    none, gx1 = cfg1_gpu.interp_backward(Fd, G, P, need_field=False)
    assert none is None and torch.equal(gx1, gx)
    acc = gf.clone()
    cfg1_gpu.interp_backward(Fd, G, P, mode="fixed", need_pos=False, accumulate=True, grad_field=acc)
    assert torch.equal(acc, 2 * gf)


@pytest.mark.parametrize("dtype", DTYPES)
def test_spread_backward_one_pass_cfg1(ot, cfg1, cfg1_gpu, dtype):
    """Backward of spreading in one pass: the forces' gradient is the
    interpolation of the field's gradient, the positions' the phi'
    contraction with the forces."""
    w, o = cfg1
    pts, frc, _ = _inputs(w, o, dtype)
    gfield = as_dtype(np.random.default_rng(8).standard_normal((o.n_leaves, 3)), dtype)
    P, F, Gf = to_dev(pts, dtype), to_dev(frc, dtype), to_dev(gfield, dtype)
    gF, gx = cfg1_gpu.spread_backward(Gf, F, P)
    assert torch.equal(gF, cfg1_gpu.interpolate(Gf, P))
    assert torch.equal(gx, cfg1_gpu.grad_pos(Gf, F, P))
    U, S = o.interpolate(gfield, pts, with_scale=True)
    assert scaled_err(gF.cpu().numpy(), U, S) <= TOL[dtype]
    want, S = o.grad_pos(gfield, frc, pts, with_scale=True)
    assert scaled_err(gx.cpu().numpy(), want, S) <= TOL[dtype]
    gF1, none = cfg1_gpu.spread_backward(Gf, F, P, need_pos=False)
    assert none is None and torch.equal(gF1, gF)


@pytest.mark.parametrize("dtype", DTYPES)
def test_backward_one_pass_nonperiodic(ot, dtype):
    """Both backward passes with walls (nodes outside dropped) on a deep tree."""
    spec = synth.band_tree(2, 9, [synth.Sphere((0.3, 0.6, 0.5), 0.2), synth.Sphere((0.8, 0.2, 0.15), 0.1)],
                           periodic=False, seed=5)
    t, o = gpu_tree(spec), oracle_tree(spec)
    rng = np.random.default_rng(9)
    pts = as_dtype(np.concatenate([synth.fibonacci_sphere(synth.Sphere((0.3, 0.6, 0.5), 0.2), 3000, wrap=False),
                                   rng.random((3000, 3)), _extra_points(rng, 9, 300)]), dtype)
    g = as_dtype(rng.standard_normal(pts.shape), dtype)
    fld = as_dtype(rng.standard_normal((spec.n_leaves, 3)), dtype)
    P, G, Fd = to_dev(pts, dtype), to_dev(g, dtype), to_dev(fld, dtype)
    gf, gx = t.interp_backward(Fd, G, P, mode="atomic")
    f, Sf, cnt, A = o.spread(g, pts, with_scale=True)
    assert spread_excess(gf.cpu().numpy(), f, Sf, A, cnt, dtype) <= 1.0
    want, S = o.grad_pos(fld, g, pts, with_scale=True)
    assert scaled_err(gx.cpu().numpy(), want, S) <= TOL[dtype]
    gF, gx2 = t.spread_backward(Fd, G, P)     # the same contraction: field with the vectors G
    assert torch.equal(gx2, gx)
    U, S = o.interpolate(fld, pts, with_scale=True)
    assert scaled_err(gF.cpu().numpy(), U, S) <= TOL[dtype]


def test_backward_empty_input(ot, cfg1_gpu):
    P = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    Fd = torch.ones((cfg1_gpu.n_leaves, 3), dtype=torch.float32, device="cuda")
    gf, gx = cfg1_gpu.interp_backward(Fd, P, P, mode="fixed")
    assert torch.count_nonzero(gf) == 0 and gx.numel() == 0
    gF, gx = cfg1_gpu.spread_backward(Fd, P, P)
    assert gF.numel() == 0 and gx.numel() == 0


# ---------------------------------------------------------------------------
# Batched persistent pass
# ---------------------------------------------------------------------------
def _batch_case(w):
    """Instances of the cfg1 workload (one marker set, particles split into
    uneven groups) with mixed per-instance ops."""
    off = [0, 1000, 1500, 1507, 4000, 11000]
    ops = [7, 3, 1, 7, 6]
    return off, ops


@pytest.mark.parametrize("dtype", DTYPES)
def test_batch_matches_plain_launches(ot, cfg1, cfg1_gpu, dtype):
    w, o = cfg1
    off, ops = _batch_case(w)
    pts, frc, fld = _inputs(w, o, dtype, extra=False)
    P, F, Fd = to_dev(pts, dtype), to_dev(frc, dtype), to_dev(fld, dtype)
    n = P.shape[0]
    for tile, block in ((256, 256), (1024, 256), (128, 64)):
        plan = ot.BatchPlan(cfg1_gpu, off, ops, dtype=dtype, mode="fixed", block=block, tile=tile)
        ids = torch.full((n,), -7, dtype=torch.int32, device="cuda")
        vel = torch.full((n, 3), -7.0, dtype=dtype, device="cuda")
        fo = torch.empty((cfg1_gpu.n_leaves, 3), dtype=dtype, device="cuda")
        plan.run(P, field=Fd, force=F, ids=ids, vel=vel, field_out=fo)
        torch.cuda.synchronize()
        ref_ids = cfg1_gpu.locate(P)
        ref_vel = cfg1_gpu.interpolate(Fd, P)
        spread_rows = torch.zeros(n, dtype=torch.bool, device="cuda")
        for i, op in enumerate(ops):
            a, b = off[i], off[i + 1]
            if op & 1:
                assert torch.equal(ids[a:b], ref_ids[a:b])
            else:
                assert (ids[a:b] == -7).all()
            if op & 2:
                assert torch.equal(vel[a:b], ref_vel[a:b])
            else:
                assert (vel[a:b] == -7).all()
            if op & 4:
                spread_rows[a:b] = True
        mask = spread_rows.cpu().numpy()
        f, S, cnt, A = o.spread(frc[mask], pts[mask], with_scale=True)
        q = fixed_point_quantum(frc)      # the plan's scale covers all n forces
        assert spread_excess(fo.cpu().numpy(), f, S, A, cnt, torch.float32, q) <= 1.0
        plan.close()


@pytest.mark.parametrize("sort", [False, True])
@pytest.mark.parametrize("dtype", DTYPES)
def test_batch_gradient_plans_match_one_pass(ot, cfg1, cfg1_gpu, dtype, sort):
    """Batched gradient passes, with the points sorted by host or not, equal
    the one-pass backward entries bit for bit: FIXED spreading does not
    depend on the order, and every point's sums are formed the same way."""
    w, o = cfg1
    pts, g, fld = _inputs(w, o, dtype, extra=False)
    P, G, Fd = to_dev(pts, dtype), to_dev(g, dtype), to_dev(fld, dtype)
    n, nl = P.shape[0], cfg1_gpu.n_leaves
    off = [0, 1000, 1500, 1507, 4000, n]
    # backward of interpolation: spread the upstream gradient, and the position gradient
    ops = [ot.OT_OP_SPREAD | ot.OT_OP_GRAD_POS] * 5
    plan = ot.BatchPlan(cfg1_gpu, off, ops, dtype=dtype, mode="fixed", sort_points=sort, block=128, tile=256)
    gf = torch.empty((nl, 3), dtype=dtype, device="cuda")
    gx = torch.full((n, 3), -7.0, dtype=dtype, device="cuda")
    ref_f, ref_x = cfg1_gpu.interp_backward(Fd, G, P, mode="fixed")
    for _ in range(2):   # capture, then replay
        plan.run(P, field=Fd, force=G, field_out=gf, grad=gx)
        torch.cuda.synchronize()
        assert torch.equal(gf, ref_f)
        assert torch.equal(gx, ref_x)
    plan.close()
    # backward of spreading: interpolate the field's gradient, and the position gradient
    plan = ot.BatchPlan(cfg1_gpu, off, [ot.OT_OP_INTERPOLATE | ot.OT_OP_GRAD_POS] * 5, dtype=dtype,
                        sort_points=sort, block=128, tile=256)
    gF = torch.empty((n, 3), dtype=dtype, device="cuda")
    gx2 = torch.empty((n, 3), dtype=dtype, device="cuda")
    plan.run(P, field=Fd, force=G, vel=gF, grad=gx2)
    ref_F, ref_x2 = cfg1_gpu.spread_backward(Fd, G, P)
    assert torch.equal(gF, ref_F)
    assert torch.equal(gx2, ref_x2)
    plan.close()


def test_batch_gradient_plan_mixed_instances(ot, cfg1, cfg1_gpu):
    """Unsorted gradient plans may mix the three gradient op sets per
    instance; ot_batch_run and ot_batch_run_grad refuse the other kind."""
    w, o = cfg1
    dtype = torch.float64
    pts, g, fld = _inputs(w, o, dtype, extra=False)
    P, G, Fd = to_dev(pts, dtype), to_dev(g, dtype), to_dev(fld, dtype)
    n, nl = P.shape[0], cfg1_gpu.n_leaves
    off = [0, 1000, 1500, 1507, 4000, n]
    GP, I, S = ot.OT_OP_GRAD_POS, ot.OT_OP_INTERPOLATE, ot.OT_OP_SPREAD
    ops = [GP | S, GP, GP | I, GP | S, GP | I]
    plan = ot.BatchPlan(cfg1_gpu, off, ops, dtype=dtype, mode="atomic")
    vel = torch.full((n, 3), -7.0, dtype=dtype, device="cuda")
    fo = torch.empty((nl, 3), dtype=dtype, device="cuda")
    gx = torch.empty((n, 3), dtype=dtype, device="cuda")
    plan.run(P, field=Fd, force=G, vel=vel, field_out=fo, grad=gx)
    torch.cuda.synchronize()
    assert torch.equal(gx, cfg1_gpu.grad_pos(Fd, G, P))
    ref_vel = cfg1_gpu.interpolate(Fd, P)
    rows = torch.zeros(n, dtype=torch.bool)
    for i, op in enumerate(ops):
        a, b = off[i], off[i + 1]
        if op & I:
            assert torch.equal(vel[a:b], ref_vel[a:b])
        else:
            assert (vel[a:b] == -7).all()
        if op & S:
            rows[a:b] = True
    m = rows.numpy()
    f, Sf, cnt, A = o.spread(g[m], pts[m], with_scale=True)
    assert spread_excess(fo.cpu().numpy(), f, Sf, A, cnt, dtype) <= 1.0
    with pytest.raises(ot.OtError):
        ot._check(ot.lib.ot_batch_run(plan._h, ot._ptr(Fd), ot._ptr(G), ot._ptr(P), None, ot._ptr(vel),
                                      ot._ptr(fo), ot._stream()))
    plan.close()
    fwd = ot.BatchPlan(cfg1_gpu, off, [7] * 5, dtype=dtype)
    with pytest.raises(ot.OtError):
        ot._check(ot.lib.ot_batch_run_grad(fwd._h, ot._ptr(Fd), ot._ptr(G), ot._ptr(P), None, ot._ptr(vel),
                                           ot._ptr(fo), ot._ptr(gx), ot._stream()))
    fwd.close()
    with pytest.raises(ot.OtError):   # gradient and forward-only ops in one plan
        ot.BatchPlan(cfg1_gpu, off, [7, GP, 7, 7, 7], dtype=dtype)


def test_batch_graph_replays_are_identical(ot, cfg1, cfg1_gpu):
    w, o = cfg1
    pts, frc, fld = _inputs(w, o, torch.float32, extra=False)
    P, F, Fd = to_dev(pts, torch.float32), to_dev(frc, torch.float32), to_dev(fld, torch.float32)
    n = P.shape[0]
    plan = ot.BatchPlan(cfg1_gpu, [0, 1000, n], [7, 7], dtype=torch.float32, mode="fixed", graph=True)
    ids = torch.empty(n, dtype=torch.int32, device="cuda")
    vel = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    fo = torch.empty((cfg1_gpu.n_leaves, 3), dtype=torch.float32, device="cuda")
    plan.run(P, field=Fd, force=F, ids=ids, vel=vel, field_out=fo)
    torch.cuda.synchronize()
    ref = (ids.clone(), vel.clone(), fo.clone())
    eager = cfg1_gpu.spread(F, P, mode="fixed")
    assert torch.equal(fo, eager)
    for r in range(4):
        ids.fill_(-1)
        vel.zero_()
        fo.fill_(123.0)
        _ = cfg1_gpu.interpolate(Fd, P)          # eager work between replays
        torch.cuda.synchronize()
        plan.run(P, field=Fd, force=F, ids=ids, vel=vel, field_out=fo)
        torch.cuda.synchronize()
        assert torch.equal(ids, ref[0]) and torch.equal(vel, ref[1]) and torch.equal(fo, ref[2])
    plan.close()
    # the same plan without the graph: its launches enqueued directly
    direct = ot.BatchPlan(cfg1_gpu, [0, 1000, n], [7, 7], dtype=torch.float32, mode="fixed")
    ids.fill_(-1)
    vel.zero_()
    fo.fill_(123.0)
    direct.run(P, field=Fd, force=F, ids=ids, vel=vel, field_out=fo)
    torch.cuda.synchronize()
    assert torch.equal(ids, ref[0]) and torch.equal(vel, ref[1]) and torch.equal(fo, ref[2])
    direct.close()


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("mode", ["fixed", "atomic"])
def test_batch_sorted_points_match_plain(ot, cfg1, cfg1_gpu, dtype, mode):
    """Sorting the points by host leaf inside the plan changes nothing:
    ids and velocities are bitwise those of the plain launches, fixed-point
    spreading is bitwise the same, atomic spreading within tolerance."""
    w, o = cfg1
    pts, frc, fld = _inputs(w, o, dtype, extra=True)
    P, F, Fd = to_dev(pts, dtype), to_dev(frc, dtype), to_dev(fld, dtype)
    n = P.shape[0]
    off = [0, 1000, 5000, n]
    plan = ot.BatchPlan(cfg1_gpu, off, [7, 7, 7], dtype=dtype, mode=mode, sort_points=True, block=256, tile=512)
    ids = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    vel = torch.zeros((n, 3), dtype=dtype, device="cuda")
    fo = torch.empty((cfg1_gpu.n_leaves, 3), dtype=dtype, device="cuda")
    for _ in range(2):
        plan.run(P, field=Fd, force=F, ids=ids, vel=vel, field_out=fo)
        torch.cuda.synchronize()
        assert torch.equal(ids, cfg1_gpu.locate(P))
        assert torch.equal(vel, cfg1_gpu.interpolate(Fd, P))
        ref = cfg1_gpu.spread(F, P, mode=mode)
        if mode == "fixed":
            assert torch.equal(fo, ref)
        else:
            f, S, cnt, A = o.spread(frc, pts, with_scale=True)
            assert spread_excess(fo.cpu().numpy(), f, S, A, cnt, dtype) <= 1.0
    with pytest.raises(ot.OtError):
        ot.BatchPlan(cfg1_gpu, off, [7, 3, 7], dtype=dtype, mode=mode, sort_points=True)
    plan.close()


@pytest.mark.parametrize("dtype", DTYPES)
def test_batch_gradient_plan_walled_deep_tree(ot, dtype):
    """Gradient plans on a walled tree with several table levels (nodes
    outside the cube dropped, points outside it without a host), sorted:
    equal to the one-pass entries bit for bit."""
    spec = synth.band_tree(2, 9, [synth.Sphere((0.3, 0.6, 0.5), 0.2), synth.Sphere((0.8, 0.2, 0.15), 0.1)],
                           periodic=False, seed=5)
    t = gpu_tree(spec)
    rng = np.random.default_rng(12)
    pts = as_dtype(np.concatenate([synth.fibonacci_sphere(synth.Sphere((0.3, 0.6, 0.5), 0.2), 3000, wrap=False),
                                   rng.random((3000, 3)), _extra_points(rng, 9, 300)]), dtype)
    g = as_dtype(rng.standard_normal(pts.shape), dtype)
    fld = as_dtype(rng.standard_normal((spec.n_leaves, 3)), dtype)
    P, G, Fd = to_dev(pts, dtype), to_dev(g, dtype), to_dev(fld, dtype)
    n = P.shape[0]
    off = [0, 3000, n]
    plan = ot.BatchPlan(t, off, [ot.OT_OP_SPREAD | ot.OT_OP_GRAD_POS] * 2, dtype=dtype, mode="fixed",
                        sort_points=True)
    gf = torch.empty((t.n_leaves, 3), dtype=dtype, device="cuda")
    gx = torch.empty((n, 3), dtype=dtype, device="cuda")
    plan.run(P, field=Fd, force=G, field_out=gf, grad=gx)
    ref_f, ref_x = t.interp_backward(Fd, G, P, mode="fixed")
    assert torch.equal(gf, ref_f)
    assert torch.equal(gx, ref_x)
    plan.close()
