"""The host-major pass of sorted batched plans (points sharing a host share
its 27 node lookups, field values and spreading targets) against the
per-point pass and the plain launches: host ids and velocities bit for bit,
fixed-point spreading bit for bit (the same rounded contributions, summed
exactly), atomic spreading within the oracle bound.  Dense point sets make
long runs of points per host (the windows the pass takes); sparse ones are
handed to the per-point pass, and mixtures exercise both in one run."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import (as_dtype, fixed_point_quantum, gpu_tree, oracle_tree, scaled_err, spread_excess, to_dev,
                      TOL)

pytestmark = pytest.mark.gpu

DTYPES = [torch.float32, torch.float64]


@pytest.fixture(scope="module")
def ot():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2605_20565_amd as m
    return m


@pytest.fixture(scope="module")
def band():
    """Periodic l 5 -> 8 tree around two spheres (level jumps of 1 by balance)."""
    spec = synth.band_tree(5, 8, [synth.Sphere((0.4, 0.5, 0.55), 0.15), synth.Sphere((0.8, 0.2, 0.3), 0.08)],
                           periodic=True, seed=21)
    return spec, oracle_tree(spec), gpu_tree(spec)


@pytest.fixture(scope="module")
def walled():
    spec = synth.band_tree(4, 7, [synth.Sphere((0.3, 0.6, 0.5), 0.2), synth.Sphere((0.85, 0.15, 0.1), 0.1)],
                           periodic=False, seed=5)
    return spec, oracle_tree(spec), gpu_tree(spec)


def _points(spec, rng, dense, sparse):
    """`dense` uniform points concentrated in a few boxes (many per host) plus
    `sparse` markers on a sphere, random order, a few outside the cube and NaN."""
    boxes = rng.random((6, 3)) * 0.8
    d = boxes[rng.integers(0, 6, dense)] + rng.random((dense, 3)) * 0.2
    m = synth.fibonacci_sphere(synth.Sphere((0.4, 0.5, 0.55), 0.15), sparse, wrap=spec.periodic)
    extra = np.array([[np.nan, 0.2, 0.2], [-0.01, 0.5, 0.5], [1.0, 0.5, 0.5], [0.5, 0.5, np.nextafter(1.0, 0)]])
    pts = np.concatenate([d, m, extra])
    return pts[rng.permutation(pts.shape[0])]


def _run(ot, t, pts, frc, fld, dtype, mode, ops=7, **kw):
    P, F, U = to_dev(pts, dtype), to_dev(frc, dtype), to_dev(fld, dtype)
    n = P.shape[0]
    plan = ot.BatchPlan(t, [0, n // 3, n], [ops, ops], dtype=dtype, mode=mode, **kw)
    ids = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    vel = torch.full((n, 3), -7.0, dtype=dtype, device="cuda")
    fo = torch.empty((t.n_leaves, 3), dtype=dtype, device="cuda")
    plan.run(P, field=U if ops & 2 else None, force=F if ops & 4 else None, ids=ids if ops & 1 else None,
             vel=vel if ops & 2 else None, field_out=fo if ops & 4 else None)
    torch.cuda.synchronize()
    win = plan.windows()
    plan.close()
    return ids, vel, fo, win


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("tree", ["band", "walled"])
def test_host_major_equals_per_point_and_plain(ot, request, dtype, tree):
    spec, o, t = request.getfixturevalue(tree)
    rng = np.random.default_rng(101)
    pts = as_dtype(_points(spec, rng, 200_000, 3000), dtype)
    frc = as_dtype(rng.standard_normal(pts.shape), dtype)
    fld = as_dtype(rng.standard_normal((spec.n_leaves, 3)), dtype)
    ids, vel, fo, (nw, fb) = _run(ot, t, pts, frc, fld, dtype, "fixed", sort_points=True, host_major=True)
    assert nw == (pts.shape[0] + 255) // 256
    assert 0 < fb < nw // 2, (nw, fb)   # most windows host-major, the marker windows handed over
    ids_p, vel_p, fo_p, (nw_p, _) = _run(ot, t, pts, frc, fld, dtype, "fixed", sort_points=True)
    assert nw_p == 0
    assert torch.equal(ids, ids_p) and torch.equal(vel, vel_p) and torch.equal(fo, fo_p)
    P, F, U = to_dev(pts, dtype), to_dev(frc, dtype), to_dev(fld, dtype)
    assert torch.equal(ids, t.locate(P))
    assert torch.equal(vel, t.interpolate(U, P))
    assert torch.equal(fo, t.spread(F, P, mode="fixed"))
    # against the oracle on a sample of points and all leaves
    k = np.sort(rng.choice(pts.shape[0], size=3000, replace=False))
    Uo, S = o.interpolate(fld, pts[k], with_scale=True)
    assert scaled_err(vel.cpu().numpy()[k], Uo, S) <= TOL[dtype]
    f, Sf, cnt, A = o.spread(frc, pts, with_scale=True)
    assert spread_excess(fo.cpu().numpy(), f, Sf, A, cnt, dtype, fixed_point_quantum(frc)) <= 1.0


@pytest.mark.parametrize("dtype", DTYPES)
def test_host_major_atomic_within_bound(ot, band, dtype):
    spec, o, t = band
    rng = np.random.default_rng(7)
    pts = as_dtype(_points(spec, rng, 100_000, 2000), dtype)
    frc = as_dtype(rng.standard_normal(pts.shape), dtype)
    fld = as_dtype(rng.standard_normal((spec.n_leaves, 3)), dtype)
    ids, vel, fo, (nw, fb) = _run(ot, t, pts, frc, fld, dtype, "atomic", sort_points=True, host_major=True)
    assert fb < nw
    P, U = to_dev(pts, dtype), to_dev(fld, dtype)
    assert torch.equal(vel, t.interpolate(U, P))
    f, S, cnt, A = o.spread(frc, pts, with_scale=True)
    assert spread_excess(fo.cpu().numpy(), f, S, A, cnt, dtype) <= 1.0


@pytest.mark.parametrize("ops", [2, 3, 4, 5, 6])
def test_host_major_op_subsets(ot, band, ops):
    """Interpolation alone, spreading alone, with or without host ids."""
    spec, o, t = band
    dtype = torch.float32
    rng = np.random.default_rng(ops)
    pts = as_dtype(_points(spec, rng, 60_000, 500), dtype)
    frc = as_dtype(rng.standard_normal(pts.shape), dtype)
    fld = as_dtype(rng.standard_normal((spec.n_leaves, 3)), dtype)
    ids, vel, fo, _ = _run(ot, t, pts, frc, fld, dtype, "fixed", ops=ops, sort_points=True, host_major=True)
    P, F, U = to_dev(pts, dtype), to_dev(frc, dtype), to_dev(fld, dtype)
    if ops & 1:
        assert torch.equal(ids, t.locate(P))
    else:
        assert (ids == -7).all()
    if ops & 2:
        assert torch.equal(vel, t.interpolate(U, P))
    else:
        assert (vel == -7).all()
    if ops & 4:
        assert torch.equal(fo, t.spread(F, P, mode="fixed"))


def test_host_major_dense_hosts_and_full_windows(ot, band):
    """Every point of a window in one host (runs of 256), and windows whose
    run count sits at the limit: still equal to the plain launches."""
    spec, o, t = band
    dtype = torch.float32
    rng = np.random.default_rng(9)
    # 4096 points inside one level-5 leaf, and 128 hosts with 2 points each repeated
    one = np.array([0.01, 0.01, 0.01]) + rng.random((4096, 3)) * 0.02
    cells = (rng.integers(0, 32, (128, 3)) + 0.5) / 32.0
    two = np.repeat(cells, 2, axis=0) + (rng.random((256, 3)) - 0.5) * 0.01
    pts = as_dtype(np.concatenate([one, two, one[:300] * 0.5 + 0.3]), dtype)
    frc = as_dtype(rng.standard_normal(pts.shape), dtype)
    fld = as_dtype(rng.standard_normal((spec.n_leaves, 3)), dtype)
    ids, vel, fo, _ = _run(ot, t, pts, frc, fld, dtype, "fixed", sort_points=True, host_major=True)
    P, F, U = to_dev(pts, dtype), to_dev(frc, dtype), to_dev(fld, dtype)
    assert torch.equal(ids, t.locate(P))
    assert torch.equal(vel, t.interpolate(U, P))
    assert torch.equal(fo, t.spread(F, P, mode="fixed"))
