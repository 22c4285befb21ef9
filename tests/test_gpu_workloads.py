"""Full-size parity on the five bubble/particle workloads, in the launch
configuration the benchmark times (batched persistent pass, FP32, points
sorted by host leaf inside the run, fixed-point spreading), plus the
differentiable pair.

The oracle cannot redo 10^7..10^8 points, so it checks sampled outputs one by
one: host ids and velocities of sampled points, and the spread value of
sampled leaves.  A leaf's spread value only involves points within three of
its own cell widths (host level >= leaf level - 1 under 2:1 balance, stencil
reach 3/2 host cells), so the oracle spreads exactly the points of the
surrounding coarse bins and reads the sampled leaves off that.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import (ETA, TOL, as_dtype, fixed_point_quantum, gpu_tree, oracle_tree, scaled_err,
                      spread_excess, to_dev)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ot():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2605_20565_amd as m
    return m


def _say(msg):
    print(f"[workloads] {msg}", flush=True)


def _near_points(points, leaf_centres, level, chunk=1 << 23):
    """Indices of the points in the 27 coarse level-`level` bins around each
    leaf centre (periodic)."""
    m = 1 << level
    want = np.zeros(m ** 3, dtype=bool)
    c = np.floor(np.mod(leaf_centres, 1.0) * m).astype(np.int64)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                cc = (c + np.array([dx, dy, dz])) % m
                want[cc[:, 0] + m * (cc[:, 1] + m * cc[:, 2])] = True
    out = []
    for a in range(0, points.shape[0], chunk):
        p = points[a:a + chunk]
        q = np.floor(np.mod(p, 1.0) * m).astype(np.int64) % m
        out.append(a + np.nonzero(want[q[:, 0] + m * (q[:, 1] + m * q[:, 2])])[0])
    return np.concatenate(out)


def _sample_leaves(o, rng, n, prefer_fine=True):
    fine = np.nonzero(o.levels == o.l_max)[0]
    coarse = np.nonzero(o.levels < o.l_max)[0]
    a = rng.choice(fine, size=min(n // 2, fine.size), replace=False) if prefer_fine and fine.size else []
    b = rng.choice(coarse, size=min(n - len(a), coarse.size), replace=False)
    return np.sort(np.concatenate([np.asarray(a, dtype=np.int64), b]))


def _leaf_centres(o, ids):
    xs = np.array([oracle.morton_decode(int(k), o.l_max) for k in o.keys[ids]], dtype=np.float64)
    half = np.ldexp(0.5, o.l_max - o.levels[ids].astype(np.int64))
    return (xs + half[:, None]) * math.ldexp(1.0, -o.l_max)


def _check_sampled(w, o, pts, frc, fld, ids, vel, fo, dtype, rng, n_pts=20000, n_leaves=120, quantum=None,
                   spread=True):
    """ids / vel at sampled points and spread values at sampled leaves."""
    k = np.sort(rng.choice(pts.shape[0], size=min(n_pts, pts.shape[0]), replace=False))
    want_ids = o.locate(pts[k])
    assert np.array_equal(ids[k].astype(np.int64), want_ids)
    U, S = o.interpolate(fld, pts[k], with_scale=True)
    assert scaled_err(vel[k], U, S) <= TOL[dtype]
    if not spread:
        return 0
    # spread at sampled leaves: bins of the leaf's own coarsest possible host
    # level cover the reach (3 cells at level l_min - 1 ... conservative: use
    # bins one level coarser than l_min, plus their neighbours)
    leaves = _sample_leaves(o, rng, n_leaves)
    near = _near_points(pts, _leaf_centres(o, leaves), max(0, o.l_min - 2))
    _say(f"oracle spread of {len(near)} points around {len(leaves)} sampled leaves")
    f, Sf, cnt, A = o.spread(frc[near], pts[near], with_scale=True)
    got = fo[leaves]
    assert spread_excess(got, f[leaves], Sf[leaves], A[leaves], cnt[leaves], dtype, quantum) <= 1.0
    return len(near)


def _run_bench_config(ot, w, dtype, mode="fixed", sort_points=True, ops=None):
    t = gpu_tree(w.tree)
    pts = as_dtype(w.points, dtype)
    frc = as_dtype(w.forces, dtype)
    P, F = to_dev(pts, dtype), to_dev(frc, dtype)
    Fd = t.permute_rows(to_dev(w.field, dtype))
    n = P.shape[0]
    offs = [int(v) for v in w.instances]
    ops = ops or [7] * (len(offs) - 1)
    plan = ot.BatchPlan(t, offs, ops, dtype=dtype, mode=mode, sort_points=sort_points)
    ids = torch.empty(n, dtype=torch.int32, device="cuda")
    vel = torch.empty((n, 3), dtype=dtype, device="cuda")
    fo = torch.empty((t.n_leaves, 3), dtype=dtype, device="cuda")
    plan.run(P, field=Fd, force=F, ids=ids, vel=vel, field_out=fo)
    torch.cuda.synchronize()
    return t, plan, (P, F, Fd), (pts, frc), (ids, vel, fo)


# ---------------------------------------------------------------------------
# Workload 2: 8 bubbles + 10^7 uniform particles, l 7 -> 10
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def cfg2():
    w = synth.workload(2)
    return w, oracle_tree(w.tree)


def test_cfg2_fp32_batched_sorted_fixed(ot, cfg2):
    w, o = cfg2
    dt = torch.float32
    t, plan, dev, (pts, frc), (ids, vel, fo) = _run_bench_config(ot, w, dt)
    fld = as_dtype(o.permute_rows(w.field), dt)
    rng = np.random.default_rng(2)
    near = _check_sampled(w, o, pts, frc, fld, ids.cpu().numpy(), vel.cpu().numpy(), fo.cpu().numpy(), dt, rng,
                          quantum=fixed_point_quantum(frc))
    assert near > 1000
    # leaf ids of the 8 bubbles' markers are all at the finest level
    mk = slice(0, int(w.instances[8]))
    assert (o.levels[ids[mk].cpu().numpy()] == o.l_max).all()
    # conservation: the sum over leaves equals the sum of the forces within the quantisation bound
    q = fixed_point_quantum(frc)
    tot = fo.double().sum(dim=0).cpu().numpy()
    assert np.all(np.abs(tot - frc.sum(axis=0)) <= 27 * frc.shape[0] * q + 1e-6 * np.abs(frc).sum(axis=0))
    # determinism of the whole batched pass
    fo2 = torch.empty_like(fo)
    plan.run(dev[0], field=dev[2], force=dev[1], ids=ids, vel=vel, field_out=fo2)
    torch.cuda.synchronize()
    assert torch.equal(fo, fo2)
    plan.close()


def test_cfg2_fp64_plain_and_adjoint(ot, cfg2):
    """FP64 plain launches (the speedup's denominator) against the oracle,
    and the adjoint identity at full size."""
    w, o = cfg2
    dt = torch.float64
    t = gpu_tree(w.tree)
    P, F = to_dev(w.points, dt), to_dev(w.forces, dt)
    Fd = t.permute_rows(to_dev(w.field, dt))
    ids, vel, fo = t.track(P, field=Fd, force=F, mode="atomic")
    torch.cuda.synchronize()
    fld = o.permute_rows(w.field)
    rng = np.random.default_rng(3)
    _check_sampled(w, o, w.points, w.forces, fld, ids.cpu().numpy(), vel.cpu().numpy(), fo.cpu().numpy(), dt, rng,
                   n_pts=10000, n_leaves=80)
    u = torch.randn((t.n_leaves, 3), dtype=dt, device="cuda", generator=torch.Generator("cuda").manual_seed(5))
    lhs = float((fo * u).sum())
    rhs = float((F * t.interpolate(u, P)).sum())
    assert abs(lhs - rhs) <= 1e-11 * (float((fo.abs() * u.abs()).sum()) + 1.0)


# ---------------------------------------------------------------------------
# Workload 3: 256 bubbles (d log-uniform) + 64 particle groups, l 7 -> 10
# ---------------------------------------------------------------------------
def test_cfg3_batched_uneven_instances(ot):
    _say("generating workload 3")
    w = synth.workload(3)
    o = oracle_tree(w.tree)
    dt = torch.float32
    n_inst = len(w.instances) - 1
    assert n_inst == 320
    t, plan, dev, (pts, frc), (ids, vel, fo) = _run_bench_config(ot, w, dt)
    fld = as_dtype(o.permute_rows(w.field), dt)
    rng = np.random.default_rng(33)
    _check_sampled(w, o, pts, frc, fld, ids.cpu().numpy(), vel.cpu().numpy(), fo.cpu().numpy(), dt, rng,
                   n_pts=15000, n_leaves=100, quantum=fixed_point_quantum(frc))
    # the unsorted persistent pass and per-instance launches agree with it
    P, F, Fd = dev
    plan_u = ot.BatchPlan(t, [int(v) for v in w.instances], [7] * n_inst, dtype=dt, mode="fixed")
    ids_u, vel_u, fo_u = torch.empty_like(ids), torch.empty_like(vel), torch.empty_like(fo)
    plan_u.run(P, field=Fd, force=F, ids=ids_u, vel=vel_u, field_out=fo_u)
    torch.cuda.synchronize()
    assert torch.equal(ids_u, ids) and torch.equal(vel_u, vel) and torch.equal(fo_u, fo)
    for i in rng.choice(n_inst, size=12, replace=False):
        a, b = int(w.instances[i]), int(w.instances[i + 1])
        assert torch.equal(t.locate(P[a:b]), ids[a:b])
        assert torch.equal(t.interpolate(Fd, P[a:b]), vel[a:b])
    plan.close()
    plan_u.close()


# ---------------------------------------------------------------------------
# Workload 4: 10^8 particles in Gaussian shells around 32 bubbles, l 8 -> 11
# ---------------------------------------------------------------------------
@pytest.mark.slow
def test_cfg4_spreading_stress(ot):
    _say("generating workload 4 (10^8 points)")
    w = synth.workload(4)
    _say("oracle tree")
    o = oracle_tree(w.tree)
    dt = torch.float32
    _say("batched pass")
    t, plan, dev, (pts, frc), (ids, vel, fo) = _run_bench_config(ot, w, dt)
    _say("sampled checks")
    fld = as_dtype(o.permute_rows(w.field), dt)
    rng = np.random.default_rng(44)
    _check_sampled(w, o, pts, frc, fld, ids.cpu().numpy(), vel.cpu().numpy(), fo.cpu().numpy(), dt, rng,
                   n_pts=10000, spread=False)
    # conservation at full size, within the quantisation bound
    q = fixed_point_quantum(frc)
    tot = fo.double().sum(dim=0).cpu().numpy()
    assert np.all(np.abs(tot - frc.sum(axis=0)) <= 27 * frc.shape[0] * q + 1e-6 * np.abs(frc).sum(axis=0))
    # element-wise spreading parity on a 10^6-point subsample through the same batched, sorted configuration
    _say("subsample spreading parity")
    sub = np.sort(rng.choice(pts.shape[0], size=1_000_000, replace=False))
    ps, fs = pts[sub], frc[sub]
    sp = ot.BatchPlan(t, [0, len(sub)], [7], dtype=dt, mode="fixed", sort_points=True)
    Ps, Fs = to_dev(ps, dt), to_dev(fs, dt)
    ids_s = torch.empty(len(sub), dtype=torch.int32, device="cuda")
    vel_s = torch.empty((len(sub), 3), dtype=dt, device="cuda")
    fo_s = torch.empty_like(fo)
    sp.run(Ps, field=dev[2], force=Fs, ids=ids_s, vel=vel_s, field_out=fo_s)
    torch.cuda.synchronize()
    sp.close()
    _check_sampled(w, o, ps, fs, fld, ids_s.cpu().numpy(), vel_s.cpu().numpy(), fo_s.cpu().numpy(), dt, rng,
                   n_pts=5000, n_leaves=60, quantum=fixed_point_quantum(fs))
    _say("determinism and modes")
    P, F, Fd = dev
    # bitwise reproducible over five runs of the batched fixed-point pass
    for _ in range(4):
        fo2 = torch.empty_like(fo)
        plan.run(P, field=Fd, force=F, ids=ids, vel=vel, field_out=fo2)
        torch.cuda.synchronize()
        assert torch.equal(fo, fo2)
    plan.close()
    # FP32 atomics and FP64 atomics stay within tolerance of each other at sampled leaves
    fa = t.spread(F, P, mode="atomic")
    leaves = torch.from_numpy(_sample_leaves(o, rng, 2000)).cuda()
    rel = (fa[leaves].double() - fo[leaves].double()).abs().max() / fo.double().abs().max()
    assert float(rel) < 1e-5


# ---------------------------------------------------------------------------
# Workload 5: differentiable pair, 10^6 markers on the workload-2 tree
# ---------------------------------------------------------------------------
def test_cfg5_autograd_against_oracle(ot, cfg2):
    _say("generating workload 5")
    w5 = synth.workload(5)
    o = oracle_tree(w5.tree)
    dt = torch.float32
    t = gpu_tree(w5.tree)
    pts = as_dtype(w5.points, dt)
    fld = as_dtype(o.permute_rows(w5.field), dt)
    rng = np.random.default_rng(55)
    g = as_dtype(rng.standard_normal(pts.shape), dt)
    X = to_dev(pts, dt).requires_grad_(True)
    u = to_dev(fld, dt).requires_grad_(True)
    U = ot.interpolate(t, u, X, mode="fixed")
    (U * to_dev(g, dt)).sum().backward()
    gx = X.grad.cpu().numpy()
    gu = u.grad.cpu().numpy()
    k = np.sort(rng.choice(pts.shape[0], size=20000, replace=False))
    want, S = o.grad_pos(fld, g[k], pts[k], with_scale=True)
    assert scaled_err(gx[k], want, S) <= TOL[dt]
    # grad of the field = spread of the upstream gradient (sampled leaves)
    leaves = _sample_leaves(o, rng, 100)
    near = _near_points(pts, _leaf_centres(o, leaves), max(0, o.l_min - 2))
    f, Sf, cnt, A = o.spread(g[near], pts[near], with_scale=True)
    assert spread_excess(gu[leaves], f[leaves], Sf[leaves], A[leaves], cnt[leaves], dt,
                         fixed_point_quantum(g)) <= 1.0


def test_cfg5_batched_gradient_plan_equals_one_pass(ot):
    """Workload 5 at full size (10^6 markers, 125 k per bubble): the sorted
    batched backward of interpolation equals the plain one-pass entry bit
    for bit (FIXED), in the launch shape the bench's plan uses."""
    _say("generating workload 5 (batched gradient)")
    w5 = synth.workload(5)
    dt = torch.float32
    t = gpu_tree(w5.tree)
    P = to_dev(as_dtype(w5.points, dt), dt)
    rng = np.random.default_rng(56)
    G = to_dev(as_dtype(rng.standard_normal(w5.points.shape), dt), dt)
    u = t.permute_rows(to_dev(as_dtype(w5.field, dt), dt))
    ref_f, ref_x = t.interp_backward(u, G, P, mode="fixed")
    plan = ot.BatchPlan(t, [0, P.shape[0]], [ot.OT_OP_SPREAD | ot.OT_OP_GRAD_POS], dtype=dt, mode="fixed",
                        sort_points=True)
    gf = torch.empty_like(u)
    gx = torch.empty_like(P)
    plan.run(P, field=u, force=G, field_out=gf, grad=gx)
    torch.cuda.synchronize()
    assert torch.equal(gf, ref_f)
    assert torch.equal(gx, ref_x)
    plan.close()


def test_cfg2_mdf_markers_equal_dense_composition(ot, cfg2):
    """Multi-direct forcing on workload 2's 65,880 bubble markers (2.66 M
    leaves): the kept stencils and per-leaf pair sums give, bit for bit, the
    dense composition of the library's interpolation and spreading (FIXED),
    with the elementwise steps as true divisions."""
    w, o = cfg2
    dt_ = torch.float32
    t = gpu_tree(w.tree)
    idx = [i for i, k in enumerate(w.kinds) if k == "markers"]
    sel = np.concatenate([np.arange(w.instances[i], w.instances[i + 1]) for i in idx])
    P = to_dev(as_dtype(w.points[sel], dt_), dt_)
    rng = np.random.default_rng(21)
    target = to_dev(as_dtype(0.1 * rng.standard_normal(P.shape), dt_), dt_)
    u0 = t.permute_rows(to_dev(as_dtype(w.field, dt_), dt_))
    n_iter, step, rho = 3, 0.75, 1.25
    ug, flg, feg = t.mdf(u0, P, target, n_iter, step, rho, mode="fixed")
    u = u0.clone()
    step_t, rho_t = torch.full_like(P, step), torch.full_like(u0, rho)
    fl = torch.zeros_like(P)
    fe = torch.zeros_like(u0)
    for _ in range(n_iter):
        F = (target - t.interpolate(u, P)) / step_t
        f = t.spread(F, P, mode="fixed")
        u = u + f / rho_t
        fl = fl + F
        fe = fe + f
    assert torch.equal(ug, u)
    assert torch.equal(flg, fl)
    assert torch.equal(feg, fe)


def test_autograd_matches_central_differences_fp64(ot):
    """FP64 gradients of the pair against central differences with
    h = 1e-4 finest dx, points kept away from cell faces and phi kinks."""
    w = synth.workload(1)
    o = oracle_tree(w.tree)
    t = gpu_tree(w.tree)
    rng = np.random.default_rng(66)
    pts = w.points[::11].copy()
    L = w.tree.l_max
    host, level, _ = o.stencil_leaves(pts)
    s = pts * np.ldexp(1.0, level)[:, None]
    frac = s - np.floor(s)
    away = np.all(np.minimum.reduce([np.abs(frac - c) for c in (0.0, 0.5, 1.0)]) > 0.01, axis=1)
    pts = pts[away]
    dt = torch.float64
    X = torch.from_numpy(pts).cuda().requires_grad_(True)
    u = torch.from_numpy(o.permute_rows(w.field)).cuda().requires_grad_(True)
    F = torch.from_numpy(rng.standard_normal(pts.shape)).cuda().requires_grad_(True)
    gU = torch.from_numpy(rng.standard_normal(pts.shape)).cuda()
    gf = torch.from_numpy(rng.standard_normal((t.n_leaves, 3))).cuda()
    U = ot.interpolate(t, u, X, mode="atomic")
    f = ot.spread(t, F, X, mode="atomic")
    loss = (U * gU).sum() + (f * gf).sum()
    loss.backward()
    h = 1e-4 * math.ldexp(1.0, -L)

    def L_of(Xv):
        with torch.no_grad():
            return float((t.interpolate(u, Xv) * gU).sum() + (t.spread(F, Xv, mode="atomic") * gf).sum())

    fd = np.zeros_like(pts)
    for d in range(3):
        for k in range(0, pts.shape[0], max(1, pts.shape[0] // 60)):
            e = torch.zeros_like(X)
            e[k, d] = h
            fd[k, d] = (L_of(X.detach() + e) - L_of(X.detach() - e)) / (2 * h)
    chk = np.arange(0, pts.shape[0], max(1, pts.shape[0] // 60))
    got = X.grad.cpu().numpy()[chk]
    scale = np.abs(got).max() + 1.0
    assert np.abs(got - fd[chk]).max() <= 1e-6 * scale
    # and the linear parts: d/du of <U, gU> is spread(gU); d/dF of <f, gf> is interpolate(gf)
    assert torch.allclose(u.grad, t.spread(gU, X.detach(), mode="atomic"), rtol=0, atol=1e-12)
    assert torch.allclose(F.grad, t.interpolate(gf, X.detach()), rtol=0, atol=1e-12)


def test_cfg5_gradient_central_differences_and_oracle(ot):
    """Workload 5 (10^6 markers on the workload-2 tree): the position
    gradient of <interpolate(u), gU> + <spread(F), gf> through the pair's
    autograd backward, against FP64 central differences with h = 1e-4 finest
    dx (points kept away from cell faces and phi kinks; the gradient holds
    the host fixed) and against the oracle gradient, in FP64 and FP32.  Each
    point's terms depend on its own position only, so the differences are
    taken for a sample with all perturbed positions in one batch, the
    spreading term through its adjoint <F, interpolate(gf)>."""
    _say("generating workload 5 (finite differences)")
    w5 = synth.workload(5)
    o = oracle_tree(w5.tree)
    t = gpu_tree(w5.tree)
    rng = np.random.default_rng(77)
    k = np.sort(rng.choice(w5.points.shape[0], size=6000, replace=False))
    pts = w5.points[k]
    host, level, _ = o.stencil_leaves(pts)
    s = pts * np.ldexp(1.0, level)[:, None]
    frac = s - np.floor(s)
    away = np.all(np.minimum.reduce([np.abs(frac - c) for c in (0.0, 0.5, 1.0)]) > 0.01, axis=1)
    pts = pts[away][:3000]
    n = pts.shape[0]
    fld = o.permute_rows(w5.field)
    gU = rng.standard_normal((n, 3))
    F = rng.standard_normal((n, 3))
    gf = rng.standard_normal((t.n_leaves, 3))
    for dt in (torch.float64, torch.float32):
        # the oracle sees exactly the values the GPU sees
        a_p, a_f, a_u, a_g, a_gf = (as_dtype(v, dt) for v in (pts, F, fld, gU, gf))
        w1, S1 = o.grad_pos(a_u, a_g, a_p, with_scale=True)
        w2, S2 = o.grad_pos(a_gf, a_f, a_p, with_scale=True)
        want = w1 + w2
        P = to_dev(as_dtype(pts, dt), dt).requires_grad_(True)
        u = to_dev(as_dtype(fld, dt), dt)
        Fd = to_dev(as_dtype(F, dt), dt)
        loss = (ot.interpolate(t, u, P, mode="fixed") * to_dev(as_dtype(gU, dt), dt)).sum() + \
            (ot.spread(t, Fd, P, mode="fixed") * to_dev(as_dtype(gf, dt), dt)).sum()
        loss.backward()
        got = P.grad.double().cpu().numpy()
        if dt == torch.float64:
            h = 1e-4 * math.ldexp(1.0, -w5.tree.l_max)
            X = torch.from_numpy(pts).cuda()
            uu, gg = torch.from_numpy(fld).cuda(), torch.from_numpy(gf).cuda()
            GU, FF = torch.from_numpy(gU).cuda(), torch.from_numpy(F).cuda()
            fd = np.zeros_like(pts)
            for d in range(3):
                e = torch.zeros_like(X)
                e[:, d] = h
                lp = (t.interpolate(uu, X + e) * GU).sum(1) + (t.interpolate(gg, X + e) * FF).sum(1)
                lm = (t.interpolate(uu, X - e) * GU).sum(1) + (t.interpolate(gg, X - e) * FF).sum(1)
                fd[:, d] = ((lp - lm) / (2 * h)).cpu().numpy()
            scale = np.abs(got).max() + 1.0
            assert np.abs(got - fd).max() <= 1e-6 * scale
        # against the oracle gradient on the scaled metric (sum of both terms' scales)
        assert scaled_err(got, want, S1 + S2) <= TOL[dt]
