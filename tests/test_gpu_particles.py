"""GPU point-particle step (ot_particle_step) against the FP64 oracle
(oracle/particles.py) over a few steps on the band tree of workload 1 and on a
walled random tree: positions, velocities and accelerations within
10 x tol of their magnitudes (tol 1e-12 FP64, 1e-5 FP32); host ids equal
Algorithm 1 on the GPU's own new positions (bit for bit)."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import TOL, as_dtype, gpu_tree, oracle_tree, to_dev
from oracle import particles as pp

pytestmark = pytest.mark.gpu

PRM = dict(r_p=2e-3, rho_p=2.5, rho_f=1.0, nu=2e-3, g=np.array([0.0, 0.0, -1.0]))


@pytest.fixture(scope="module")
def ot():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2605_20565_amd as m
    return m


def _cases():
    w = synth.workload(1)
    rng = np.random.default_rng(12)
    return {"band": (w.tree, w.field), "walls": (synth.random_tree(2, 5, rng, periodic=False), None)}


@pytest.mark.parametrize("name", ["band", "walls"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_particle_steps_match_oracle(ot, name, dtype):
    spec, field0 = _cases()[name]
    o, t = oracle_tree(spec), gpu_tree(spec)
    rng = np.random.default_rng(7)
    n = 4000
    field = field0 if field0 is not None else rng.standard_normal((len(spec.levels), 3)) * 0.1
    fld = as_dtype(o.permute_rows(field), dtype)
    x = as_dtype(rng.random((n, 3)), dtype)
    v = as_dtype(rng.standard_normal((n, 3)) * 0.05, dtype)
    vp = v.copy()
    ap = np.zeros((n, 3))
    dt0 = 2e-3
    X, V, VP, AP = (to_dev(a, dtype) for a in (x, v, vp, ap))
    ids = torch.from_numpy(o.locate(x).astype(np.int32)).cuda()
    F = to_dev(fld, dtype)
    tol = 10 * TOL[dtype]
    for m in range(3):
        x, v, vp, ap, want_ids = pp.step(o, fld, x, v, vp, ap, dt0, first=(m == 0), **PRM)
        t.particle_step(F, X, V, VP, AP, ids, dt0, first=(m == 0), **PRM)
        gx, gv, ga = (a.cpu().double().numpy() for a in (X, V, AP))
        assert np.abs(gx - x).max() <= tol * max(1.0, np.abs(x).max())
        assert np.abs(gv - v).max() <= tol * max(1e-3, np.abs(v).max())
        assert np.abs(ga - ap).max() <= tol * max(1e-3, np.abs(ap).max())
        assert np.array_equal(ids.cpu().numpy(), o.locate(gx))
        # carry on from the GPU's own state (the oracle sees exactly what the GPU holds)
        x, v, vp, ap = gx, gv, VP.cpu().double().numpy(), ga


def _bits(a):
    """The tensor's bit patterns (NaN rows compare equal to themselves)."""
    return a.view(torch.int32 if a.dtype == torch.float32 else torch.int64)


@pytest.mark.parametrize("name", ["band", "walls"])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_particle_sort_orders_by_host(ot, name, dtype):
    """ot_particle_sort: rows are the input rows permuted bit for bit, host ids
    (Algorithm 1 on the oracle) ascending with the particles without a host
    last, equal hosts in input order; a step on the sorted state equals the
    step on the input state, permuted."""
    spec, field0 = _cases()[name]
    o, t = oracle_tree(spec), gpu_tree(spec)
    rng = np.random.default_rng(31)
    n = 20_000
    x = rng.random((n, 3))
    x[::97] = x[::97] * 1.4 - 0.2           # some outside the cube (walls: no host)
    x[5] = [np.nan, 0.5, 0.5]
    x[6:400] = x[6]                         # one host with many particles
    x = as_dtype(x, dtype)
    v, vp, ap = (as_dtype(rng.standard_normal((n, 3)) * 0.05, dtype) for _ in range(3))
    X, V, VP, AP = (to_dev(a, dtype) for a in (x, v, vp, ap))
    Xs, Vs, VPs, APs, ids, perm = t.particle_sort(X, V, VP, AP)
    p = perm.cpu().numpy().astype(np.int64)
    assert np.array_equal(np.sort(p), np.arange(n))
    for a, b in ((Xs, X), (Vs, V), (VPs, VP), (APs, AP)):
        assert torch.equal(_bits(a), _bits(b)[perm.long()])
    want = o.locate(x)
    got = ids.cpu().numpy()
    assert np.array_equal(got, want[p])
    key = np.where(got < 0, np.int64(t.n_leaves), got.astype(np.int64))   # no host: last
    assert np.all(np.diff(key) >= 0)
    same = np.diff(key) == 0
    assert np.all(np.diff(p)[same] > 0)     # stable
    # a step on the sorted state is the step on the input state, permuted
    field = field0 if field0 is not None else rng.standard_normal((len(spec.levels), 3)) * 0.1
    F = to_dev(as_dtype(o.permute_rows(field), dtype), dtype)
    ids_in = t.locate(X)
    ids_s = ids.clone()
    t.particle_step(F, X, V, VP, AP, ids_in, 2e-3, **PRM)
    t.particle_step(F, Xs, Vs, VPs, APs, ids_s, 2e-3, **PRM)
    for a, b in ((Xs, X), (Vs, V), (VPs, VP), (APs, AP)):
        assert torch.equal(_bits(a), _bits(b)[perm.long()])
    assert torch.equal(ids_s, ids_in[perm.long()])
    # caller workspace and output arrays
    work = torch.empty(ot.lib.ot_particle_sort_workspace_bytes(n), dtype=torch.uint8, device="cuda")
    outs = tuple(torch.empty_like(X) for _ in range(4))
    r = t.particle_sort(X, V, VP, AP, out=outs, work=work)
    assert all(a is b for a, b in zip(r[:4], outs))
    Xs2, _, _, _, ids2, perm2 = t.particle_sort(X, V, VP, AP)
    assert torch.equal(r[4], ids2) and torch.equal(r[5], perm2) and torch.equal(_bits(r[0]), _bits(Xs2))
