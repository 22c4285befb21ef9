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
