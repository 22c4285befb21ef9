"""Property tests of the HIP path against the FP64 oracle on drawn trees
(hypothesis): random partitions (balanced or not, periodic or walled, one to
three levels below l_min) and adversarial points (dyadic faces, edges and
corners, 0, 1 - ulp, outside the cube, NaN).  Host ids must match bit for
bit; interpolation within the scaled tolerance; FIXED spreading within its
bound; and a sorted batched plan must equal the plain fused launch bit for
bit (FIXED sums do not depend on the order)."""
import math

import numpy as np
import pytest
import torch
from hypothesis import HealthCheck, given, settings, strategies as st

import synth
from gpu_util import TOL, as_dtype, fixed_point_quantum, gpu_tree, oracle_tree, scaled_err, spread_excess, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ot():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2605_20565_amd as m
    return m


def _points(rng, l_max, n):
    g = rng.integers(0, 1 << l_max, (n, 3)) * math.ldexp(1.0, -l_max)
    mix = rng.random((n, 3))
    m = rng.random((n, 3)) < 0.5
    mix[m] = g[m]
    odd = np.array([[0.0, 0.0, 0.0], [np.nextafter(1.0, 0.0)] * 3, [1.0, 0.5, 0.5], [-1e-9, 0.5, 0.5],
                    [0.5, 1.25, -0.5], [np.nan, 0.5, 0.5]])
    return np.concatenate([rng.random((n, 3)), g, mix, odd])


@settings(max_examples=25, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(seed=st.integers(0, 2 ** 32 - 1), l_min=st.integers(0, 3), depth=st.integers(1, 3),
       p_refine=st.floats(0.05, 0.5), periodic=st.booleans(), balance=st.booleans(), f64=st.booleans())
def test_fuzz_drawn_trees_against_oracle(ot, seed, l_min, depth, p_refine, periodic, balance, f64):
    dtype = torch.float64 if f64 else torch.float32
    rng = np.random.default_rng(seed)
    spec = synth.random_tree(l_min, l_min + depth, rng, p_refine=p_refine, periodic=periodic, balance=balance)
    t, o = gpu_tree(spec), oracle_tree(spec)
    pts = as_dtype(_points(rng, spec.l_max, 200), dtype)
    frc = as_dtype(rng.standard_normal(pts.shape), dtype)
    fld = as_dtype(rng.standard_normal((spec.n_leaves, 3)), dtype)
    P, F, Fd = to_dev(pts, dtype), to_dev(frc, dtype), to_dev(fld, dtype)
    ids, vel, fo = t.track(P, field=Fd, force=F, mode="fixed")
    assert np.array_equal(ids.cpu().numpy().astype(np.int64), o.locate(pts))
    U, S = o.interpolate(fld, pts, with_scale=True)
    assert scaled_err(vel.cpu().numpy(), U, S) <= TOL[dtype]
    f, Sf, cnt, A = o.spread(frc, pts, with_scale=True)
    assert spread_excess(fo.cpu().numpy(), f, Sf, A, cnt, dtype, fixed_point_quantum(frc)) <= 1.0
    # the sorted batched pass over two uneven instances equals the plain launch
    n = P.shape[0]
    plan = ot.BatchPlan(t, [0, n // 3, n], [7, 7], dtype=dtype, mode="fixed", sort_points=True)
    ids_b = torch.empty_like(ids)
    vel_b = torch.empty_like(vel)
    fo_b = torch.empty_like(fo)
    plan.run(P, field=Fd, force=F, ids=ids_b, vel=vel_b, field_out=fo_b)
    torch.cuda.synchronize()
    assert torch.equal(ids_b, ids)
    assert torch.equal(vel_b, vel)
    assert torch.equal(fo_b, fo)
    plan.close()
