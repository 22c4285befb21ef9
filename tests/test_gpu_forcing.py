"""GPU mean IBM-force subtraction (Sec. 5.2) against the oracle: the
volume-weighted domain average of a leaf field within 1e-12 of sum |F| |cell|
(both precisions sum in FP64), the subtracted field element by element at
the stated tolerance, the same bits on every run; and on a uniform periodic
tree the mean of spread forces is 2^-3l sum F (each point's weights sum to 1)."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import TOL, as_dtype, fixed_point_quantum, gpu_tree, to_dev
from oracle.forcing import volume_mean

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ot():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2605_20565_amd as m
    return m


def _check(ot, spec, t, dtype, seed):
    rng = np.random.default_rng(seed)
    f = as_dtype(rng.standard_normal((spec.n_leaves, 3)) * 3 + rng.standard_normal(3), dtype)
    # leaf rows in id order: the oracle needs the levels in the same order
    _, lv = t.leaves()
    levels = lv.cpu().numpy().astype(np.int64)
    want = volume_mean(f, levels)
    F = to_dev(f, dtype)
    m1 = t.force_mean(F.clone(), subtract=False)
    G = F.clone()
    m2 = t.force_mean(G, subtract=True)
    torch.cuda.synchronize()
    assert torch.equal(m1, m2)                                     # same bits on every run
    scale = (np.abs(f) * np.ldexp(1.0, -3 * levels)[:, None]).sum(axis=0)
    assert np.all(np.abs(m1.cpu().numpy() - want) <= 1e-12 * scale)
    g = G.cpu().double().numpy()
    assert np.all(np.abs(g - (f - want)) <= TOL[dtype] * (np.abs(f) + np.abs(want)) + 1e-12 * scale)
    # the subtracted field has (close to) zero mean
    m3 = t.force_mean(G.clone(), subtract=False).cpu().numpy()
    assert np.all(np.abs(m3) <= 4 * TOL[dtype] * scale)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_force_mean_band_tree(ot, dtype):
    spec = synth.band_tree(4, 7, [synth.Sphere((0.5, 0.45, 0.5), 0.2)], periodic=True, seed=6)
    _check(ot, spec, gpu_tree(spec), dtype, 1)


def test_force_mean_workload2_tree(ot):
    w = synth.workload(2, scale=0.01)
    _check(ot, w.tree, gpu_tree(w.tree), torch.float32, 2)


def test_mean_of_spread_forces_on_uniform_tree(ot):
    spec = synth.uniform_tree(5, seed=3)
    t = gpu_tree(spec)
    rng = np.random.default_rng(4)
    pts = as_dtype(rng.random((5000, 3)), torch.float64)
    frc = as_dtype(rng.standard_normal((5000, 3)), torch.float64)
    fo = t.spread(to_dev(frc, torch.float64), to_dev(pts, torch.float64), mode="fixed")
    m = t.force_mean(fo, subtract=True).cpu().numpy()
    q = fixed_point_quantum(frc)
    want = np.ldexp(frc.sum(axis=0), -15)
    assert np.all(np.abs(m - want) <= 27 * 5000 * q * np.ldexp(1.0, -15) + 1e-13 * np.abs(frc).sum(axis=0))
    assert float(fo.sum(dim=0).abs().max()) <= 1e-9


def test_force_mean_given_workspace_and_errors(ot):
    spec = synth.uniform_tree(3, seed=1)
    t = gpu_tree(spec)
    f = torch.randn((t.n_leaves, 3), dtype=torch.float64, device="cuda")
    work = torch.empty(int(ot.lib.ot_force_mean_workspace_bytes()), dtype=torch.uint8, device="cuda")
    mean = torch.empty(3, dtype=torch.float64, device="cuda")
    ot._check(ot.lib.ot_force_mean(t.handle, ot._ptr(f), ot.OT_F64, 0, ot._ptr(mean), ot._ptr(work), ot._stream()))
    torch.cuda.synchronize()
    assert torch.allclose(mean, f.mean(dim=0), rtol=1e-13, atol=1e-15)
    assert ot.lib.ot_force_mean(t.handle, None, ot.OT_F64, 0, ot._ptr(mean), None, None) == -1
    assert ot.lib.ot_force_mean(None, ot._ptr(f), ot.OT_F64, 0, ot._ptr(mean), None, None) == -1
