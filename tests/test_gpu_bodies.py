"""GPU per-body sums (ot_body_sums) against the FP64 oracle (oracle/bodies.py).

Both sum in FP64 (the GPU in a fixed tree order, the oracle serially), so the
bound is 1e-12 of the absolute sums (sum |v dV| and sum |r||v dV|).  The rigid
-motion identities are checked on the GPU too, and repeated calls must agree
bit for bit.
"""
import numpy as np
import pytest
import torch

import synth
from gpu_util import as_dtype, to_dev
from oracle.bodies import body_sums as orc_body_sums

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ot():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2605_20565_amd as m
    return m


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("per_point_dv", [False, True])
def test_body_sums_match_oracle_workload2_markers(ot, dtype, per_point_dv):
    w = synth.workload(2, scale=0.01)
    nb = sum(1 for k in w.kinds if k == "markers")
    offs = np.asarray(w.instances[:nb + 1], dtype=np.int64)
    n = int(offs[-1])
    pos = as_dtype(w.points[:n], dtype)
    vec = as_dtype(w.forces[:n], dtype)
    cen = as_dtype(np.array([s.centre for s in w.spheres]), dtype)
    rng = np.random.default_rng(4)
    dv = as_dtype(rng.random(n), dtype) if per_point_dv else 0.37
    S, M = orc_body_sums(vec, pos, offs, cen, dv)
    r = pos - np.repeat(cen, np.diff(offs), axis=0)
    r -= np.floor(r + 0.5)
    a = np.abs(vec) * (dv[:, None] if per_point_dv else dv)
    sS = np.add.reduceat(a, offs[:-1], axis=0)
    sM = np.add.reduceat(a * np.linalg.norm(r, axis=1)[:, None], offs[:-1], axis=0)
    g_dv = to_dev(dv, dtype) if per_point_dv else 0.37
    Sg, Mg = ot.body_sums(to_dev(vec, dtype), to_dev(pos, dtype), offs, to_dev(cen, dtype), g_dv)
    assert (np.abs(Sg.cpu().numpy() - S) <= 1e-12 * sS).all()
    assert (np.abs(Mg.cpu().numpy() - M) <= 1e-12 * sM + 1e-300).all()
    Sg2, Mg2 = ot.body_sums(to_dev(vec, dtype), to_dev(pos, dtype), offs, to_dev(cen, dtype), g_dv)
    assert torch.equal(Sg, Sg2) and torch.equal(Mg, Mg2)


def test_body_sums_rigid_motion_on_gpu(ot):
    c = np.array([0.97, 0.5, 0.03])                     # wraps around two faces
    h = 1.0 / 64
    m = 6
    g = np.arange(-m, m + 1) * h
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    r = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    r = r[(r * r).sum(axis=1) <= (m * h) ** 2]
    pos = np.mod(c + r, 1.0)
    v, om = np.array([0.3, -0.1, 0.2]), np.array([1.0, 2.0, -0.5])
    u = v + np.cross(om, r)
    dV = h ** 3
    Sg, Mg = ot.body_sums(to_dev(u, torch.float64), to_dev(pos, torch.float64), [0, len(pos)],
                          to_dev(c[None, :], torch.float64), dV)
    inertia = dV * ((r * r).sum() * np.eye(3) - r.T @ r)
    np.testing.assert_allclose(Sg.cpu().numpy()[0], v * dV * len(pos), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(Mg.cpu().numpy()[0], inertia @ om, rtol=1e-10, atol=1e-16)
