"""Pins of the oracle's point-particle step (Sec. 2.3, point-like particles).

- Trilinear interpolation reproduces linear fields exactly away from walls
  on a uniform grid, and constants on an adaptive tree (weights sum to 1).
- With drag negligible (huge particle density) the acceleration is the
  constant g: AB2 after one Euler step gives v exactly linear in time and
  x = x0 + v0 t + g t^2 / 2 - h^2 g / 2 (the Euler start's offset).
- The step of a particle is dt0 / 2^(l - l_min) of its host level.
- In still fluid the velocity converges to the terminal velocity where
  drag balances buoyancy, f(Re) |v| / tau = (1 - rho_f/rho_p) g, solved here
  by bisection.
"""
import numpy as np
import pytest

import synth
from oracle import particles as pp


def _tree(orc, spec):
    return orc.Tree.from_anchors(spec.anchors, spec.levels, spec.l_min, spec.l_max, spec.periodic)


def test_trilinear_exact_for_linear_fields(orc):
    spec = synth.uniform_tree(4, seed=1, periodic=False)
    t = _tree(orc, spec)
    c = synth.leaf_centres(spec)[t.perm]                  # leaf centres in Morton (id) order
    A = np.array([[1.0, -2.0, 0.5], [0.3, 0.0, 1.5], [-1.0, 2.0, 0.25]])
    b = np.array([0.1, -0.2, 0.3])
    field = c @ A.T + b
    rng = np.random.default_rng(0)
    pos = 1.0 / 16 + rng.random((200, 3)) * (1.0 - 2.0 / 16)   # at least half a cell from the walls
    np.testing.assert_allclose(pp.trilinear(t, field, pos), pos @ A.T + b, rtol=1e-12, atol=1e-12)


def test_trilinear_reproduces_constants_adaptive(orc):
    sphere = synth.Sphere((0.5, 0.5, 0.5), 0.2)
    t = _tree(orc, synth.band_tree(3, 5, [sphere], seed=2))
    pos = np.random.default_rng(3).random((300, 3))
    field = np.tile([1.5, -0.5, 2.0], (t.n_leaves, 1))
    np.testing.assert_allclose(pp.trilinear(t, field, pos), np.tile([1.5, -0.5, 2.0], (300, 1)), rtol=1e-13)


def test_ab2_exact_under_constant_acceleration(orc):
    t = _tree(orc, synth.uniform_tree(3, seed=0))
    g = np.array([0.0, 0.0, -9.81])
    x0 = np.array([[0.3, 0.4, 0.9]])
    v0 = np.array([[0.02, -0.01, 0.0]])
    h, steps = 1e-3, 20
    kw = dict(r_p=1e-4, rho_p=1e12, rho_f=1.0, nu=1e-6, g=g)
    x, v, vp, ap = x0, v0, v0.copy(), np.zeros((1, 3))
    for m in range(steps):
        x, v, vp, ap, _ = pp.step(t, np.zeros((t.n_leaves, 3)), x, v, vp, ap, h, first=(m == 0), **kw)
    T = steps * h
    np.testing.assert_allclose(v, v0 + g * T, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(x, np.mod(x0 + v0 * T + 0.5 * g * T * T - 0.5 * h * h * g, 1.0), rtol=1e-9, atol=1e-12)


def test_step_follows_host_level(orc):
    sphere = synth.Sphere((0.5, 0.5, 0.5), 0.2)
    spec = synth.band_tree(3, 5, [sphere], seed=2)
    t = _tree(orc, spec)
    pos = np.array([[0.7, 0.5, 0.5], [0.05, 0.05, 0.05]])   # on the band (level 5), far from it (level 3)
    lev = t.levels[t.locate(pos)]
    assert list(lev) == [5, 3]
    v = np.array([[1e-3, 0, 0], [1e-3, 0, 0]])
    kw = dict(r_p=1e-4, rho_p=1e12, rho_f=1.0, nu=1e-6, g=np.zeros(3))
    x, *_ = pp.step(t, np.zeros((t.n_leaves, 3)), pos, v, v, np.zeros((2, 3)), 0.01, first=True, **kw)
    dx = x[:, 0] - pos[:, 0]
    np.testing.assert_allclose(dx, [0.01 / 4 * 1e-3, 0.01 * 1e-3], rtol=1e-9)   # x+ - x cancels digits


def test_terminal_velocity(orc):
    t = _tree(orc, synth.uniform_tree(2, seed=0))
    r_p, rho_p, rho_f, nu, g = 2e-4, 2.5, 1.0, 1e-5, 9.81
    tau = 2 * rho_p * r_p ** 2 / (9 * rho_f * nu)
    rhs = (1 - rho_f / rho_p) * g
    lo, hi = 0.0, rhs * tau                      # Stokes velocity bounds the corrected one from above
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        re = 2 * r_p * mid / nu
        if (1 + 0.15 * re ** 0.687) * mid / tau < rhs:
            lo = mid
        else:
            hi = mid
    vt = 0.5 * (lo + hi)
    x = np.array([[0.5, 0.5, 0.5]])
    v = np.zeros((1, 3))
    vp, ap = v.copy(), np.zeros((1, 3))
    for m in range(400):
        x, v, vp, ap, _ = pp.step(t, np.zeros((t.n_leaves, 3)), x, v, vp, ap, tau / 20, r_p=r_p, rho_p=rho_p,
                                  rho_f=rho_f, nu=nu, g=np.array([0, 0, -g]), first=(m == 0))
    np.testing.assert_allclose(v[0], [0, 0, -vt], rtol=1e-9, atol=1e-12)
