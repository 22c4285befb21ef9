"""Pins of the oracle's multi-direct forcing (IBM subsection of Sec. 2.2).

On a uniform grid the weights of one marker satisfy sum_n w_n^2 =
(sum_o phi(r_o)^2)^3 = 1/8 for every position (the 3-point kernel is built so
that sum phi^2 = 1/2).  One forcing iteration with marker force (U - u_k)/dt
and correction u += f/rho therefore changes the interpolated marker velocity
by (U - u_k) / (8 dt rho): the slip of a lone marker decays by the factor
1 - 1/(8 dt rho) per iteration, exactly.  Markers whose stencils do not
overlap decay independently.  The spread forces of every iteration sum to the
marker forces (partition of unity).  A dropped term, a wrong sign, a missing
dt or rho, or a correction that does not feed the next iteration breaks one of
these.
"""
import numpy as np
import pytest

import synth


def _tree(orc, spec):
    return orc.Tree.from_anchors(spec.anchors, spec.levels, spec.l_min, spec.l_max, spec.periodic)


def _ibm():
    from oracle import ibm
    return ibm


@pytest.mark.parametrize("dt,rho", [(1.0, 1.0), (2.0, 1.5), (0.5, 4.0)])
def test_lone_marker_slip_decays_geometrically(orc, dt, rho):
    t = _tree(orc, synth.uniform_tree(4, seed=3))
    rng = np.random.default_rng(11)
    pos = rng.random((1, 3))
    field = rng.standard_normal((t.n_leaves, 3))
    target = np.array([[1.0, -2.0, 0.5]])
    slip0 = target - t.interpolate(field, pos)
    q = 1.0 - 1.0 / (8.0 * dt * rho)
    for m in range(0, 6):
        u, _, _ = _ibm().mdf(t, field, pos, target, m, dt, rho)
        slip = target - t.interpolate(u, pos)
        np.testing.assert_allclose(slip, slip0 * q ** m, rtol=1e-12, atol=1e-12)


def test_distant_markers_decay_independently(orc):
    t = _tree(orc, synth.uniform_tree(5, seed=1))
    # stencils 3 cells wide; markers 8 cells apart on a 32^3 periodic grid
    pos = np.array([[0.11, 0.13, 0.17], [0.36, 0.41, 0.43], [0.61, 0.62, 0.68]])
    field = np.zeros((t.n_leaves, 3))
    target = np.array([[1.0, 0.0, 0.0], [0.0, 2.0, 0.0], [0.5, 0.5, -1.0]])
    u, f_lag, _ = _ibm().mdf(t, field, pos, target, 4)
    slip = target - t.interpolate(u, pos)
    np.testing.assert_allclose(slip, target * (7.0 / 8.0) ** 4, rtol=1e-12, atol=1e-13)
    # marker force summed over iterations: sum_m (7/8)^m U
    np.testing.assert_allclose(f_lag, target * sum((7.0 / 8.0) ** m for m in range(4)), rtol=1e-12)


def test_forces_conserved_each_iteration_adaptive(orc):
    sphere = synth.Sphere((0.5, 0.5, 0.5), 0.2)
    t = _tree(orc, synth.band_tree(3, 5, [sphere], seed=2))
    pos = synth.fibonacci_sphere(sphere, 400)
    rng = np.random.default_rng(5)
    field = rng.standard_normal((t.n_leaves, 3))
    target = rng.standard_normal(pos.shape)
    u, f_lag, f_eul = _ibm().mdf(t, field, pos, target, 3, dt=0.7, rho=1.3)
    np.testing.assert_allclose(f_eul.sum(axis=0), f_lag.sum(axis=0), rtol=1e-11, atol=1e-10)
    # and the velocity change is the spread force over rho
    np.testing.assert_allclose(u - field, f_eul / 1.3, rtol=1e-12, atol=1e-12)


def test_zero_iterations_is_identity(orc):
    t = _tree(orc, synth.uniform_tree(3, seed=0))
    field = np.random.default_rng(0).standard_normal((t.n_leaves, 3))
    u, f_lag, f_eul = _ibm().mdf(t, field, np.array([[0.3, 0.3, 0.3]]), np.ones((1, 3)), 0)
    assert np.array_equal(u, field) and not f_lag.any() and not f_eul.any()
