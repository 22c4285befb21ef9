"""Pins of the oracle's per-body sums (force/torque and enclosed momenta of
Sec. 2.3) against rigid-body identities that hold exactly for any lattice:

- a rigid velocity v + w x r sampled at points symmetric about the centre
  (sum r = 0) has linear momentum v sum dV;
- its angular momentum is I w with I = sum (|r|^2 Id - r r^T) dV, the inertia
  tensor formed independently;
- sums do not change when the body is moved across the periodic boundary
  (nearest image), and split into the sums of their segments.
A wrong sign or index in the cross product, a missing dV, or no nearest-image
rule breaks one of these.
"""
import numpy as np

from oracle.bodies import body_sums


def _lattice_in_sphere(centre, radius, h):
    m = int(np.ceil(radius / h))
    g = np.arange(-m, m + 1) * h
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    r = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    r = r[(r * r).sum(axis=1) <= radius * radius]          # symmetric under r -> -r
    return np.asarray(centre) + r, r


def test_rigid_motion_momenta():
    c = np.array([0.4, 0.55, 0.6])
    pos, r = _lattice_in_sphere(c, 0.1, 1.0 / 64)
    v, w = np.array([0.3, -0.1, 0.2]), np.array([1.0, 2.0, -0.5])
    u = v + np.cross(w, r)
    dV = (1.0 / 64) ** 3
    S, M = body_sums(u, pos, [0, len(pos)], [c], dV)
    np.testing.assert_allclose(S[0], v * dV * len(pos), rtol=1e-12, atol=1e-15)
    inertia = dV * ((r * r).sum() * np.eye(3) - r.T @ r)
    np.testing.assert_allclose(M[0], inertia @ w, rtol=1e-11, atol=1e-16)


def test_periodic_wrap_and_segments():
    rng = np.random.default_rng(2)
    c = np.array([0.02, 0.97, 0.5])                         # straddles two periodic faces
    r = rng.normal(scale=0.03, size=(300, 3))
    pos = np.mod(c + r, 1.0)
    vec = rng.standard_normal((300, 3))
    dV = rng.random(300)
    S, M = body_sums(vec, pos, [0, 300], [c], dV)
    S2, M2 = body_sums(vec, np.mod(pos - c + 0.5, 1.0), [0, 300], [[0.5, 0.5, 0.5]], dV)
    np.testing.assert_allclose(S, S2, rtol=1e-13)
    np.testing.assert_allclose(M, M2, rtol=1e-9, atol=1e-13)
    # two segments sum to the whole, with each segment's own centre
    Sa, Ma = body_sums(vec, pos, [0, 120, 300], [c, c], dV)
    np.testing.assert_allclose(Sa.sum(axis=0), S[0], rtol=1e-13)
    np.testing.assert_allclose(Ma.sum(axis=0), M[0], rtol=1e-12, atol=1e-15)
