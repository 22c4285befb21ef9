"""Point-particle step (Sec. 2.3, point-like particles; test infrastructure).

Plain FP64 per particle, in this order:
1. host leaf by Algorithm 1 (``Tree.locate``) and its level l;
2. fluid velocity u at the particle by trilinear interpolation at level l:
   nodes are the level-l cells i0, i0 + 1 per axis around s = x 2^l - 1/2
   (i0 = floor(s), weights 1 - t and t, t = s - i0); each node's value is read
   from the leaf that contains the node's centre (the same reading as the
   delta-function stencil; parity unpinned where the 8 nodes cross a level
   jump, which the paper does not spell out: the pins hold constants on
   adaptive trees and linear fields on uniform ones); periodic wrap, or
   nodes outside a walled domain dropped with their weight;
3. particle Reynolds number Re = 2 r_p |u - v| / nu, drag correction
   f = 1 + 0.15 Re^0.687, acceleration
   a = f (u - v) / tau + (1 - rho_f / rho_p) g,  tau = 2 rho_p r_p^2 / (9 rho_f nu)
   (the momentum balance divided by m_p = 4/3 pi r_p^3 rho_p, mu = rho_f nu);
4. time step of the host level, dt_l = dt0 / 2^(l - l_min) (each finer level
   takes two sub-steps of its parent);
5. second-order Adams-Bashforth for velocity and position,
   v+ = v + dt_l (3/2 a - 1/2 a_prev),  x+ = x + dt_l (3/2 v - 1/2 v_prev),
   or forward Euler on the first step; x+ wrapped into the periodic cube;
6. the new host by Algorithm 1.
Reading: everything is in physical units.  The paper stores accelerations in
the lattice units of the host level and rescales the previous one when a
particle changes level (a_c = 2 a_f); with acoustic scaling
(dx and dt both halve per level) a lattice acceleration is a dt^2/dx, so that
rescale is exactly the unit change, and in physical units the previous
acceleration carries over unchanged.  Velocities need no rescale (v dt/dx is
level independent).  Only the tests and bench.py's oracle leg use this module.
"""
from __future__ import annotations

import numpy as np


def trilinear(tree, field, pos):
    """Fluid velocity at each point by trilinear interpolation at its host level."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    field = np.asarray(field, dtype=np.float64).reshape(tree.n_leaves, 3)
    ids = tree.locate(pos)
    out = np.zeros_like(pos)
    for k in range(pos.shape[0]):
        if ids[k] < 0:
            continue
        l = int(tree.levels[ids[k]])
        M = 1 << l
        s = pos[k] * M - 0.5
        i0 = np.floor(s)
        t = s - i0
        for ox in (0, 1):
            for oy in (0, 1):
                for oz in (0, 1):
                    c = i0 + np.array([ox, oy, oz])
                    if tree.periodic:
                        c = np.mod(c, M)
                    elif np.any(c < 0) or np.any(c >= M):
                        continue                      # node outside the walls: dropped
                    w = ((t[0] if ox else 1 - t[0]) * (t[1] if oy else 1 - t[1]) * (t[2] if oz else 1 - t[2]))
                    leaf = tree.locate(((c + 0.5) / M)[None, :])[0]
                    out[k] += w * field[leaf]
    return out


def acceleration(u, v, r_p, rho_p, rho_f, nu, g):
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    rel = u - v
    re = 2.0 * r_p * np.linalg.norm(rel, axis=-1) / nu
    f = 1.0 + 0.15 * re ** 0.687
    tau = 2.0 * rho_p * r_p ** 2 / (9.0 * rho_f * nu)
    return f[..., None] * rel / tau + (1.0 - rho_f / rho_p) * np.asarray(g, dtype=np.float64)


def step(tree, field, pos, vel, vel_prev, acc_prev, dt0, r_p, rho_p, rho_f, nu, g, first: bool = False):
    """One step of every particle by its own level's dt.  Returns
    (pos, vel, vel_prev, acc_prev, ids) after the step (vel_prev/acc_prev are
    the values the next step needs: this step's v and a)."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    ids = tree.locate(pos)
    u = trilinear(tree, field, pos)
    a = acceleration(u, vel, r_p, rho_p, rho_f, nu, g)
    lev = np.where(ids >= 0, tree.levels[np.maximum(ids, 0)].astype(np.int64), tree.l_min)
    dt = dt0 / np.ldexp(1.0, lev - tree.l_min)
    dt = np.where(ids >= 0, dt, 0.0)[:, None]           # a particle with no host stays put
    if first:
        v_new = vel + dt * a
        x_new = pos + dt * vel
    else:
        v_new = vel + dt * (1.5 * a - 0.5 * acc_prev)
        x_new = pos + dt * (1.5 * vel - 0.5 * vel_prev)
    if tree.periodic:
        x_new = np.mod(x_new, 1.0)
    return x_new, v_new, np.array(vel, dtype=np.float64), a, tree.locate(x_new)
