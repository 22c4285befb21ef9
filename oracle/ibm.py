"""Multi-direct forcing of the immersed-boundary method (test infrastructure).

Plain FP64 composition of the oracle's interpolation and spreading, in the
order of the IBM subsection of Sec. 2.2: each iteration interpolates the
current leaf velocity to the markers, forms the marker force from the slip
against the prescribed marker velocity, spreads it back, and corrects the
leaf velocity.  Only the tests, ``__graft_entry__.smoke()`` and ``bench.py``'s
oracle leg use it.

Readings (the paper gives the steps, not these details):
- the interpolation and spreading weights are the oracle's (no cell-volume
  factor: the (dx)^D of the sums cancels W's 1/dx^D);
- the velocity correction is u <- u + F/rho exactly as printed, with dt only
  inside the marker force F_k = (U_k - u_k)/dt;
- each iteration starts from the previous iteration's corrected velocity, and
  the forces of all iterations are summed (the total forcing applied in the
  time step).
"""
from __future__ import annotations

import numpy as np


def mdf(tree, field, pos, target, n_iter: int, dt: float = 1.0, rho: float = 1.0):
    """Returns (u, F_lag, F_eul): the corrected leaf velocity (n_leaves, 3),
    the marker forces summed over the iterations (n, 3) and the spread forces
    summed over the iterations (n_leaves, 3)."""
    u = np.array(field, dtype=np.float64, copy=True).reshape(tree.n_leaves, 3)
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    target = np.asarray(target, dtype=np.float64).reshape(-1, 3)
    f_lag = np.zeros_like(target)
    f_eul = np.zeros_like(u)
    for _ in range(n_iter):
        u_k = tree.interpolate(u, pos)           # interpolation to the markers
        F_k = (target - u_k) / dt                # marker force from the slip
        f = tree.spread(F_k, pos)                # spreading to the leaves
        u = u + f / rho                          # velocity correction
        f_lag += F_k
        f_eul += f
    return u, f_lag, f_eul
