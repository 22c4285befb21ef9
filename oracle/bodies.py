"""Per-body sums of the IBM coupling (test infrastructure).

For each body b, a contiguous segment of points k (its surface markers, or
the Lagrangian points placed inside it), plain FP64 loops give

    S_b = sum_k v_k dV_k               M_b = sum_k (X_k - x_b) x v_k dV_k

With v = F_k (marker forces) these are the IBM force and torque on the body
up to sign, F^ibm = -S and T^ibm = -M; with v = u(X_in) at interior points
they are the linear and angular momentum of the enclosed fluid (times rho_f)
whose rates of change correct F^ibm and T^ibm (Sec. 2.3, fully resolved
bodies).  Reading: the text attaches the names L and P the other way round
from the equations they enter; here the sum of v is the linear momentum and
the sum of r x v the angular one, as in the force and torque balances.  In a
periodic unit cube X_k - x_b is taken as the nearest periodic image.
Only the tests and bench.py's oracle leg use this module.
"""
from __future__ import annotations

import numpy as np


def body_sums(vec, pos, offsets, centres, dV, periodic: bool = True):
    """vec, pos: (n, 3); offsets: (n_body + 1,) ascending; centres:
    (n_body, 3); dV: scalar or (n,) volume elements.  Returns (S, M), each
    (n_body, 3)."""
    vec = np.asarray(vec, dtype=np.float64).reshape(-1, 3)
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    centres = np.asarray(centres, dtype=np.float64).reshape(-1, 3)
    n = pos.shape[0]
    dv = np.broadcast_to(np.asarray(dV, dtype=np.float64), (n,))
    nb = len(offsets) - 1
    S = np.zeros((nb, 3))
    M = np.zeros((nb, 3))
    for b in range(nb):
        for k in range(int(offsets[b]), int(offsets[b + 1])):
            r = [pos[k, d] - centres[b, d] for d in range(3)]
            if periodic:
                r = [x - np.floor(x + 0.5) for x in r]      # nearest image
            v = vec[k] * dv[k]
            S[b] += v
            M[b] += np.array([r[1] * v[2] - r[2] * v[1],
                              r[2] * v[0] - r[0] * v[2],
                              r[0] * v[1] - r[1] * v[0]])
    return S, M
