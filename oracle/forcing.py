"""Mean IBM-force subtraction (test infrastructure; Sec. 5.2, the equation
that removes the domain average of the IBM forcing in a periodic box).

The forcing field lives on the leaves of the adaptive tree, one value per
leaf, constant over the leaf's cube.  Its spatial average over the whole
domain Pi (the unit cube, |V_Pi| = 1) is then

    <F>_Pi = (1 / |V_Pi|) sum_j F_j |cell_j|,    |cell_j| = 2^(-3 l_j),

and the compensated forcing is F_j - <F>_Pi on every leaf.  Reading: the
integral of the leaf field is that of its piecewise-constant extension (the
leaves tile the cube, so the sum is over the partition).  The library's
spreading returns sum_k w F_k per leaf (no cell-volume factor); it is a force
density when the caller pre-scales each F_k by dV_k / dx_l^3, and this mean
is taken of whatever leaf field is given.

Each mean is the correctly rounded value of the exact sum: the products
F_j 2^(-3 l_j) are exact in FP64 (a power-of-two scaling) and math.fsum adds
them without intermediate rounding.  Only the tests and bench.py's oracle
leg use this module.
"""
from __future__ import annotations

import math

import numpy as np


def volume_mean(field, levels):
    """<F>_Pi of a leaf field (n_leaves, 3) given the leaf levels (n_leaves,)."""
    f = np.asarray(field, dtype=np.float64).reshape(-1, 3)
    vol = np.ldexp(1.0, -3 * np.asarray(levels, dtype=np.int64))
    return np.array([math.fsum((f[:, c] * vol).tolist()) for c in range(3)])


def subtract_mean(field, levels):
    """(F - <F>_Pi, <F>_Pi)."""
    m = volume_mean(field, levels)
    return np.asarray(field, dtype=np.float64).reshape(-1, 3) - m, m
