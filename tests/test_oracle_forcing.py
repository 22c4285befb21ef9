"""Pins of the oracle's mean IBM-force subtraction (Sec. 5.2): the domain
average of a leaf field weights each leaf by its cube's volume 2^-3l.

- a constant field has itself as mean and vanishes after subtraction;
- after subtraction the volume-weighted sum is zero;
- on a uniform tree the mean is the plain arithmetic mean;
- a hand-built two-level tree gives the volume weights 1/8 and 1/64 by hand;
- subtracting again changes nothing beyond rounding (the mean is now zero).
A missing volume factor, a wrong level exponent or a per-leaf instead of a
volume average breaks one of these."""
import numpy as np
import pytest

import synth
from oracle.forcing import subtract_mean, volume_mean


def _band():
    return synth.band_tree(3, 6, [synth.Sphere((0.4, 0.5, 0.6), 0.2)], periodic=True, seed=4)


def test_constant_field_has_zero_remainder():
    spec = _band()
    c = np.array([0.3, -1.25, 7.0])
    f = np.tile(c, (spec.n_leaves, 1))
    g, m = subtract_mean(f, spec.levels)
    np.testing.assert_allclose(m, c, rtol=1e-15)
    assert np.abs(g).max() <= 8 * np.finfo(float).eps * np.abs(c).max()


def test_volume_weighted_sum_vanishes_after_subtraction():
    spec = _band()
    rng = np.random.default_rng(3)
    f = rng.standard_normal((spec.n_leaves, 3)) * 5 + 2
    g, m = subtract_mean(f, spec.levels)
    vol = np.ldexp(1.0, -3 * spec.levels.astype(np.int64))
    assert abs(vol.sum() - 1.0) < 1e-15              # the leaves tile the cube
    s = (g * vol[:, None]).sum(axis=0)
    assert np.abs(s).max() <= 1e-13 * (np.abs(f) * vol[:, None]).sum()
    # the mean differs from the plain per-leaf average on an adaptive tree
    assert np.abs(m - f.mean(axis=0)).max() > 1e-3


def test_uniform_tree_mean_is_arithmetic_mean():
    spec = synth.uniform_tree(4, seed=2)
    rng = np.random.default_rng(5)
    f = rng.standard_normal((spec.n_leaves, 3))
    np.testing.assert_allclose(volume_mean(f, spec.levels), f.mean(axis=0), rtol=1e-13, atol=1e-16)


def test_hand_built_two_level_tree():
    # the root split once (8 leaves of level 1), one of them split again (8 of level 2)
    levels = np.array([1] * 7 + [2] * 8)
    f = np.zeros((15, 3))
    f[:7, 0] = 8.0          # 7 * 8 * (1/8) = 7
    f[7:, 0] = 64.0         # 8 * 64 * (1/64) = 8
    f[3, 1] = 1.0           # 1/8
    f[9, 2] = -2.0          # -2/64
    np.testing.assert_array_equal(volume_mean(f, levels), [15.0, 0.125, -0.03125])


def test_subtracting_twice_changes_nothing():
    spec = _band()
    rng = np.random.default_rng(8)
    f = rng.standard_normal((spec.n_leaves, 3)) + 3
    g, _ = subtract_mean(f, spec.levels)
    h, m2 = subtract_mean(g, spec.levels)
    assert np.abs(m2).max() <= 1e-15 * np.abs(f).max()
    assert np.abs(h - g).max() <= 1e-15 * np.abs(f).max()
