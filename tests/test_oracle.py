"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
3-point delta formula gives by hand, the design conditions of that kernel,
hand-worked host ids on a hand-built tree, the linear containment scan,
a recursive construction of the Z-order, the textbook uniform-grid IBM
interpolation, and conservation / adjoint / finite-difference identities.
"""
import math
import os

import numpy as np
import pytest

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append([float(v) for v in line.split()])
    return np.asarray(rows)


def _phi_np(r):
    """The phi equation of Sec. 2.2 (independent numpy transcription used only
    as the textbook side of the uniform-grid comparison)."""
    a = np.abs(r)
    inner = (1.0 + np.sqrt(np.clip(1.0 - 3.0 * r * r, 0.0, None))) / 3.0
    outer = (5.0 - 3.0 * a - np.sqrt(np.clip(-2.0 + 6.0 * a - 3.0 * r * r, 0.0, None))) / 6.0
    return np.where(a <= 0.5, inner, np.where(a <= 1.5, outer, 0.0))


def _tree(orc, spec):
    return orc.Tree.from_anchors(spec.anchors, spec.levels, spec.l_min, spec.l_max, spec.periodic)


# ---------------------------------------------------------------------------
# phi
# ---------------------------------------------------------------------------
def test_phi_printed_values(orc):
    for r, v in _golden("phi_values.txt"):
        assert orc.phi(r) == pytest.approx(v, abs=1e-15), r


def test_phi_design_conditions(orc):
    """Sum_i phi(r-i) = 1, sum_i (r-i) phi(r-i) = 0, sum_i phi(r-i)^2 = 1/2:
    the conditions the 3-point kernel is built from (any dropped term, sign
    or coefficient in either branch breaks one of them)."""
    rng = np.random.default_rng(0)
    for r in np.concatenate([rng.random(2000), [0.0, 0.5, 0.25, 0.999999]]):
        ds = [r - i for i in range(-2, 4)]
        ph = [orc.phi(d) for d in ds]
        assert sum(ph) == pytest.approx(1.0, abs=1e-14)
        assert sum(d * p for d, p in zip(ds, ph)) == pytest.approx(0.0, abs=1e-14)
        assert sum(p * p for p in ph) == pytest.approx(0.5, abs=1e-14)


def test_phi_symmetric_and_support(orc):
    for r in np.linspace(-2, 2, 801):
        assert orc.phi(r) == orc.phi(-r)
        assert orc.phi(r) >= 0.0
        if abs(r) >= 1.5:
            assert orc.phi(r) == 0.0


def test_dphi_matches_finite_differences(orc):
    h = 1e-6
    for r in np.linspace(-1.6, 1.6, 641):
        if min(abs(abs(r) - 0.5), abs(abs(r) - 1.5)) < 1e-3:
            continue
        fd = (orc.phi(r + h) - orc.phi(r - h)) / (2 * h)
        assert orc.dphi(r) == pytest.approx(fd, abs=1e-8), r


def test_dphi_continuous_and_moments(orc):
    # C^1: one-sided values agree at the branch points
    assert orc.dphi(0.5) == pytest.approx(-1.0, abs=1e-14)
    assert orc.dphi(0.5 + 1e-12) == pytest.approx(-1.0, abs=1e-5)
    assert orc.dphi(-0.5) == pytest.approx(1.0, abs=1e-14)
    assert orc.dphi(1.5 - 1e-12) == pytest.approx(0.0, abs=1e-5)
    rng = np.random.default_rng(1)
    for r in rng.random(500):
        ds = [r - i for i in range(-2, 4)]
        dp = [orc.dphi(d) for d in ds]
        assert sum(dp) == pytest.approx(0.0, abs=1e-13)                       # d/dr of sum phi
        assert sum(d * p for d, p in zip(ds, dp)) == pytest.approx(-1.0, abs=1e-13)  # d/dr of 1st moment
        assert sum(orc.phi(d) * p for d, p in zip(ds, dp)) == pytest.approx(0.0, abs=1e-13)


def _edge_phi_conjugate(eps):
    """phi(3/2 - eps) from the outer branch multiplied by its conjugate:
    (1/2 + 3 eps)^2 - (1/4 + 3 eps - 3 eps^2) = 12 eps^2, so
    phi = 2 eps^2 / (1/2 + 3 eps + sqrt(1/4 + 3 eps - 3 eps^2)), a form with no
    cancellation, evaluated here in 60-digit decimal arithmetic."""
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    e = Decimal(eps)
    return float(2 * e * e / (Decimal("0.5") + 3 * e + (Decimal("0.25") + 3 * e - 3 * e * e).sqrt()))


def _edge_dphi_conjugate(eps):
    """phi'(3/2 - eps) = -eps (7 - 6 eps + q) / (q (1 + q)), q = sqrt(1 + 12 eps - 12 eps^2),
    the derivative branch rewritten the same way (60-digit decimal)."""
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    e = Decimal(eps)
    q = (1 + 12 * e - 12 * e * e).sqrt()
    return float(-e * (7 - 6 * e + q) / (q * (1 + q)))


@pytest.mark.parametrize("k", [4, 10, 20, 30, 40, 50])
def test_phi_edge_of_support_relative_accuracy(orc, k):
    """Near |r| = 3/2 the printed outer branch cancels; evaluated in FP64 it is
    only ~2^-53 absolute (wrong in every digit for eps below ~2^-27).  The
    oracle evaluates it in binary128: FP64-relative precision plus about
    2^-113 absolute."""
    eps = 2.0 ** -k
    for r, sgn in ((1.5 - eps, 1.0), (-(1.5 - eps), -1.0)):
        want = _edge_phi_conjugate(eps)
        assert orc.phi(r) == pytest.approx(want, rel=4e-16, abs=2.0 ** -110), (k, r)
        dwant = sgn * _edge_dphi_conjugate(eps)
        assert orc.dphi(r) == pytest.approx(dwant, rel=4e-16, abs=2.0 ** -108), (k, r)


# ---------------------------------------------------------------------------
# Morton order
# ---------------------------------------------------------------------------
def test_morton_hand_values(orc):
    assert orc.morton_encode(1, 0, 0, 4) == 1
    assert orc.morton_encode(0, 1, 0, 4) == 2
    assert orc.morton_encode(0, 0, 1, 4) == 4
    assert orc.morton_encode(1, 1, 1, 4) == 7
    assert orc.morton_encode(2, 0, 0, 4) == 8
    # x=011, y=101, z=110 -> bit0 (1,1,0)=3, bit1 (1,0,1)=5, bit2 (0,1,1)=6 -> 3 + 5*8 + 6*64
    assert orc.morton_encode(3, 5, 6, 4) == 3 + 5 * 8 + 6 * 64
    rng = np.random.default_rng(2)
    for _ in range(200):
        x, y, z = (int(v) for v in rng.integers(0, 1 << 21, 3))
        assert orc.morton_decode(orc.morton_encode(x, y, z, 21), 21) == (x, y, z)


def _zorder_recursive(level):
    """Cells of a uniform level-`level` grid listed in Z-order by recursive
    octant subdivision (children visited x fastest, then y, then z)."""
    out = []

    def rec(x, y, z, l):
        if l == level:
            out.append((x, y, z))
            return
        for c in range(8):
            rec(2 * x + (c & 1), 2 * y + ((c >> 1) & 1), 2 * z + ((c >> 2) & 1), l + 1)

    rec(0, 0, 0, 0)
    return out


def test_uniform_tree_ids_follow_recursive_zorder(orc):
    for level in (1, 2, 3):
        spec = synth.uniform_tree(level, seed=level)
        tree = _tree(orc, spec)
        assert tree.check_partition() == 0
        order = _zorder_recursive(level)
        rank = {c: i for i, c in enumerate(order)}
        h = 1.0 / (1 << level)
        cells = np.array(order, dtype=np.float64)
        pts = (cells + 0.3) * h
        ids = tree.locate(pts)
        assert np.array_equal(ids, np.arange(len(order)))
        rng = np.random.default_rng(level)
        p = rng.random((500, 3))
        want = [rank[tuple(int(v) for v in np.floor(q * (1 << level)))] for q in p]
        assert np.array_equal(tree.locate(p), want)


# ---------------------------------------------------------------------------
# Host-cell search (Algorithm 1)
# ---------------------------------------------------------------------------
def _hand_tree(orc, periodic):
    anchors, levels = [], []
    for c in range(8):                       # children of level-1 cell (0,0,0), L = 2
        anchors.append((c & 1, (c >> 1) & 1, (c >> 2) & 1))
        levels.append(2)
    for c in range(1, 8):                    # the other level-1 cells
        anchors.append((2 * (c & 1), 2 * ((c >> 1) & 1), 2 * ((c >> 2) & 1)))
        levels.append(1)
    p = np.random.default_rng(5).permutation(15)
    return orc.Tree.from_anchors(np.array(anchors)[p], np.array(levels)[p], 1, 2, periodic)


def test_hand_tree_golden_ids(orc):
    g = _golden("hand_tree_locate.txt")
    for periodic, col in ((True, 3), (False, 4)):
        tree = _hand_tree(orc, periodic)
        assert tree.check_partition() == 0
        for method in ("alg1", "linear"):
            ids = tree.locate(g[:, :3], method)
            assert np.array_equal(ids, g[:, col].astype(np.int64)), (periodic, method)


def _adversarial_points(rng, spec, n):
    """Random points plus points on dyadic faces/edges/corners, 0 and 1-ulp."""
    L = spec.l_max
    p = [rng.random((n, 3))]
    g = rng.integers(0, 1 << L, (n, 3)) * math.ldexp(1.0, -L)   # exact grid corners
    p.append(g)
    mix = rng.random((n, 3))
    mask = rng.random((n, 3)) < 0.5
    mix[mask] = g[mask]
    p.append(mix)
    edge = np.array([[0.0, 0.0, 0.0], [np.nextafter(1.0, 0.0)] * 3, [0.5, 0.5, 0.5],
                     [np.nextafter(0.5, 0.0), 0.5, np.nextafter(0.5, 1.0)]])
    p.append(edge)
    return np.concatenate(p)


@pytest.mark.parametrize("seed", range(6))
def test_alg1_equals_linear_scan_random_trees(orc, seed):
    rng = np.random.default_rng(100 + seed)
    l_min = int(rng.integers(0, 3))
    l_max = l_min + int(rng.integers(1, 4))
    spec = synth.random_tree(l_min, l_max, rng, p_refine=0.35, periodic=bool(seed % 2),
                             balance=seed < 4)
    tree = _tree(orc, spec)
    assert tree.check_partition() == 0
    pts = _adversarial_points(rng, spec, 300)
    a = tree.locate(pts, "alg1")
    b = tree.locate(pts, "linear")
    assert np.array_equal(a, b)
    assert (a >= 0).all()
    # the returned leaf's half-open cube contains the point
    I = np.floor(pts * (1 << spec.l_max)).astype(np.int64) % (1 << spec.l_max)
    for k in range(0, pts.shape[0], 7):
        x, y, z = orc.morton_decode(int(tree.keys[a[k]]), spec.l_max)
        size = 1 << (spec.l_max - int(tree.levels[a[k]]))
        assert all(lo <= v < lo + size for lo, v in zip((x, y, z), I[k]))


def test_locate_outside_and_nan(orc):
    spec = synth.random_tree(1, 3, np.random.default_rng(3), periodic=False)
    tree = _tree(orc, spec)
    pts = np.array([[-1e-300, 0.5, 0.5], [1.0, 0.5, 0.5], [0.5, np.nan, 0.5],
                    [np.inf, 0.1, 0.1], [0.5, 0.5, 0.5]])
    ids = tree.locate(pts)
    assert list(ids[:4]) == [-1, -1, -1, -1] and ids[4] >= 0
    # periodic: shifting by whole periods (exact in binary) keeps the host
    spec_p = synth.random_tree(1, 3, np.random.default_rng(3), periodic=True)
    tp = _tree(orc, spec_p)
    p = np.random.default_rng(4).integers(0, 1 << 10, (200, 3)) / 1024.0
    for shift in (1.0, -1.0, 3.0, -7.0):
        assert np.array_equal(tp.locate(p + shift), tp.locate(p))
    assert tp.locate(np.array([[np.nan, 0.1, 0.1]]))[0] == -1


def test_get_cell_at_shift_identity():
    """floor(x 2^l) == floor(x 2^L) >> (L - l) for binary floating point x
    (why the oracle may form Algorithm 1's test cells from finest-level
    integer coordinates)."""
    rng = np.random.default_rng(9)
    xs = np.concatenate([rng.random(20000), rng.integers(0, 1 << 21, 2000) / float(1 << 21),
                         np.nextafter(rng.integers(1, 1 << 10, 2000) / 1024.0, 0.0)])
    for L in (6, 10, 21):
        IL = np.floor(xs * 2.0 ** L).astype(np.int64)
        for l in range(0, L + 1, 3):
            assert np.array_equal(np.floor(xs * 2.0 ** l).astype(np.int64), IL >> (L - l))


def test_partition_check_rejects_bad_trees(orc):
    spec = synth.random_tree(1, 3, np.random.default_rng(7))
    keys = orc.encode_keys(spec.anchors, 3)
    good = orc.Tree(keys, spec.levels, 1, 3)
    assert good.check_partition() == 0
    # drop a leaf -> gap
    assert orc.Tree(keys[1:], spec.levels[1:], 1, 3).check_partition() == 1
    # duplicate a leaf
    assert orc.Tree(np.append(keys, keys[0]), np.append(spec.levels, spec.levels[0]), 1, 3).check_partition() == 2
    # coarsen one fine leaf in place -> overlap with its siblings
    lv = spec.levels.copy()
    j = int(np.argmax(lv))
    lv[j] -= 1
    assert orc.Tree(keys, lv, 1, 3).check_partition() in (1, 3)
    # level out of range
    lv2 = spec.levels.copy()
    lv2[0] = 7
    assert orc.Tree(keys, lv2, 1, 3).check_partition() == 3


# ---------------------------------------------------------------------------
# Interpolation / spreading
# ---------------------------------------------------------------------------
def test_uniform_stencil_golden(orc):
    spec = synth.uniform_tree(2, seed=11)
    tree = _tree(orc, spec)
    a = spec.anchors.astype(np.float64)
    fld = np.stack([a[:, 0] ** 2, 10 * a[:, 1], 100 * a[:, 2]], axis=1)
    g = _golden("uniform_stencil.txt")
    U = tree.interpolate(tree.permute_rows(fld), g[:, :3])
    assert np.allclose(U, g[:, 3:], rtol=0, atol=1e-13)


def test_uniform_grid_textbook_interpolation(orc):
    """On a uniform periodic grid the method is textbook IBM interpolation:
    U(X) = sum over all cells c of phi((X-x_c)/h) phi(...) phi(...) u_c."""
    level = 3
    m = 1 << level
    spec = synth.uniform_tree(level, seed=12)
    tree = _tree(orc, spec)
    rng = np.random.default_rng(13)
    vals = rng.standard_normal((m, m, m, 3))
    a = spec.anchors
    fld = vals[a[:, 0], a[:, 1], a[:, 2]]
    pts = rng.random((300, 3))
    U = tree.interpolate(tree.permute_rows(fld), pts)
    want = np.zeros_like(pts)
    for k, X in enumerate(pts):
        base = np.floor(X * m - 0.5).astype(np.int64)
        for dz in range(-1, 3):
            for dy in range(-1, 3):
                for dx in range(-1, 3):
                    c = base + np.array([dx, dy, dz])
                    r = X * m - (c + 0.5)
                    w = np.prod(_phi_np(r))
                    want[k] += w * vals[c[0] % m, c[1] % m, c[2] % m]
    assert np.allclose(U, want, rtol=0, atol=1e-13)


@pytest.mark.parametrize("delta", [1e-9, 1e-14, 3e-16])
def test_wrapped_point_far_edge_weight(orc, delta):
    """A point just below 0 on a periodic uniform grid lies in the last cell
    at offset 1 - delta m, and the node two cells back (column m - 2) sits at
    distance 3/2 - delta m, near the edge of the support: its weight is
    phi(3/2 - eps), eps = delta m, to the oracle's phi precision (FP64
    relative plus about 2^-113 absolute).  An offset rounded to FP64 first
    (1 - eps is not representable) would miss eps by up to 2^-53 absolute, a
    relative error of order 2^-53/eps in eps and twice that in the weight."""
    level = 3
    m = 1 << level
    spec = synth.uniform_tree(level, seed=12)
    tree = _tree(orc, spec)
    a = spec.anchors
    fld = np.repeat((a[:, 0] == m - 2).astype(np.float64)[:, None], 3, axis=1)
    X = np.array([[-delta, 0.5 / m, 0.5 / m]])
    U = tree.interpolate(tree.permute_rows(fld), X)
    eps = delta * m   # exact: a power-of-two scaling
    want = _edge_phi_conjugate(eps)   # times the y and z weight sums, 1 up to rounding
    assert U[0] == pytest.approx(np.full(3, want), rel=1e-14, abs=2.0 ** -110), (delta, U[0], want)


def _cfg1(orc, periodic=True):
    w = synth.workload(1)
    spec = w.tree
    spec.periodic = periodic
    return w, _tree(orc, spec)


def test_constant_field_is_reproduced_everywhere(orc):
    """Partition of unity holds for any host level and across level jumps."""
    w, tree = _cfg1(orc)
    fld = np.tile([1.5, -2.0, 0.25], (tree.n_leaves, 1))
    U = tree.interpolate(fld, w.points)
    assert np.abs(U - np.array([1.5, -2.0, 0.25])).max() < 1e-14


def test_linear_field_exact_away_from_level_jumps(orc):
    w, tree = _cfg1(orc, periodic=False)
    c = synth.leaf_centres(w.tree)
    A = np.array([[0.3, -1.2, 2.0], [0.7, 0.1, -0.4], [-1.1, 0.5, 0.9]])
    fld = tree.permute_rows(c @ A.T + np.array([0.1, 0.2, 0.3]))
    rng = np.random.default_rng(21)
    pts = 0.1 + 0.8 * rng.random((4000, 3))
    host, level, nodes = tree.stencil_leaves(pts)
    same = np.all(tree.levels[nodes] == level[:, None], axis=1) & np.all(nodes >= 0, axis=1)
    assert same.sum() > 3000
    U = tree.interpolate(fld, pts[same])
    want = pts[same] @ A.T + np.array([0.1, 0.2, 0.3])
    assert np.abs(U - want).max() < 1e-13
    # and it is not exact at the jumps (the check above is not vacuous)
    Uj = tree.interpolate(fld, pts[~same])
    assert np.abs(Uj - (pts[~same] @ A.T + [0.1, 0.2, 0.3])).max() > 1e-6


def test_spread_conserves_total_force(orc):
    w, tree = _cfg1(orc)
    f = tree.spread(w.forces, w.points)
    assert np.allclose(f.sum(axis=0), w.forces.sum(axis=0), rtol=0, atol=1e-10)


def test_spread_is_adjoint_of_interpolate(orc):
    """<spread(F), u> = <F, interpolate(u)> with plain dot products."""
    w, tree = _cfg1(orc)
    rng = np.random.default_rng(31)
    u = rng.standard_normal((tree.n_leaves, 3))
    lhs = float((tree.spread(w.forces, w.points) * u).sum())
    rhs = float((w.forces * tree.interpolate(u, w.points)).sum())
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_node_leaves_within_one_level_on_balanced_tree(orc):
    w, tree = _cfg1(orc)
    host, level, nodes = tree.stencil_leaves(w.points)
    assert (host >= 0).all() and (nodes >= 0).all()
    d = tree.levels[nodes].astype(int) - level[:, None]
    assert d.min() >= -1 and d.max() <= 1
    assert np.array_equal(nodes[:, 13], host)   # centre node lies in the host leaf


def test_grad_matches_central_differences(orc):
    """d/dX (v . U(X)) by central differences (h = 1e-4 finest dx, FP64)
    against the analytic phi' gradient, host held fixed."""
    w, tree = _cfg1(orc)
    rng = np.random.default_rng(41)
    fld = tree.permute_rows(w.field)
    pts = w.points[::7]
    v = rng.standard_normal(pts.shape)
    g, S = tree.grad_pos(fld, v, pts, with_scale=True)
    h = 1e-4 * math.ldexp(1.0, -tree.l_max)
    host, level, _ = tree.stencil_leaves(pts)
    checked = 0
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        hp, _, _ = tree.stencil_leaves(pts + e)
        hm, _, _ = tree.stencil_leaves(pts - e)
        s = pts[:, d] * np.ldexp(1.0, level)
        t = s - np.floor(s)
        kink = np.minimum.reduce([np.abs(t - 0.5 + o - k) for o in (-1, 0, 1) for k in (-0.5, 0.5)])
        ok = (hp == host) & (hm == host) & (kink * np.ldexp(1.0, tree.l_max - level) > 1e-3)
        Up = tree.interpolate(fld, pts[ok] + e)
        Um = tree.interpolate(fld, pts[ok] - e)
        fd = ((Up - Um) * v[ok]).sum(axis=1) / (2 * h)
        err = np.abs(fd - g[ok, d]) / np.maximum(S[ok, d], 1e-300)
        assert err.max() < 1e-6, d
        checked += int(ok.sum())
    assert checked > 3000


def test_node_leaf_contains_node_centre(orc):
    """The reading taken where a stencil node is refined or coarsened: the
    node value comes from the leaf whose half-open cube contains the node's
    centre.  Node centres are formed here from plain geometry."""
    w, tree = _cfg1(orc)
    L = tree.l_max
    host, level, nodes = tree.stencil_leaves(w.points)
    lv = level.astype(np.int64)
    m = np.left_shift(1, lv)
    i0 = np.floor(w.points * m[:, None]).astype(np.int64) % m[:, None]
    anchors = np.array([orc.morton_decode(int(k), L) for k in tree.keys], dtype=np.int64)
    size = np.left_shift(1, L - tree.levels.astype(np.int64))
    jumps = 0
    for q in range(27):
        o = np.array([q % 3 - 1, (q // 3) % 3 - 1, q // 9 - 1])
        n = (i0 + o) % m[:, None]
        centre = np.floor((n + 0.5) * np.ldexp(1.0, L - lv)[:, None]).astype(np.int64)
        leaf = nodes[:, q]
        a = anchors[leaf]
        assert np.all((a <= centre) & (centre < a + size[leaf][:, None])), q
        jumps += int((tree.levels[leaf] != level).sum())
    assert jumps > 1000     # level jumps are exercised


# ---------------------------------------------------------------------------
# Properties over drawn trees (hypothesis): Algorithm 1 equals the linear
# scan, constants are reproduced, spreading conserves the total force and is
# the adjoint of interpolation, on any partition the generator can make.
# ---------------------------------------------------------------------------
from hypothesis import HealthCheck, given, settings, strategies as st


@settings(max_examples=30, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(seed=st.integers(0, 2 ** 32 - 1), l_min=st.integers(0, 2), depth=st.integers(1, 3),
       p_refine=st.floats(0.05, 0.5), periodic=st.booleans(), balance=st.booleans())
def test_property_drawn_trees(orc, seed, l_min, depth, p_refine, periodic, balance):
    rng = np.random.default_rng(seed)
    spec = synth.random_tree(l_min, l_min + depth, rng, p_refine=p_refine, periodic=periodic, balance=balance)
    tree = _tree(orc, spec)
    assert tree.check_partition() == 0
    pts = _adversarial_points(rng, spec, 60)
    a = tree.locate(pts, "alg1")
    assert np.array_equal(a, tree.locate(pts, "linear"))
    if not periodic:
        return   # walls drop nodes: the sums below hold for periodic cubes
    c = np.array([0.75, -1.5, 2.0])
    U = tree.interpolate(np.tile(c, (tree.n_leaves, 1)), pts)
    np.testing.assert_allclose(U, np.tile(c, (pts.shape[0], 1)), rtol=1e-13, atol=0)
    F = rng.standard_normal(pts.shape)
    f = tree.spread(F, pts)
    np.testing.assert_allclose(f.sum(axis=0), F.sum(axis=0), rtol=1e-12, atol=1e-12 * np.abs(F).sum())
    u = rng.standard_normal((tree.n_leaves, 3))
    lhs, rhs = float((f * u).sum()), float((F * tree.interpolate(u, pts)).sum())
    assert abs(lhs - rhs) <= 1e-12 * (np.abs(f).sum() * np.abs(u).max() + 1.0)
