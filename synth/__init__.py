"""Seeded synthetic workloads for the Lagrangian-point tracking step.

This module feeds the oracle and the GPU library the *same* inputs.  It holds
none of the tracking method's arithmetic: no Morton keys, no host search, no
delta weights.  It produces

* octrees as leaf anchors (integer corner coordinates in units of 2^-L) plus
  levels, refined around bubble surfaces the way the paper's auxiliary IBM
  forest is (Sec. 3.3: refined only near the markers) and 2:1 balanced across
  faces, edges and corners (Sec. 3.1, balancing);
* Lagrangian markers on bubble surfaces (Fibonacci lattice), uniformly
  distributed point particles, Gaussian shells of particles;
* leaf velocity fields (Taylor-Green, random Fourier modes with k^-5/3
  amplitudes) and N(0,1) point forces.

Leaves come out in a seeded random order, so every consumer has to sort them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

GOLDEN_ANGLE = math.pi * (3.0 - math.sqrt(5.0))


@dataclass
class Sphere:
    centre: Tuple[float, float, float]
    radius: float


@dataclass
class TreeSpec:
    anchors: np.ndarray        # (n, 3) uint32, corner of each leaf in units of 2^-l_max
    levels: np.ndarray         # (n,) uint8
    l_min: int
    l_max: int
    periodic: bool

    @property
    def n_leaves(self) -> int:
        return int(self.levels.shape[0])


# ---------------------------------------------------------------------------
# Trees
# ---------------------------------------------------------------------------
def _lin(ix, iy, iz, m):
    return ix.astype(np.int64) + m * (iy.astype(np.int64) + m * iz.astype(np.int64))


def _unlin(c, m):
    c = np.asarray(c, dtype=np.int64)
    return c % m, (c // m) % m, c // (m * m)


def _cells_meeting_shell(level: int, s: Sphere, band: float, periodic: bool) -> np.ndarray:
    """Linear indices of level-`level` cells whose closed cube meets the shell
    R - band <= |x - c| <= R + band."""
    m = 1 << level
    h = 1.0 / m
    c = np.asarray(s.centre, dtype=np.float64)
    lo = np.floor((c - s.radius - band) * m).astype(np.int64) - 1
    hi = np.floor((c + s.radius + band) * m).astype(np.int64) + 1
    if not periodic:
        lo = np.maximum(lo, 0)
        hi = np.minimum(hi, m - 1)
    ax = [np.arange(lo[d], hi[d] + 1, dtype=np.int64) for d in range(3)]
    if any(a.size == 0 for a in ax):
        return np.empty(0, dtype=np.int64)
    # Separable per-axis distances: nearest and farthest point of [i h, (i+1) h].
    near2, far2 = [], []
    for d in range(3):
        a0 = ax[d] * h - c[d]
        a1 = a0 + h
        near = np.where(a0 > 0, a0, np.where(a1 < 0, -a1, 0.0))
        far = np.maximum(np.abs(a0), np.abs(a1))
        near2.append(near * near)
        far2.append(far * far)
    dmin2 = near2[0][None, None, :] + near2[1][None, :, None] + near2[2][:, None, None]
    dmax2 = far2[0][None, None, :] + far2[1][None, :, None] + far2[2][:, None, None]
    rin, rout = max(s.radius - band, 0.0), s.radius + band
    hit = (dmin2 <= rout * rout) & (dmax2 >= rin * rin)
    iz, iy, ix = np.nonzero(hit)
    ix, iy, iz = ax[0][ix] % m, ax[1][iy] % m, ax[2][iz] % m
    return np.unique(_lin(ix, iy, iz, m))


def _balance_and_leaves(refined: dict, l_min: int, l_max: int, periodic: bool):
    """Close the refined-cell sets under corner 2:1 balance, then list leaves.

    A cell C refined at level l needs all 26 neighbours of C (and C itself) to
    exist as level-l cells, i.e. their parents must be refined at level l-1.
    Sweeping from fine to coarse reaches the fixed point in one pass."""
    offs = np.array([(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)],
                    dtype=np.int64)
    for l in range(l_max - 1, l_min, -1):
        cur = refined.get(l, np.empty(0, dtype=np.int64))
        if cur.size == 0:
            continue
        m = 1 << l
        ix, iy, iz = _unlin(cur, m)
        nx = ix[:, None] + offs[None, :, 0]
        ny = iy[:, None] + offs[None, :, 1]
        nz = iz[:, None] + offs[None, :, 2]
        if periodic:
            nx, ny, nz = nx % m, ny % m, nz % m
            ok = np.ones(nx.shape, dtype=bool)
        else:
            ok = (nx >= 0) & (nx < m) & (ny >= 0) & (ny < m) & (nz >= 0) & (nz < m)
        par = _lin(nx[ok] >> 1, ny[ok] >> 1, nz[ok] >> 1, m >> 1)
        prev = refined.get(l - 1, np.empty(0, dtype=np.int64))
        refined[l - 1] = np.union1d(prev, np.unique(par))

    return _leaves_only(refined, l_min, l_max)


def band_tree(l_min: int, l_max: int, spheres: Sequence[Sphere], band_cells: float = 2.0,
              periodic: bool = True, seed: Optional[int] = 0) -> TreeSpec:
    """Octree uniform at l_min, refined to l_max in a band of `band_cells`
    finest cells around each sphere surface, then 2:1 corner balanced."""
    band = band_cells / (1 << l_max)
    refined = {}
    for l in range(l_min, l_max):
        parts = [_cells_meeting_shell(l, s, band, periodic) for s in spheres]
        parts = [p for p in parts if p.size]
        refined[l] = np.unique(np.concatenate(parts)) if parts else np.empty(0, dtype=np.int64)
    anchors, levels = _balance_and_leaves(refined, l_min, l_max, periodic)
    if seed is not None:
        p = np.random.default_rng(seed).permutation(levels.shape[0])
        anchors, levels = anchors[p], levels[p]
    return TreeSpec(np.ascontiguousarray(anchors), np.ascontiguousarray(levels), l_min, l_max, periodic)


def random_tree(l_min: int, l_max: int, rng: np.random.Generator, p_refine: float = 0.3,
                periodic: bool = True, balance: bool = True) -> TreeSpec:
    """Small random octree: each cell below l_max is refined with probability
    p_refine (then optionally 2:1 balanced).  Leaves in random order."""
    refined = {}
    for l in range(l_min, l_max):
        m = 1 << l
        if l == l_min:
            cand = np.arange(m ** 3, dtype=np.int64)
        else:
            par = refined.get(l - 1, np.empty(0, dtype=np.int64))
            px, py, pz = _unlin(par, m >> 1)
            ch = np.arange(8, dtype=np.int64)
            cand = _lin((2 * px[:, None] + (ch & 1)).ravel(), (2 * py[:, None] + ((ch >> 1) & 1)).ravel(),
                        (2 * pz[:, None] + ((ch >> 2) & 1)).ravel(), m)
        refined[l] = np.unique(cand[rng.random(cand.size) < p_refine])
    if balance:
        anchors, levels = _balance_and_leaves(refined, l_min, l_max, periodic)
    else:
        anchors, levels = _leaves_only(refined, l_min, l_max)
    p = rng.permutation(levels.shape[0])
    return TreeSpec(np.ascontiguousarray(anchors[p]), np.ascontiguousarray(levels[p]), l_min, l_max, periodic)


def _leaves_only(refined: dict, l_min: int, l_max: int):
    anchors, levels = [], []
    for l in range(l_min, l_max + 1):
        m = 1 << l
        if l == l_min:
            cells = np.arange(m ** 3, dtype=np.int64)
        else:
            par = refined.get(l - 1, np.empty(0, dtype=np.int64))
            if par.size == 0:
                continue
            px, py, pz = _unlin(par, m >> 1)
            ch = np.arange(8, dtype=np.int64)
            cells = _lin((2 * px[:, None] + (ch & 1)).ravel(), (2 * py[:, None] + ((ch >> 1) & 1)).ravel(),
                         (2 * pz[:, None] + ((ch >> 2) & 1)).ravel(), m)
        if l < l_max:
            r = refined.get(l, np.empty(0, dtype=np.int64))
            if r.size:
                if l == l_min:
                    keep = np.ones(m ** 3, dtype=bool)
                    keep[r] = False
                    cells = np.nonzero(keep)[0]
                else:
                    cells = cells[~np.isin(cells, r, assume_unique=True)]
        if cells.size == 0:
            continue
        x, y, z = _unlin(cells, m)
        sh = l_max - l
        anchors.append(np.stack([x << sh, y << sh, z << sh], axis=1).astype(np.uint32))
        levels.append(np.full(cells.size, l, dtype=np.uint8))
    return np.concatenate(anchors), np.concatenate(levels)


def uniform_tree(level: int, seed: Optional[int] = 0, periodic: bool = True) -> TreeSpec:
    return band_tree(level, level, [], periodic=periodic, seed=seed)


def leaf_centres(tree: TreeSpec) -> np.ndarray:
    """Cell-centre coordinates of the leaves, (n, 3) float64."""
    half = np.ldexp(0.5, tree.l_max - tree.levels.astype(np.int64))
    return (tree.anchors.astype(np.float64) + half[:, None]) * math.ldexp(1.0, -tree.l_max)


def leaf_sizes(tree: TreeSpec) -> np.ndarray:
    return np.ldexp(1.0, -tree.levels.astype(np.int64))


# ---------------------------------------------------------------------------
# Lagrangian points
# ---------------------------------------------------------------------------
def fibonacci_sphere(s: Sphere, n: int, wrap: bool = True) -> np.ndarray:
    """n markers on a sphere surface on a Fibonacci (golden-angle) lattice."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    th = GOLDEN_ANGLE * i
    p = np.stack([r * np.cos(th), r * np.sin(th), z], axis=1) * s.radius + np.asarray(s.centre)
    return np.mod(p, 1.0) if wrap else p


def uniform_points(n: int, rng: np.random.Generator) -> np.ndarray:
    return rng.random((n, 3))


def gaussian_shell_points(n: int, spheres: Sequence[Sphere], sigma: float,
                          rng: np.random.Generator, chunk: int = 1 << 22) -> np.ndarray:
    """Points at c + (R + sigma g) u, g ~ N(0,1), u uniform on the unit
    sphere, bubble drawn uniformly; wrapped into the unit cube."""
    out = np.empty((n, 3), dtype=np.float64)
    cs = np.asarray([s.centre for s in spheres], dtype=np.float64)
    rs = np.asarray([s.radius for s in spheres], dtype=np.float64)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        m = b - a
        k = rng.integers(0, len(spheres), m)
        u = rng.standard_normal((m, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        rad = rs[k] + sigma * rng.standard_normal(m)
        out[a:b] = np.mod(cs[k] + rad[:, None] * u, 1.0)
    return out


def place_bubbles(diams: Sequence[float], rng: np.random.Generator, gap: float) -> List[Sphere]:
    """Non-overlapping bubble centres by rejection (periodic distance),
    centre distance >= (d_i + d_j)/2 + gap."""
    out: List[Sphere] = []
    for d in diams:
        for _ in range(100000):
            c = rng.random(3)
            ok = True
            for s in out:
                dv = np.abs(c - np.asarray(s.centre))
                dv = np.minimum(dv, 1.0 - dv)
                if np.sqrt((dv * dv).sum()) < (d / 2 + s.radius) + gap:
                    ok = False
                    break
            if ok:
                out.append(Sphere(tuple(float(v) for v in c), d / 2))
                break
        else:
            raise RuntimeError("could not place bubble")
    return out


# ---------------------------------------------------------------------------
# Fields and forces
# ---------------------------------------------------------------------------
def taylor_green(x: np.ndarray) -> np.ndarray:
    tp = 2.0 * math.pi
    u = np.sin(tp * x[:, 0]) * np.cos(tp * x[:, 1]) * np.cos(tp * x[:, 2])
    v = -np.cos(tp * x[:, 0]) * np.sin(tp * x[:, 1]) * np.cos(tp * x[:, 2])
    return np.stack([u, v, np.zeros_like(u)], axis=1)


@dataclass
class FourierModes:
    k: np.ndarray      # (m, 3) integer wave vectors
    a: np.ndarray      # (m, 3) amplitudes, a_m . k_m = 0
    theta: np.ndarray  # (m,) phases


def fourier_modes(rng: np.random.Generator, n_modes: int = 32, kmax: int = 16) -> FourierModes:
    ks, amps = [], []
    while len(ks) < n_modes:
        k = rng.integers(-kmax, kmax + 1, 3)
        nk = float(np.sqrt((k * k).sum()))
        if nk < 1.0 or nk > kmax:
            continue
        v = rng.standard_normal(3)
        kh = k / nk
        a = v - (v @ kh) * kh
        a *= nk ** (-5.0 / 3.0) / np.linalg.norm(a)
        ks.append(k)
        amps.append(a)
    return FourierModes(np.asarray(ks, dtype=np.float64), np.asarray(amps),
                        rng.random(n_modes) * 2.0 * math.pi)


def fourier_field(x: np.ndarray, modes: FourierModes, chunk: int = 1 << 20) -> np.ndarray:
    """sum_m a_m cos(2 pi k_m . x + theta_m): divergence free, periodic."""
    out = np.zeros((x.shape[0], 3), dtype=np.float64)
    for a in range(0, x.shape[0], chunk):
        b = min(x.shape[0], a + chunk)
        ph = 2.0 * math.pi * (x[a:b] @ modes.k.T) + modes.theta[None, :]
        out[a:b] = np.cos(ph) @ modes.a
    return out


def normal_forces(n: int, rng: np.random.Generator) -> np.ndarray:
    return rng.standard_normal((n, 3))


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    tree: TreeSpec
    field: np.ndarray                  # (n_leaves, 3) in the tree's leaf order (unsorted)
    points: np.ndarray                 # (n, 3) float64
    forces: np.ndarray                 # (n, 3) float64
    instances: np.ndarray              # (n_inst + 1,) offsets into points
    kinds: List[str] = field(default_factory=list)   # per instance: "markers" / "particles"
    spheres: List[Sphere] = field(default_factory=list)
    seed: int = 0

    @property
    def n_points(self) -> int:
        return int(self.points.shape[0])


def _finest_dx(l_max: int) -> float:
    return math.ldexp(1.0, -l_max)


def workload(cfg: int, scale: float = 1.0, seed_base: Optional[int] = None) -> Workload:
    """Workloads shaped like the paper's bubble/particle cases.

    cfg 1: l 5->6, one sphere (d = 0.25, centred), 1,000 markers, 10^4
           uniform particles, Taylor-Green leaf field.
    cfg 2: l 7->10, 8 bubbles d = 0.05 (markers at finest spacing), 10^7
           uniform particles, 32 random Fourier modes.
    cfg 3: l 7->10, 256 bubbles d log-uniform in [0.01, 0.1], 64 particle
           groups of 10^4..10^6 (log-uniform) uniform particles.
    cfg 4: l 8->11, 32 bubbles d = 0.03, 10^8 particles in Gaussian shells
           (sigma = 2 finest dx).
    cfg 5: config-2 tree and field, 10^6 markers over the 8 bubbles.
    `scale` multiplies the particle counts (marker counts stay whole)."""
    seed = (cfg * 1000) if seed_base is None else seed_base
    rng = np.random.default_rng(seed)
    if cfg == 1:
        l_min, l_max = 5, 6
        spheres = [Sphere((0.5, 0.5, 0.5), 0.125)]
        tree = band_tree(l_min, l_max, spheres, seed=seed + 1)
        fld = taylor_green(leaf_centres(tree))
        marks = [fibonacci_sphere(spheres[0], 1000)]
        parts = [uniform_points(max(1, int(round(1e4 * scale))), rng)]
    elif cfg in (2, 5):
        l_min, l_max = 7, 10
        spheres = place_bubbles([0.05] * 8, rng, gap=4.0 * math.ldexp(1.0, -7))
        tree = band_tree(l_min, l_max, spheres, seed=seed + 1)
        fld = fourier_field(leaf_centres(tree), fourier_modes(rng))
        if cfg == 2:
            nm = int(round(4.0 * math.pi * 0.025 ** 2 / _finest_dx(l_max) ** 2))
            marks = [fibonacci_sphere(s, nm) for s in spheres]
            parts = [uniform_points(max(1, int(round(1e7 * scale))), rng)]
        else:
            per = max(1, int(round(125000 * scale)))
            marks = [fibonacci_sphere(s, per) for s in spheres]
            parts = []
    elif cfg == 3:
        l_min, l_max = 7, 10
        diams = np.exp(rng.uniform(math.log(0.01), math.log(0.1), 256))
        diams = np.sort(diams)[::-1]
        spheres = place_bubbles(list(diams), rng, gap=4.0 * math.ldexp(1.0, -7))
        tree = band_tree(l_min, l_max, spheres, seed=seed + 1)
        fld = fourier_field(leaf_centres(tree), fourier_modes(rng))
        dx = _finest_dx(l_max)
        marks = [fibonacci_sphere(s, int(round(math.pi * (2 * s.radius) ** 2 / dx ** 2))) for s in spheres]
        sizes = np.exp(rng.uniform(math.log(1e4), math.log(1e6), 64))
        parts = [uniform_points(max(1, int(round(sz * scale))), rng) for sz in sizes]
    elif cfg == 4:
        l_min, l_max = 8, 11
        spheres = place_bubbles([0.03] * 32, rng, gap=4.0 * math.ldexp(1.0, -8))
        tree = band_tree(l_min, l_max, spheres, seed=seed + 1)
        fld = fourier_field(leaf_centres(tree), fourier_modes(rng))
        marks = []
        parts = [gaussian_shell_points(max(1, int(round(1e8 * scale))), spheres,
                                       2.0 * _finest_dx(l_max), rng)]
    else:
        raise ValueError(f"unknown workload {cfg}")
    groups = marks + parts
    kinds = ["markers"] * len(marks) + ["particles"] * len(parts)
    offsets = np.zeros(len(groups) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([g.shape[0] for g in groups])
    pts = np.concatenate(groups) if groups else np.empty((0, 3))
    forces = normal_forces(pts.shape[0], rng)
    return Workload(f"cfg{cfg}", tree, fld, np.ascontiguousarray(pts), forces, offsets, kinds,
                    spheres, seed)
