"""FP64 CPU oracle of the Lagrangian-point tracking step (test infrastructure).

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It wraps ``octree_oracle.c`` (plain C,
FP64) with numpy; the product library never loads it.

Every function follows the paper cited in ``octree_oracle.c``:
Algorithm 1 (host-cell search), the linear scan it replaces (Sec. 3.2), the
IBM interpolation / spreading sums and the 3-point delta function (Sec. 2.2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "octree_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle into ``liboracle.so`` with gcc (OpenMP, -O2, libquadmath)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lquadmath", "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Tree(ctypes.Structure):
    _fields_ = [("n_leaves", ctypes.c_int64),
                ("keys", ctypes.c_void_p),
                ("levels", ctypes.c_void_p),
                ("l_min", ctypes.c_int32),
                ("l_max", ctypes.c_int32),
                ("periodic", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, u32 = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32
        TP = ctypes.POINTER(_Tree)
        sig = {
            "orc_morton_encode": (ctypes.c_uint64, [u32, u32, u32, i32]),
            "orc_morton_decode": (None, [ctypes.c_uint64, i32, P, P, P]),
            "orc_encode_keys": (None, [i64, P, i32, P]),
            "orc_sort_leaves": (None, [i64, P, P]),
            "orc_check_partition": (i32, [TP]),
            "orc_locate": (None, [TP, P, i64, i32, P]),
            "orc_phi": (ctypes.c_double, [ctypes.c_double]),
            "orc_dphi": (ctypes.c_double, [ctypes.c_double]),
            "orc_interpolate": (None, [TP, P, P, i64, P, P]),
            "orc_spread": (None, [TP, P, P, i64, P, P, P, P]),
            "orc_grad_pos": (None, [TP, P, P, P, i64, P, P]),
            "orc_stencil_leaves": (None, [TP, P, i64, P, P, P]),
            "orc_num_threads": (i32, []),
            "orc_set_num_threads": (None, [i32]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# ---------------------------------------------------------------------------
# Morton keys and tree construction
# ---------------------------------------------------------------------------
def morton_encode(x: int, y: int, z: int, l_max: int) -> int:
    return int(lib().orc_morton_encode(x, y, z, l_max))


def morton_decode(k: int, l_max: int):
    a, b, c = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    lib().orc_morton_decode(k, l_max, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
    return a.value, b.value, c.value


def encode_keys(anchors: np.ndarray, l_max: int) -> np.ndarray:
    a = np.ascontiguousarray(anchors, dtype=np.uint32).reshape(-1, 3)
    keys = np.empty(a.shape[0], dtype=np.uint64)
    lib().orc_encode_keys(a.shape[0], _p(a), l_max, _p(keys))
    return keys


class Tree:
    """A Morton-sorted leaf array (one root tree over the unit cube).

    ``perm[sorted] = input index`` maps sorted rows back to the caller's rows.
    """

    def __init__(self, keys: np.ndarray, levels: np.ndarray, l_min: int, l_max: int,
                 periodic: bool = True, presorted: bool = False):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        levels = np.ascontiguousarray(levels, dtype=np.uint8)
        if presorted:
            self.perm = np.arange(keys.shape[0], dtype=np.int64)
        else:
            self.perm = np.empty(keys.shape[0], dtype=np.int64)
            lib().orc_sort_leaves(keys.shape[0], _p(keys), _p(self.perm))
        self.keys = np.ascontiguousarray(keys[self.perm])
        self.levels = np.ascontiguousarray(levels[self.perm])
        self.l_min, self.l_max, self.periodic = int(l_min), int(l_max), bool(periodic)
        self._c = _Tree(self.keys.shape[0], self.keys.ctypes.data, self.levels.ctypes.data,
                        self.l_min, self.l_max, int(self.periodic))

    @classmethod
    def from_anchors(cls, anchors, levels, l_min, l_max, periodic=True):
        return cls(encode_keys(anchors, l_max), levels, l_min, l_max, periodic)

    @property
    def n_leaves(self) -> int:
        return int(self.keys.shape[0])

    def check_partition(self) -> int:
        return int(lib().orc_check_partition(ctypes.byref(self._c)))

    def permute_rows(self, rows: np.ndarray) -> np.ndarray:
        """Rows given in the caller's leaf order -> Morton order."""
        return np.ascontiguousarray(np.asarray(rows)[self.perm])

    # -- the tracking step ---------------------------------------------------
    def locate(self, pos, method: str = "alg1") -> np.ndarray:
        pos = _f64(pos).reshape(-1, 3)
        ids = np.empty(pos.shape[0], dtype=np.int64)
        lib().orc_locate(ctypes.byref(self._c), _p(pos), pos.shape[0],
                         0 if method == "alg1" else 1, _p(ids))
        return ids

    def interpolate(self, field, pos, with_scale: bool = False):
        field = _f64(field).reshape(self.n_leaves, 3)
        pos = _f64(pos).reshape(-1, 3)
        U = np.empty_like(pos)
        S = np.empty_like(pos) if with_scale else None
        lib().orc_interpolate(ctypes.byref(self._c), _p(field), _p(pos), pos.shape[0], _p(U),
                              _p(S) if with_scale else None)
        return (U, S) if with_scale else U

    def spread(self, force, pos, with_scale: bool = False):
        """f, or (f, S, count, A) with S = sum |w F|, count = contributions and
        A = sum |F| over contributions, per leaf."""
        force = _f64(force).reshape(-1, 3)
        pos = _f64(pos).reshape(-1, 3)
        f = np.empty((self.n_leaves, 3), dtype=np.float64)
        S = np.empty_like(f) if with_scale else None
        A = np.empty_like(f) if with_scale else None
        cnt = np.empty(self.n_leaves, dtype=np.int64) if with_scale else None
        lib().orc_spread(ctypes.byref(self._c), _p(force), _p(pos), pos.shape[0], _p(f),
                         _p(S) if with_scale else None, _p(cnt) if with_scale else None,
                         _p(A) if with_scale else None)
        return (f, S, cnt, A) if with_scale else f

    def grad_pos(self, field, vec, pos, with_scale: bool = False):
        field = _f64(field).reshape(self.n_leaves, 3)
        vec = _f64(vec).reshape(-1, 3)
        pos = _f64(pos).reshape(-1, 3)
        g = np.empty_like(pos)
        S = np.empty_like(pos) if with_scale else None
        lib().orc_grad_pos(ctypes.byref(self._c), _p(field), _p(vec), _p(pos), pos.shape[0],
                           _p(g), _p(S) if with_scale else None)
        return (g, S) if with_scale else g

    def stencil_leaves(self, pos):
        pos = _f64(pos).reshape(-1, 3)
        n = pos.shape[0]
        host = np.empty(n, dtype=np.int64)
        level = np.empty(n, dtype=np.int32)
        nodes = np.empty((n, 27), dtype=np.int64)
        lib().orc_stencil_leaves(ctypes.byref(self._c), _p(pos), n, _p(host), _p(level), _p(nodes))
        return host, level, nodes


def phi(r: float) -> float:
    return float(lib().orc_phi(float(r)))


def dphi(r: float) -> float:
    return float(lib().orc_dphi(float(r)))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))
