"""MI355X (gfx950) Lagrangian-point tracking on adaptive octrees.

Thin ctypes binding of ``libocttrack.so`` (declared in ``include/octrack.h``):
host-cell search (Algorithm 1 semantics), 3-point regularized-delta
interpolation and force spreading (Sec. 2.2), their position gradient, and a
batched persistent pass.  Torch tensors provide device memory and streams;
every step of the computation runs in the library's HIP kernels.  There is
no CPU fallback: importing this package fails if the library is not built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# OCTRACK_LIB: load another build of the library (e.g. a profiling build)
LIB_PATH = os.environ.get("OCTRACK_LIB") or os.path.join(_HERE, "libocttrack.so")

OT_OK = 0
OT_F32, OT_F64 = 0, 1
OT_SPREAD_ATOMIC, OT_SPREAD_FIXED = 0, 1
OT_OP_LOCATE, OT_OP_INTERPOLATE, OT_OP_SPREAD, OT_OP_GRAD_POS = 1, 2, 4, 8

ERRORS = {-1: "OT_ERR_INVALID", -2: "OT_ERR_NOT_PARTITION", -3: "OT_ERR_UNSORTED_DUP",
          -4: "OT_ERR_LEVEL_RANGE", -5: "OT_ERR_OOM", -6: "OT_ERR_HIP", -7: "OT_ERR_CAPACITY"}


class OtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class TreeDesc(ctypes.Structure):
    _fields_ = [("l_min", ctypes.c_int32), ("l_max", ctypes.c_int32), ("periodic", ctypes.c_int32)]


class TreeInfo(ctypes.Structure):
    _fields_ = [("n_leaves", ctypes.c_int64), ("l_min", ctypes.c_int32), ("l_max", ctypes.c_int32),
                ("periodic", ctypes.c_int32), ("table_levels", ctypes.c_int32),
                ("table_bytes", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64)]


class ParticleParams(ctypes.Structure):
    _fields_ = [("dt0", ctypes.c_double), ("r_p", ctypes.c_double), ("rho_p", ctypes.c_double),
                ("rho_f", ctypes.c_double), ("nu", ctypes.c_double), ("g", ctypes.c_double * 3),
                ("first", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("tile", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


OT_TUNE_SORT_POINTS = 1
OT_TUNE_HOST_MAJOR = 2
OT_TUNE_GRAPH = 4


EXPORTS = ("ot_encode_keys", "ot_build_tree", "ot_destroy_tree", "ot_tree_info_get", "ot_tree_leaves",
           "ot_locate", "ot_interpolate", "ot_spread", "ot_track", "ot_grad_pos", "ot_batch_plan_create",
           "ot_batch_run", "ot_batch_plan_shape", "ot_batch_plan_timing", "ot_batch_last_kernel_ms",
           "ot_batch_plan_destroy", "ot_strerror", "ot_last_error", "ot_mdf", "ot_mdf_workspace_bytes", "ot_body_sums",
           "ot_relocate", "ot_leaf_splitters", "ot_find_owner", "ot_particle_step", "ot_interp_backward",
           "ot_spread_backward", "ot_batch_run_grad", "ot_interp_grad_pos", "ot_spread_grad_pos",
           "ot_spread_workspace_bytes", "ot_batch_plan_windows", "ot_spread_noalloc", "ot_force_mean",
           "ot_force_mean_workspace_bytes", "ot_particle_sort", "ot_particle_sort_workspace_bytes")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2605_20565_amd.build` "
                          "(or __graft_entry__.build()); there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sigs = {
        "ot_encode_keys": [P, i64, i32, P, P],
        "ot_build_tree": [P, P, i64, ctypes.POINTER(TreeDesc), P, P, ctypes.POINTER(P)],
        "ot_destroy_tree": [P],
        "ot_tree_info_get": [P, ctypes.POINTER(TreeInfo)],
        "ot_tree_leaves": [P, P, P, P],
        "ot_locate": [P, P, i32, i64, P, P],
        "ot_interpolate": [P, P, P, P, i32, i64, P, P],
        "ot_spread": [P, P, P, P, i32, i64, i32, i32, P, P, P],
        "ot_spread_noalloc": [P, P, P, P, i32, i64, i32, i32, P, P],
        "ot_track": [P, i32, P, P, P, i32, i64, i32, i32, P, P, P, P, P],
        "ot_grad_pos": [P, P, P, P, P, i32, i64, P, P],
        "ot_interp_grad_pos": [P, P, P, P, P, i32, i64, P, P],
        "ot_spread_grad_pos": [P, P, P, P, P, i32, i64, P, P],
        "ot_interp_backward": [P, P, P, P, P, i32, i64, i32, i32, P, P, P, P],
        "ot_spread_backward": [P, P, P, P, P, i32, i64, P, P, P],
        "ot_batch_plan_create": [P, P, P, i32, i32, i32, ctypes.POINTER(Tuning), ctypes.POINTER(P)],
        "ot_batch_run": [P, P, P, P, P, P, P, P],
        "ot_batch_run_grad": [P, P, P, P, P, P, P, P, P],
        "ot_batch_plan_shape": [P, ctypes.POINTER(i64), ctypes.POINTER(i32)],
        "ot_batch_plan_windows": [P, ctypes.POINTER(i64), ctypes.POINTER(i64)],
        "ot_batch_plan_timing": [P, i32],
        "ot_batch_last_kernel_ms": [P, ctypes.POINTER(ctypes.c_float)],
        "ot_batch_plan_destroy": [P],
        "ot_mdf": [P, P, P, P, i32, i64, i32, ctypes.c_double, ctypes.c_double, i32, P, P, P, P],
        "ot_body_sums": [P, P, i64, P, i32, P, P, ctypes.c_double, i32, i32, P, P, P],
        "ot_force_mean": [P, P, i32, i32, P, P, P],
        "ot_relocate": [P, P, i32, i64, P, P, P],
        "ot_leaf_splitters": [P, i32, P, P],
        "ot_find_owner": [P, i32, i32, i32, P, i32, i64, P, P, P],
        "ot_particle_step": [P, P, P, P, P, P, P, i32, i64, ctypes.POINTER(ParticleParams), P],
        "ot_particle_sort": [P, i32, i64, P, P, P, P, P, P, P, P, P, P, P, P],
    }
    for name, args in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.ot_mdf_workspace_bytes.argtypes = [P, i64, i32]
    L.ot_mdf_workspace_bytes.restype = i64
    L.ot_spread_workspace_bytes.argtypes = [P]
    L.ot_spread_workspace_bytes.restype = i64
    L.ot_particle_sort_workspace_bytes.argtypes = [i64]
    L.ot_particle_sort_workspace_bytes.restype = i64
    L.ot_force_mean_workspace_bytes.argtypes = []
    L.ot_force_mean_workspace_bytes.restype = i64
    L.ot_strerror.argtypes = [i32]
    L.ot_strerror.restype = ctypes.c_char_p
    L.ot_last_error.argtypes = []
    L.ot_last_error.restype = ctypes.c_char_p
    return L


lib = _load()


def _check(rc: int) -> None:
    if rc != OT_OK:
        raise OtError(rc, lib.ot_last_error().decode())


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return OT_F32
    if t.dtype == torch.float64:
        return OT_F64
    raise TypeError(f"positions/fields must be float32 or float64, got {t.dtype}")


def _rows3(t: torch.Tensor, name: str) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dim() != 2 or t.shape[1] != 3:
        raise ValueError(f"{name} must have shape (n, 3)")
    return t.contiguous()


def _check_out(t: Optional[torch.Tensor], rows: int, dtype, device, name: str) -> None:
    if t is None:
        return
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous() or t.numel() < rows * (3 if t.dim() == 2 else 1):
        raise ValueError(f"{name}: needs a contiguous {dtype} device tensor with {rows} rows")


def _host_ids(ids: Optional[torch.Tensor], n: int, device) -> Optional[torch.Tensor]:
    """Validate caller-given host ids (int32, one per point) or pass None."""
    if ids is None:
        return None
    if ids.dtype != torch.int32 or ids.numel() != n or not ids.is_contiguous() or ids.device != device:
        raise ValueError("ids must be a contiguous int32 tensor with one host id per point, on the points' device")
    return ids


def _mode_code(mode) -> int:
    if mode in ("atomic", OT_SPREAD_ATOMIC):
        return OT_SPREAD_ATOMIC
    if mode in ("fixed", OT_SPREAD_FIXED):
        return OT_SPREAD_FIXED
    raise ValueError(f"unknown spread mode {mode!r}")


def encode_keys(anchors: torch.Tensor, l_max: int) -> torch.Tensor:
    """Morton keys (returned as int64 bit patterns) of (n, 3) uint32/int32 anchors."""
    a = anchors.contiguous()
    if a.dtype not in (torch.int32, torch.uint32):
        raise TypeError("anchors must be int32/uint32")
    keys = torch.empty(a.shape[0], dtype=torch.int64, device=a.device)
    _check(lib.ot_encode_keys(_ptr(a), a.shape[0], l_max, _ptr(keys), _stream()))
    return keys


class Tree:
    """A built octree on the current device (see ``ot_build_tree``).

    ``perm[id]`` is the input row of the leaf with Morton rank ``id``.
    """

    def __init__(self, keys: torch.Tensor, levels: torch.Tensor, l_min: int, l_max: int, periodic: bool = True):
        keys = keys.contiguous()
        levels = levels.contiguous()
        if keys.dtype not in (torch.int64, torch.uint64) or levels.dtype != torch.uint8:
            raise TypeError("keys must be int64/uint64 and levels uint8")
        n = keys.shape[0]
        self.perm = torch.empty(n, dtype=torch.int32, device=keys.device)
        desc = TreeDesc(l_min, l_max, 1 if periodic else 0)
        h = ctypes.c_void_p()
        _check(lib.ot_build_tree(_ptr(keys), _ptr(levels), n, ctypes.byref(desc), _ptr(self.perm), _stream(),
                                 ctypes.byref(h)))
        self._h = h
        self.l_min, self.l_max, self.periodic = int(l_min), int(l_max), bool(periodic)
        self.n_leaves = int(n)
        self.device = keys.device
        self.ws_bytes = int(lib.ot_spread_workspace_bytes(h))

    def workspace(self) -> torch.Tensor:
        """A fixed-point spreading workspace for this tree (``ot_spread``'s
        ``work``); the caching allocator hands out 512-byte aligned blocks."""
        return torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)

    def _work(self, mode, work: Optional[torch.Tensor]):
        if _mode_code(mode) != OT_SPREAD_FIXED:
            return None
        if work is None:
            return self.workspace()
        if work.device != self.device or work.numel() * work.element_size() < self.ws_bytes or \
                work.data_ptr() % 256:
            raise ValueError(f"work must be a 256-byte aligned device buffer of {self.ws_bytes} bytes")
        return work

    @classmethod
    def from_anchors(cls, anchors: torch.Tensor, levels: torch.Tensor, l_min: int, l_max: int,
                     periodic: bool = True) -> "Tree":
        return cls(encode_keys(anchors, l_max), levels, l_min, l_max, periodic)

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib.ot_destroy_tree(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def info(self) -> TreeInfo:
        inf = TreeInfo()
        _check(lib.ot_tree_info_get(self._h, ctypes.byref(inf)))
        return inf

    def leaves(self) -> Tuple[torch.Tensor, torch.Tensor]:
        k = torch.empty(self.n_leaves, dtype=torch.int64, device=self.device)
        lv = torch.empty(self.n_leaves, dtype=torch.uint8, device=self.device)
        _check(lib.ot_tree_leaves(self._h, _ptr(k), _ptr(lv), _stream()))
        return k, lv

    def permute_rows(self, rows: torch.Tensor) -> torch.Tensor:
        """Rows in the caller's leaf order -> leaf-id (Morton) order."""
        return rows.index_select(0, self.perm.long()).contiguous()

    # -- the tracking step -------------------------------------------------
    def locate(self, pos: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        pos = _rows3(pos, "pos")
        _check_out(out, pos.shape[0], torch.int32, pos.device, "out")
        ids = out if out is not None else torch.empty(pos.shape[0], dtype=torch.int32, device=pos.device)
        _check(lib.ot_locate(self._h, _ptr(pos), _dtype_code(pos), pos.shape[0], _ptr(ids), _stream()))
        return ids

    def interpolate(self, field: torch.Tensor, pos: torch.Tensor, out: Optional[torch.Tensor] = None,
                    ids: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Velocities at pos; ids: the points' host ids when already known (skips the search)."""
        pos = _rows3(pos, "pos")
        field = _rows3(field, "field")
        if field.dtype != pos.dtype or field.shape[0] != self.n_leaves:
            raise ValueError("field must be (n_leaves, 3) with the dtype of pos")
        _check_out(out, pos.shape[0], pos.dtype, pos.device, "out")
        ids = _host_ids(ids, pos.shape[0], pos.device)
        vel = out if out is not None else torch.empty_like(pos)
        _check(lib.ot_interpolate(self._h, _ptr(field), _ptr(pos), _ptr(ids), _dtype_code(pos), pos.shape[0],
                                  _ptr(vel), _stream()))
        return vel

    def spread(self, force: torch.Tensor, pos: torch.Tensor, mode="atomic", out: Optional[torch.Tensor] = None,
               accumulate: bool = False, ids: Optional[torch.Tensor] = None,
               work: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Leaf field of the spread forces; ids: known host ids; work: FIXED mode's workspace
        (``workspace()``; a fresh one per call when None)."""
        pos = _rows3(pos, "pos")
        force = _rows3(force, "force")
        if force.dtype != pos.dtype or force.shape[0] != pos.shape[0]:
            raise ValueError("force must be (n, 3) with the dtype of pos")
        if out is None:
            out = torch.empty((self.n_leaves, 3), dtype=pos.dtype, device=pos.device)
            accumulate = False
        _check_out(out, self.n_leaves, pos.dtype, pos.device, "out")
        ids = _host_ids(ids, pos.shape[0], pos.device)
        work = self._work(mode, work)
        _check(lib.ot_spread(self._h, _ptr(force), _ptr(pos), _ptr(ids), _dtype_code(pos), pos.shape[0],
                             _mode_code(mode), 1 if accumulate else 0, _ptr(out), _ptr(work), _stream()))
        return out

    def track(self, pos: torch.Tensor, field: Optional[torch.Tensor] = None, force: Optional[torch.Tensor] = None,
              ops: int = OT_OP_LOCATE | OT_OP_INTERPOLATE | OT_OP_SPREAD, mode="atomic",
              ids: Optional[torch.Tensor] = None, vel: Optional[torch.Tensor] = None,
              field_out: Optional[torch.Tensor] = None, accumulate: bool = False,
              work: Optional[torch.Tensor] = None):
        """Fused pass: returns (ids, vel, field_out) (None where the op is off)."""
        pos = _rows3(pos, "pos")
        n = pos.shape[0]
        if ops & OT_OP_LOCATE and ids is None:
            ids = torch.empty(n, dtype=torch.int32, device=pos.device)
        if ops & OT_OP_INTERPOLATE and vel is None:
            vel = torch.empty_like(pos)
        if ops & OT_OP_SPREAD and field_out is None:
            field_out = torch.empty((self.n_leaves, 3), dtype=pos.dtype, device=pos.device)
            accumulate = False
        if field is not None:
            field = _rows3(field, "field")
            if field.shape[0] != self.n_leaves or field.dtype != pos.dtype:
                raise ValueError("field must be (n_leaves, 3) with the dtype of pos")
        if force is not None:
            force = _rows3(force, "force")
            if force.shape[0] != n or force.dtype != pos.dtype:
                raise ValueError("force must be (n, 3) with the dtype of pos")
        _check_out(ids, n, torch.int32, pos.device, "ids")
        _check_out(vel, n, pos.dtype, pos.device, "vel")
        _check_out(field_out, self.n_leaves, pos.dtype, pos.device, "field_out")
        work = self._work(mode, work) if ops & OT_OP_SPREAD else None
        _check(lib.ot_track(self._h, ops, _ptr(field), _ptr(force), _ptr(pos), _dtype_code(pos), n,
                            _mode_code(mode), 1 if accumulate else 0, _ptr(ids), _ptr(vel), _ptr(field_out),
                            _ptr(work), _stream()))
        return ids, vel, field_out

    def grad_pos(self, field: torch.Tensor, vec: torch.Tensor, pos: torch.Tensor,
                 out: Optional[torch.Tensor] = None, ids: Optional[torch.Tensor] = None,
                 entry: str = "ot_grad_pos") -> torch.Tensor:
        """Position gradient sum_n (vec . field[leaf(n)]) grad w (``entry`` picks the C entry point:
        ot_grad_pos, ot_interp_grad_pos (field, vec = grad_vel) or ot_spread_grad_pos (field = grad_field,
        vec = force); all three compute the same sum)."""
        pos = _rows3(pos, "pos")
        field = _rows3(field, "field")
        vec = _rows3(vec, "vec")
        if field.shape[0] != self.n_leaves or vec.shape[0] != pos.shape[0]:
            raise ValueError("field must be (n_leaves, 3) and vec (n, 3)")
        if field.dtype != pos.dtype or vec.dtype != pos.dtype:
            raise ValueError("field, vec and pos must share a dtype")
        _check_out(out, pos.shape[0], pos.dtype, pos.device, "out")
        ids = _host_ids(ids, pos.shape[0], pos.device)
        if entry not in ("ot_grad_pos", "ot_interp_grad_pos", "ot_spread_grad_pos"):
            raise ValueError(f"unknown gradient entry point {entry!r}")
        g = out if out is not None else torch.empty_like(pos)
        _check(getattr(lib, entry)(self._h, _ptr(field), _ptr(vec), _ptr(pos), _ptr(ids), _dtype_code(pos),
                                   pos.shape[0], _ptr(g), _stream()))
        return g

    def interp_backward(self, field: torch.Tensor, grad_vel: torch.Tensor, pos: torch.Tensor, mode="atomic",
                        need_field: bool = True, need_pos: bool = True, accumulate: bool = False,
                        grad_field: Optional[torch.Tensor] = None, grad_pos: Optional[torch.Tensor] = None,
                        ids: Optional[torch.Tensor] = None, work: Optional[torch.Tensor] = None):
        """Backward of `interpolate` in one pass: (spread(grad_vel), grad_pos(field, grad_vel)); an output
        not asked for is None."""
        pos = _rows3(pos, "pos")
        field = _rows3(field, "field")
        grad_vel = _rows3(grad_vel, "grad_vel")
        if field.shape[0] != self.n_leaves or grad_vel.shape[0] != pos.shape[0]:
            raise ValueError("field must be (n_leaves, 3) and grad_vel (n, 3)")
        if field.dtype != pos.dtype or grad_vel.dtype != pos.dtype:
            raise ValueError("field, grad_vel and pos must share a dtype")
        if not (need_field or need_pos):
            raise ValueError("nothing to compute")
        gf = gx = None
        if need_field:
            _check_out(grad_field, self.n_leaves, pos.dtype, pos.device, "grad_field")
            gf = grad_field if grad_field is not None else torch.empty((self.n_leaves, 3), dtype=pos.dtype,
                                                                       device=pos.device)
        if need_pos:
            _check_out(grad_pos, pos.shape[0], pos.dtype, pos.device, "grad_pos")
            gx = grad_pos if grad_pos is not None else torch.empty_like(pos)
        ids = _host_ids(ids, pos.shape[0], pos.device)
        work = self._work(mode, work) if need_field else None
        _check(lib.ot_interp_backward(self._h, _ptr(field), _ptr(grad_vel), _ptr(pos), _ptr(ids), _dtype_code(pos),
                                      pos.shape[0], _mode_code(mode), 1 if accumulate else 0, _ptr(gf), _ptr(gx),
                                      _ptr(work), _stream()))
        return gf, gx

    def spread_backward(self, grad_field: torch.Tensor, force: torch.Tensor, pos: torch.Tensor,
                        need_force: bool = True, need_pos: bool = True, ids: Optional[torch.Tensor] = None):
        """Backward of `spread` in one pass: (interpolate(grad_field), grad_pos(grad_field, force)); an output
        not asked for is None."""
        pos = _rows3(pos, "pos")
        grad_field = _rows3(grad_field, "grad_field")
        force = _rows3(force, "force")
        if grad_field.shape[0] != self.n_leaves or force.shape[0] != pos.shape[0]:
            raise ValueError("grad_field must be (n_leaves, 3) and force (n, 3)")
        if grad_field.dtype != pos.dtype or force.dtype != pos.dtype:
            raise ValueError("grad_field, force and pos must share a dtype")
        if not (need_force or need_pos):
            raise ValueError("nothing to compute")
        gF = torch.empty_like(pos) if need_force else None
        gx = torch.empty_like(pos) if need_pos else None
        ids = _host_ids(ids, pos.shape[0], pos.device)
        _check(lib.ot_spread_backward(self._h, _ptr(grad_field), _ptr(force), _ptr(pos), _ptr(ids), _dtype_code(pos),
                                      pos.shape[0], _ptr(gF), _ptr(gx), _stream()))
        return gF, gx

    def force_mean(self, field: torch.Tensor, subtract: bool = True,
                   work: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Volume average over the unit cube of a leaf field (ot_force_mean), FP64 (3,); with
        subtract=True the field, in place, loses it (Sec. 5.2's mean IBM-force subtraction)."""
        if not field.is_contiguous():
            raise ValueError("field must be contiguous (it is updated in place)")
        field = _rows3(field, "field")
        if field.shape[0] != self.n_leaves:
            raise ValueError("field must be (n_leaves, 3)")
        mean = torch.empty(3, dtype=torch.float64, device=field.device)
        _check(lib.ot_force_mean(self._h, _ptr(field), _dtype_code(field), 1 if subtract else 0, _ptr(mean),
                                 _ptr(work), _stream()))
        return mean

    def relocate(self, pos: torch.Tensor, ids: torch.Tensor, count: bool = True) -> Optional[int]:
        """Update `ids` (previous hosts, int32) in place to the hosts of the
        moved points (ot_relocate); returns how many changed (count=False:
        nothing, and no synchronisation)."""
        pos = _rows3(pos, "pos")
        if ids.dtype != torch.int32 or ids.numel() != pos.shape[0] or not ids.is_contiguous():
            raise ValueError("ids must be a contiguous int32 tensor with one entry per point")
        moved = torch.empty(1, dtype=torch.int64, device=pos.device) if count else None
        _check(lib.ot_relocate(self._h, _ptr(pos), _dtype_code(pos), pos.shape[0], _ptr(ids), _ptr(moved),
                               _stream()))
        return int(moved.item()) if count else None

    def leaf_splitters(self, P: int) -> torch.Tensor:
        out = torch.empty(P + 1, dtype=torch.int64, device=self.device)
        _check(lib.ot_leaf_splitters(self._h, int(P), _ptr(out), _stream()))
        return out

    def find_owner(self, splitters: torch.Tensor, pos: torch.Tensor) -> Tuple[torch.Tensor, torch.Tensor]:
        """(owner int32 (n,), counts int64 (P,)) under the given partition."""
        pos = _rows3(pos, "pos")
        P = splitters.numel() - 1
        owner = torch.empty(pos.shape[0], dtype=torch.int32, device=pos.device)
        counts = torch.empty(P, dtype=torch.int64, device=pos.device)
        _check(lib.ot_find_owner(_ptr(splitters.contiguous()), P, self.l_max, int(self.periodic), _ptr(pos),
                                 _dtype_code(pos), pos.shape[0], _ptr(owner), _ptr(counts), _stream()))
        return owner, counts

    def particle_step(self, field: torch.Tensor, pos: torch.Tensor, vel: torch.Tensor, vel_prev: torch.Tensor,
                      acc_prev: torch.Tensor, ids: torch.Tensor, dt0: float, r_p: float, rho_p: float, rho_f: float,
                      nu: float, g=(0.0, 0.0, 0.0), first: bool = False) -> None:
        """One point-particle step (ot_particle_step), all state in place."""
        pos = _rows3(pos, "pos")
        for name, tns in (("vel", vel), ("vel_prev", vel_prev), ("acc_prev", acc_prev)):
            if tns.shape != pos.shape or tns.dtype != pos.dtype or not tns.is_contiguous():
                raise ValueError(f"{name} must be a contiguous (n, 3) tensor of the dtype of pos")
        field = _rows3(field, "field")
        if field.shape[0] != self.n_leaves or field.dtype != pos.dtype:
            raise ValueError("field must be (n_leaves, 3) with the dtype of pos")
        if ids.dtype != torch.int32 or ids.numel() != pos.shape[0] or not ids.is_contiguous():
            raise ValueError("ids must be a contiguous int32 tensor with one entry per point")
        prm = ParticleParams(float(dt0), float(r_p), float(rho_p), float(rho_f), float(nu),
                             (ctypes.c_double * 3)(*[float(x) for x in g]), int(bool(first)), 0)
        _check(lib.ot_particle_step(self._h, _ptr(field), _ptr(pos), _ptr(vel), _ptr(vel_prev), _ptr(acc_prev),
                                    _ptr(ids), _dtype_code(pos), pos.shape[0], ctypes.byref(prm), _stream()))

    def particle_sort(self, pos: torch.Tensor, vel: torch.Tensor, vel_prev: torch.Tensor, acc_prev: torch.Tensor,
                      out=None, work: Optional[torch.Tensor] = None):
        """Particle state reordered by host leaf (ot_particle_sort): returns
        (pos, vel, vel_prev, acc_prev, ids, perm), the four arrays reordered,
        each row's host id (-1: none) and its input row.  `out`: four arrays
        of the shape of pos to write into (not the inputs); `work`: a uint8
        device buffer of ot_particle_sort_workspace_bytes(n) bytes."""
        pos = _rows3(pos, "pos")
        for name, tns in (("vel", vel), ("vel_prev", vel_prev), ("acc_prev", acc_prev)):
            if tns.shape != pos.shape or tns.dtype != pos.dtype or not tns.is_contiguous():
                raise ValueError(f"{name} must be a contiguous (n, 3) tensor of the dtype of pos")
        n = pos.shape[0]
        if out is None:
            out = tuple(torch.empty_like(pos) for _ in range(4))
        if len(out) != 4 or any(o.shape != pos.shape or o.dtype != pos.dtype or not o.is_contiguous() for o in out):
            raise ValueError("out must be four contiguous tensors shaped like pos")
        ids = torch.empty(n, dtype=torch.int32, device=pos.device)
        perm = torch.empty(n, dtype=torch.int32, device=pos.device)
        _check(lib.ot_particle_sort(self._h, _dtype_code(pos), n, _ptr(pos), _ptr(vel), _ptr(vel_prev),
                                    _ptr(acc_prev), *[_ptr(o) for o in out], _ptr(ids), _ptr(perm),
                                    _ptr(work) if work is not None else None, _stream()))
        return (*out, ids, perm)

    def mdf(self, field: torch.Tensor, pos: torch.Tensor, target: torch.Tensor, n_iter: int, dt: float = 1.0,
            rho: float = 1.0, mode: str = "fixed", inplace: bool = False,
            work: Optional[torch.Tensor] = None) -> Tuple[torch.Tensor, torch.Tensor, torch.Tensor]:
        """Multi-direct forcing (ot_mdf): returns (field, force_lag, force_eul).
        With inplace=True `field` itself is updated and returned."""
        pos = _rows3(pos, "pos")
        target = _rows3(target, "target")
        field = _rows3(field, "field")
        if field.shape[0] != self.n_leaves or target.shape[0] != pos.shape[0]:
            raise ValueError("field must be (n_leaves, 3) and target (n, 3)")
        if field.dtype != pos.dtype or target.dtype != pos.dtype:
            raise ValueError("field, target and pos must share a dtype")
        mcode = _mode_code(mode)
        u = field if inplace else field.clone()
        n = pos.shape[0]
        f_lag = torch.empty_like(pos)
        f_eul = torch.empty_like(u)
        nbytes = int(lib.ot_mdf_workspace_bytes(self._h, n, _dtype_code(pos)))
        if work is None or work.numel() * work.element_size() < nbytes or work.device != pos.device:
            work = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=pos.device)
        _check(lib.ot_mdf(self._h, _ptr(u), _ptr(pos), _ptr(target), _dtype_code(pos), n, int(n_iter),
                          float(dt), float(rho), mcode, _ptr(f_lag), _ptr(f_eul), _ptr(work), _stream()))
        return u, f_lag, f_eul


def body_sums(vec: torch.Tensor, pos: torch.Tensor, offsets, centres: torch.Tensor, dV=1.0,
              periodic: bool = True) -> Tuple[torch.Tensor, torch.Tensor]:
    """Per-body sums (ot_body_sums): returns (S, M), FP64 (n_body, 3):
    S_b = sum v dV and M_b = sum (X - x_b) x v dV over each body's points."""
    pos = _rows3(pos, "pos")
    vec = _rows3(vec, "vec")
    centres = _rows3(centres, "centres")
    if vec.shape[0] != pos.shape[0] or vec.dtype != pos.dtype or centres.dtype != pos.dtype:
        raise ValueError("vec must match pos in shape and dtype; centres in dtype")
    offs = torch.as_tensor(offsets, dtype=torch.int64, device=pos.device).contiguous()
    nb = offs.numel() - 1
    if nb != centres.shape[0]:
        raise ValueError("need one centre per body (len(offsets) - 1)")
    dv_t = None
    dv_all = 0.0
    if isinstance(dV, torch.Tensor):
        dv_t = dV.to(pos.dtype).contiguous()
        if dv_t.numel() != pos.shape[0] or dv_t.device != pos.device:
            raise ValueError("dV must be a scalar or one value per point on the points' device")
    else:
        dv_all = float(dV)
    S = torch.empty((nb, 3), dtype=torch.float64, device=pos.device)
    M = torch.empty((nb, 3), dtype=torch.float64, device=pos.device)
    _check(lib.ot_body_sums(_ptr(vec), _ptr(pos), pos.shape[0], _ptr(offs), nb, _ptr(centres),
                            _ptr(dv_t) if dv_t is not None else None, dv_all, _dtype_code(pos), int(bool(periodic)),
                            _ptr(S), _ptr(M), _stream()))
    return S, M


class BatchPlan:
    """Many point sets in one persistent pass (``ot_batch_*``); with ``graph`` its launches replay as one
    captured HIP graph."""

    def __init__(self, tree: Tree, offsets: Sequence[int], ops: Sequence[int], dtype=torch.float32,
                 mode="atomic", block: int = 0, tile: int = 0, grid: int = 0, sort_points: bool = False,
                 host_major: bool = False, graph: bool = False):
        off = (ctypes.c_int64 * len(offsets))(*[int(v) for v in offsets])
        opa = (ctypes.c_int32 * len(ops))(*[int(v) for v in ops])
        tun = Tuning(block, tile, grid, (OT_TUNE_SORT_POINTS if sort_points else 0) |
                     (OT_TUNE_HOST_MAJOR if host_major else 0) | (OT_TUNE_GRAPH if graph else 0))
        h = ctypes.c_void_p()
        code = OT_F32 if dtype == torch.float32 else OT_F64
        _check(lib.ot_batch_plan_create(tree.handle, off, opa, len(ops), code, _mode_code(mode), ctypes.byref(tun),
                                        ctypes.byref(h)))
        self._h = h
        self.tree = tree
        self.n_points = int(offsets[-1])
        self.dtype = dtype
        self.grad_ops = any(int(v) & OT_OP_GRAD_POS for v in ops)

    def shape(self) -> Tuple[int, int]:
        nt, g = ctypes.c_int64(), ctypes.c_int32()
        _check(lib.ot_batch_plan_shape(self._h, ctypes.byref(nt), ctypes.byref(g)))
        return nt.value, g.value

    def windows(self) -> Tuple[int, int]:
        """(windows of the host-major pass, windows the last run handed to the per-point pass)."""
        nw, fb = ctypes.c_int64(), ctypes.c_int64()
        _check(lib.ot_batch_plan_windows(self._h, ctypes.byref(nw), ctypes.byref(fb)))
        return nw.value, fb.value

    def set_timing(self, enable: bool) -> None:
        _check(lib.ot_batch_plan_timing(self._h, 1 if enable else 0))

    def last_kernel_ms(self) -> float:
        v = ctypes.c_float()
        _check(lib.ot_batch_last_kernel_ms(self._h, ctypes.byref(v)))
        return float(v.value)

    def run(self, pos, field=None, force=None, ids=None, vel=None, field_out=None, grad=None):
        """One pass; `grad` receives the position gradient of plans with OT_OP_GRAD_POS ops (force is then
        the per-point vector the gradient contracts the field with)."""
        n, nl = self.n_points, self.tree.n_leaves
        _check_out(pos, n, self.dtype, None, "pos")
        _check_out(force, n, self.dtype, None, "force")
        _check_out(field, nl, self.dtype, None, "field")
        _check_out(field_out, nl, self.dtype, None, "field_out")
        _check_out(vel, n, self.dtype, None, "vel")
        _check_out(ids, n, torch.int32, None, "ids")
        _check_out(grad, n, self.dtype, None, "grad")
        if self.grad_ops:
            _check(lib.ot_batch_run_grad(self._h, _ptr(field), _ptr(force), _ptr(pos), _ptr(ids), _ptr(vel),
                                         _ptr(field_out), _ptr(grad), _stream()))
            return ids, vel, field_out, grad
        if grad is not None:
            raise ValueError("grad is only written by plans with OT_OP_GRAD_POS ops")
        _check(lib.ot_batch_run(self._h, _ptr(field), _ptr(force), _ptr(pos), _ptr(ids), _ptr(vel),
                                _ptr(field_out), _stream()))
        return ids, vel, field_out

    def close(self):
        if getattr(self, "_h", None):
            lib.ot_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


from .autograd import InterpolateFn, SpreadFn, interpolate, spread  # noqa: E402,F401
