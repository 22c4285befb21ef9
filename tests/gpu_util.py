"""Helpers shared by the GPU parity tests: the same synthetic inputs go to the
HIP library (through its C ABI binding) and to the FP64 oracle, and results
are compared element by element with the metrics the tests state."""
from __future__ import annotations

import math

import numpy as np
import torch

import oracle
import synth


def gpu_tree(spec: synth.TreeSpec):
    import paper_2605_20565_amd as ot
    a = torch.from_numpy(spec.anchors.astype(np.int32)).cuda()
    lv = torch.from_numpy(spec.levels).cuda()
    return ot.Tree.from_anchors(a, lv, spec.l_min, spec.l_max, spec.periodic)


def oracle_tree(spec: synth.TreeSpec) -> oracle.Tree:
    return oracle.Tree.from_anchors(spec.anchors, spec.levels, spec.l_min, spec.l_max, spec.periodic)


def as_dtype(x: np.ndarray, dtype) -> np.ndarray:
    """Round inputs to the working precision; the oracle then sees exactly
    what the GPU sees (promoted back to FP64)."""
    return np.ascontiguousarray(x.astype(np.float32 if dtype == torch.float32 else np.float64).astype(np.float64))


def to_dev(x: np.ndarray, dtype) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


def scaled_err(got: np.ndarray, want: np.ndarray, scale: np.ndarray) -> float:
    """max |got - want| / scale, the scale being the absolute stencil sum
    (sum |w| |u| or sum |w F|): rounding in any order of the same sum stays
    below (a few) ulp x scale."""
    d = np.abs(np.asarray(got, dtype=np.float64) - want)
    s = np.maximum(scale, 1e-300)
    return float((d / s).max()) if d.size else 0.0


def fixed_point_quantum(forces: np.ndarray) -> float:
    """2^-s of the fixed-point spreading: s = min(62 - E, 51 - Ef),
    2^E >= n max|F|, 2^Ef >= max|F|."""
    n = forces.shape[0]
    m = float(np.abs(forces[np.isfinite(forces)]).max()) if forces.size else 0.0
    if m == 0.0 or n == 0:
        return 1.0
    _, E = math.frexp(n * m)
    _, Ef = math.frexp(m)
    return math.ldexp(1.0, -min(62 - E, 51 - Ef))


TOL = {torch.float64: 1e-12, torch.float32: 1e-5}

# Absolute precision of the oracle's delta weights: the printed phi formula is
# evaluated in binary128, whose outer branch (cancelling towards |r| = 3/2)
# is good to about 2^-113 absolute.  A leaf fed only by edge-of-support
# weights can hold a value of that order, so the bound keeps this term.
ETA = 2.0 ** -110


def spread_bound(S, A, cnt, dtype, quantum=None):
    """Per-leaf error bound for spreading: tol * sum|w F| + ETA * sum|F|,
    plus half a fixed-point quantum per contribution in FIXED mode."""
    b = TOL[dtype] * S + ETA * A
    if quantum is not None:
        b = b + cnt[:, None] * 0.5 * quantum * 1.0001
    return b


def spread_excess(got, f, S, A, cnt, dtype, quantum=None) -> float:
    """max |got - f| / bound (<= 1 passes)."""
    b = spread_bound(S, A, cnt, dtype, quantum)
    d = np.abs(np.asarray(got, dtype=np.float64) - f)
    return float((d / np.maximum(b, 1e-300)).max()) if d.size else 0.0
