"""ot_spread_noalloc (fixed-point spreading with the library's static device
workspace, for callers that cannot allocate) against ot_spread with a
workspace of its own, called through the C ABI: bit for bit, on two calls in
a row, the second on a smaller input (smaller tree, fewer points), so that
what the first call left in the static array must not leak into it."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import as_dtype, gpu_tree, to_dev

pytestmark = pytest.mark.gpu


def _noalloc(ot, t, F, P, ids=None, accumulate=0, out=None):
    code = ot.OT_F32 if P.dtype == torch.float32 else ot.OT_F64
    if out is None:
        out = torch.empty((t.n_leaves, 3), dtype=P.dtype, device="cuda")
    ot._check(ot.lib.ot_spread_noalloc(t.handle, ot._ptr(F), ot._ptr(P), ot._ptr(ids), code, P.shape[0],
                                       ot.OT_SPREAD_FIXED, accumulate, ot._ptr(out), ot._stream()))
    return out


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_spread_equals_spread_on_two_calls(dtype):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2605_20565_amd as ot
    rng = np.random.default_rng(17)
    w = synth.workload(1)
    t1 = gpu_tree(w.tree)
    P1 = to_dev(as_dtype(w.points, dtype), dtype)
    F1 = to_dev(as_dtype(w.forces * 3.0, dtype), dtype)
    a1 = _noalloc(ot, t1, F1, P1)
    torch.cuda.synchronize()
    assert torch.equal(a1, t1.spread(F1, P1, mode="fixed"))
    # second call: a smaller tree and fewer, smaller forces
    spec2 = synth.uniform_tree(4, seed=3)
    t2 = gpu_tree(spec2)
    P2 = to_dev(as_dtype(rng.random((700, 3)), dtype), dtype)
    F2 = to_dev(as_dtype(rng.standard_normal((700, 3)) * 0.01, dtype), dtype)
    a2 = _noalloc(ot, t2, F2, P2)
    torch.cuda.synchronize()
    assert torch.equal(a2, t2.spread(F2, P2, mode="fixed"))
    # given host ids and accumulate = 1 behave as in ot_spread
    ids2 = t2.locate(P2)
    base = torch.randn((t2.n_leaves, 3), dtype=dtype, device="cuda")
    acc_a = _noalloc(ot, t2, F2, P2, ids=ids2, accumulate=1, out=base.clone())
    acc_b = t2.spread(F2, P2, mode="fixed", out=base.clone(), accumulate=True, ids=ids2)
    torch.cuda.synchronize()
    assert torch.equal(acc_a, acc_b)
    # the first tree again, after the smaller call
    assert torch.equal(_noalloc(ot, t1, F1, P1), a1)


def test_noalloc_rejects_trees_beyond_its_workspace():
    import paper_2605_20565_amd as ot
    spec = synth.uniform_tree(7, seed=1)   # 2^21 leaves
    assert spec.n_leaves > (1 << 20)
    t = gpu_tree(spec)
    P = torch.rand((10, 3), device="cuda")
    F = torch.randn((10, 3), device="cuda")
    with pytest.raises(ot.OtError) as e:
        _noalloc(ot, t, F, P)
    assert e.value.code == -7 and b"OT_NOALLOC_MAX_LEAVES" in ot.lib.ot_last_error()
    # ATOMIC spreading needs no workspace and is not limited
    out = torch.empty((t.n_leaves, 3), device="cuda")
    ot._check(ot.lib.ot_spread_noalloc(t.handle, ot._ptr(F), ot._ptr(P), None, ot.OT_F32, 10, ot.OT_SPREAD_ATOMIC,
                                       0, ot._ptr(out), ot._stream()))
    torch.cuda.synchronize()
    assert torch.allclose(out.double().sum(0), F.double().sum(0), atol=1e-5)
