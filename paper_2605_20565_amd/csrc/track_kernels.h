// Plain-launch kernels of the tracking step (one workgroup per tile of
// consecutive points), templated on precision and spreading mode.  The
// host code in track.hip calls dispatch_ops<T, MODE>, which track_inst.hip
// instantiates once per (T, MODE) in its own object file.
#pragma once

#include <hip/hip_runtime.h>

#include "ot_common.h"
#include "track_device.h"

namespace ot {

// One workgroup per tile of `tile` consecutive points.  Spreading goes
// through the workgroup's LDS aggregation table of S slots, flushed once at
// the end.
template <typename T, int OPS, int MODE, bool PER, int S>
__global__ __launch_bounds__(512) void k_track(TreeView tv, int64_t n, int64_t tile, const T *__restrict__ pos,
                                               const T *__restrict__ field, const T *__restrict__ force,
                                               int32_t *__restrict__ ids, T *__restrict__ vel,
                                               T *__restrict__ fout, unsigned long long *__restrict__ facc,
                                               const FxState *__restrict__ fx, T *__restrict__ grad,
                                               const int32_t *__restrict__ hid)
{
    const int64_t start = (int64_t)blockIdx.x * tile;
    const int64_t end = start + tile < n ? start + tile : n;
    if constexpr ((OPS & kOpSpread) != 0) {
        using Acc = typename AccType<T, MODE>::type;
        __shared__ uint32_t keys[S];
        __shared__ Acc vals[LdsSink<T, MODE, S>::kVals];
        const double scale = MODE == kModeFixed ? fx->scale : 0.0;
        LdsSink<T, MODE, S> sink{keys, vals, fout, facc, scale};
        sink.clear();
        __syncthreads();
        track_range<T, OPS, PER>(tv, start, end, nullptr, 3, pos, field, force, ids, vel, sink, grad, hid);
        sink.flush();
    } else {
        DirectSink<T, MODE> sink{fout, facc, 0.0};
        track_range<T, OPS, PER>(tv, start, end, nullptr, 3, pos, field, force, ids, vel, sink, grad, hid);
    }
}

template <typename T, int OPS, int MODE, int S>
void launch_track(const ot_tree *t, dim3 g, dim3 b, int64_t tile, hipStream_t s, int64_t n, const T *P, const T *Fd,
                  const T *Fo, int32_t *ids, T *V, T *O, const FxWs &ws, T *Gr, const int32_t *hid)
{
    if (t->view.periodic)
        hipLaunchKernelGGL((k_track<T, OPS, MODE, true, S>), g, b, 0, s, t->view, n, tile, P, Fd, Fo, ids, V, O,
                           ws.acc, ws.fx, Gr, hid);
    else
        hipLaunchKernelGGL((k_track<T, OPS, MODE, false, S>), g, b, 0, s, t->view, n, tile, P, Fd, Fo, ids, V, O,
                           ws.acc, ws.fx, Gr, hid);
}

template <typename T, int MODE>
int dispatch_ops(int ops, const ot_tree *t, dim3 g, dim3 b, int64_t tile, hipStream_t s, int64_t n, const void *pos,
                 const void *field, const void *force, int32_t *ids, void *vel, void *fout, void *grad,
                 const FxWs &ws, const int32_t *hid)
{
    const T *P = (const T *)pos, *Fd = (const T *)field, *Fo = (const T *)force;
    T *V = (T *)vel, *O = (T *)fout, *Gr = (T *)grad;
    constexpr int kSlots = SinkSlots<T, MODE>::value;
    const bool small = tile <= kSmallTile;
#define OT_LAUNCH(OPSV)                                                                                          \
    if (small)                                                                                                   \
        launch_track<T, OPSV, MODE, ((OPSV) & kOpSpread) ? kSmallSlots : kSlots>(t, g, b, tile, s, n, P, Fd, Fo,  \
                                                                                ids, V, O, ws, Gr, hid);          \
    else                                                                                                         \
        launch_track<T, OPSV, MODE, kSlots>(t, g, b, tile, s, n, P, Fd, Fo, ids, V, O, ws, Gr, hid);              \
    break;
    switch (ops) {
    case 1: OT_LAUNCH(1)
    case 2: OT_LAUNCH(2)
    case 3: OT_LAUNCH(3)
    case 4: OT_LAUNCH(4)
    case 5: OT_LAUNCH(5)
    case 6: OT_LAUNCH(6)
    case 7: OT_LAUNCH(7)
    // gradient passes: alone, with the interpolation (backward of spreading)
    // or with the spreading (backward of interpolation)
    case kOpGrad: OT_LAUNCH(kOpGrad)
    case kOpGrad | kOpInterp: OT_LAUNCH(kOpGrad | kOpInterp)
    case kOpGrad | kOpSpread: OT_LAUNCH(kOpGrad | kOpSpread)
    default: return fail(OT_ERR_INVALID, "ops must be a non-empty combination of OT_OP_* bits");
    }
#undef OT_LAUNCH
    return OT_OK;
}


}  // namespace ot
