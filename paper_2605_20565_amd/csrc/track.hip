// Host-cell search, interpolation, spreading and the position gradient.
//
// One thread per Lagrangian point.  A point's integer cell is floor(x 2^L)
// in FP64 (so that a face decision never flips between precisions), its host
// leaf comes from the descent table (Sec. 3.2 / Algorithm 1 semantics), and
// the 3x3x3 stencil at the host level uses the 3-point delta function of
// Sec. 2.2.  Interpolation gathers the 27 node values; spreading scatters
// w F to the same 27 node leaves (atomics in the working precision, or
// int64 fixed point for order-independent sums).
#include <hip/hip_runtime.h>

#include "ot_common.h"
#include "track_device.h"

namespace ot {

namespace {

// One workgroup per tile of `tile` consecutive points.  Spreading goes
// through the workgroup's LDS aggregation table of S slots, flushed once at
// the end.
template <typename T, int OPS, int MODE, bool PER, int S>
__global__ __launch_bounds__(512) void k_track(TreeView tv, int64_t n, int64_t tile, const T *__restrict__ pos,
                                               const T *__restrict__ field, const T *__restrict__ force,
                                               int32_t *__restrict__ ids, T *__restrict__ vel,
                                               T *__restrict__ fout, unsigned long long *__restrict__ facc,
                                               const FxState *__restrict__ fx, T *__restrict__ grad)
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
        track_range<T, OPS, PER>(tv, start, end, nullptr, 3, pos, field, force, ids, vel, sink, grad);
        sink.flush();
    } else {
        DirectSink<T, MODE> sink{fout, facc, 0.0};
        track_range<T, OPS, PER>(tv, start, end, nullptr, 3, pos, field, force, ids, vel, sink, grad);
    }
}

constexpr int kMaxPointsPerThread = 4;

template <typename T, int OPS, int MODE, int S>
void launch_track(const ot_tree *t, dim3 g, dim3 b, int64_t tile, hipStream_t s, int64_t n, const T *P, const T *Fd,
                  const T *Fo, int32_t *ids, T *V, T *O, const FxState *fx, T *Gr)
{
    if (t->view.periodic)
        hipLaunchKernelGGL((k_track<T, OPS, MODE, true, S>), g, b, 0, s, t->view, n, tile, P, Fd, Fo, ids, V, O,
                           t->fx_acc, fx, Gr);
    else
        hipLaunchKernelGGL((k_track<T, OPS, MODE, false, S>), g, b, 0, s, t->view, n, tile, P, Fd, Fo, ids, V, O,
                           t->fx_acc, fx, Gr);
}

template <typename T, int MODE>
int dispatch_ops(int ops, const ot_tree *t, dim3 g, dim3 b, int64_t tile, hipStream_t s, int64_t n, const void *pos,
                 const void *field, const void *force, int32_t *ids, void *vel, void *fout, void *grad)
{
    const T *P = (const T *)pos, *Fd = (const T *)field, *Fo = (const T *)force;
    T *V = (T *)vel, *O = (T *)fout, *Gr = (T *)grad;
    const FxState *fx = (const FxState *)t->scratch;
    constexpr int kSlots = SinkSlots<T, MODE>::value;
    const bool small = tile <= kSmallTile;
#define OT_LAUNCH(OPSV)                                                                                          \
    if (small)                                                                                                   \
        launch_track<T, OPSV, MODE, ((OPSV) & kOpSpread) ? kSmallSlots : kSlots>(t, g, b, tile, s, n, P, Fd, Fo,  \
                                                                                ids, V, O, fx, Gr);               \
    else                                                                                                         \
        launch_track<T, OPSV, MODE, kSlots>(t, g, b, tile, s, n, P, Fd, Fo, ids, V, O, fx, Gr);                   \
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

}  // namespace

// Prepare the spreading target before a pass: zero the output (atomic mode,
// overwrite) or the fixed-point accumulators and compute the scale.
int spread_begin(const ot_tree *t, int dtype, int mode, int accumulate, void *fout, hipStream_t s)
{
    const int64_t n3 = t->n_leaves * 3;
    FxState *fx = (FxState *)t->scratch;
    if (mode == OT_SPREAD_ATOMIC) {
        if (!accumulate) {
            if (dtype == OT_F32) hipLaunchKernelGGL(k_fill<float>, dim3(1024), dim3(256), 0, s, (float *)fout, n3, 0.0f);
            else hipLaunchKernelGGL(k_fill<double>, dim3(1024), dim3(256), 0, s, (double *)fout, n3, 0.0);
        }
    } else {
        hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(1024), dim3(256), 0, s, t->fx_acc, n3, 0ull);
        hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(1), dim3(64), 0, s, &fx->maxbits, (int64_t)1, 0ull);
    }
    OT_HIP(hipGetLastError());
    return OT_OK;
}

int spread_scale(const ot_tree *t, int dtype, int mode, const void *force, int64_t n, hipStream_t s)
{
    if (mode != OT_SPREAD_FIXED) return OT_OK;
    FxState *fx = (FxState *)t->scratch;
    const int64_t m = force ? n * 3 : 0;
    if (m > 0) {
        unsigned gb = (unsigned)std::min<int64_t>((m + 1023) / 1024, 1024);
        if (dtype == OT_F32)
            hipLaunchKernelGGL(k_maxabs<float>, dim3(gb), dim3(256), 0, s, (const float *)force, m, &fx->maxbits);
        else
            hipLaunchKernelGGL(k_maxabs<double>, dim3(gb), dim3(256), 0, s, (const double *)force, m, &fx->maxbits);
    }
    if (dtype == OT_F32) hipLaunchKernelGGL(k_fx_prepare<float>, dim3(1), dim3(64), 0, s, fx, n);
    else hipLaunchKernelGGL(k_fx_prepare<double>, dim3(1), dim3(64), 0, s, fx, n);
    OT_HIP(hipGetLastError());
    return OT_OK;
}

int spread_prologue(const ot_tree *t, int dtype, int mode, int accumulate, const void *force, int64_t n,
                    void *fout, hipStream_t s)
{
    int rc = spread_begin(t, dtype, mode, accumulate, fout, s);
    return rc ? rc : spread_scale(t, dtype, mode, force, n, s);
}

int spread_epilogue(const ot_tree *t, int dtype, int mode, int accumulate, void *fout, hipStream_t s)
{
    if (mode != OT_SPREAD_FIXED) return OT_OK;
    const int64_t n3 = t->n_leaves * 3;
    const FxState *fx = (const FxState *)t->scratch;
    const unsigned gb = (unsigned)std::min<int64_t>((n3 + 255) / 256, 8192);
    if (dtype == OT_F32)
        hipLaunchKernelGGL(k_fx_finalize<float>, dim3(gb), dim3(256), 0, s, t->fx_acc, (float *)fout, n3, fx, accumulate);
    else
        hipLaunchKernelGGL(k_fx_finalize<double>, dim3(gb), dim3(256), 0, s, t->fx_acc, (double *)fout, n3, fx, accumulate);
    OT_HIP(hipGetLastError());
    return OT_OK;
}

int check_common(const ot_tree *t, int dtype, int64_t n, const void *pos)
{
    if (!t) return fail(OT_ERR_INVALID, "tree is NULL");
    if (dtype != OT_F32 && dtype != OT_F64) return fail(OT_ERR_INVALID, "dtype must be OT_F32 or OT_F64");
    if (n < 0) return fail(OT_ERR_INVALID, "n < 0");
    if (n > 0 && !pos) return fail(OT_ERR_INVALID, "pos is NULL");
    if (n > (int64_t(1) << 40)) return fail(OT_ERR_CAPACITY, "too many points");
    return OT_OK;
}

namespace {

// The pass's kernel alone, no clearing, scale or conversion around it.
int launch_ops(const ot_tree *t, int ops, const void *field, const void *force, const void *pos, int dtype, int64_t n,
               int mode, int32_t *ids, void *vel, void *fout, void *grad, hipStream_t s)
{
    int rc = OT_OK;
    if (n > 0) {
        // Enough workgroups to give every CU two, when there are points for
        // them: small sets get narrower workgroups and one point per thread
        // (their time is latency, not throughput); large ones up to
        // kMaxPointsPerThread points per thread.
        const int64_t want = 2 * (int64_t)t->cus;
        int threads = 256;
        while (threads > 64 && (n + threads - 1) / threads < want) threads >>= 1;
        const int64_t ppt = std::max<int64_t>(1, std::min<int64_t>(kMaxPointsPerThread, n / ((int64_t)threads * want)));
        const int64_t tile = (int64_t)threads * ppt;
        dim3 b(threads), g((unsigned)((n + tile - 1) / tile));
        if (dtype == OT_F32)
            rc = mode == OT_SPREAD_FIXED
                     ? dispatch_ops<float, kModeFixed>(ops, t, g, b, tile, s, n, pos, field, force, ids, vel, fout, grad)
                     : dispatch_ops<float, kModeAtomic>(ops, t, g, b, tile, s, n, pos, field, force, ids, vel, fout, grad);
        else
            rc = mode == OT_SPREAD_FIXED
                     ? dispatch_ops<double, kModeFixed>(ops, t, g, b, tile, s, n, pos, field, force, ids, vel, fout, grad)
                     : dispatch_ops<double, kModeAtomic>(ops, t, g, b, tile, s, n, pos, field, force, ids, vel, fout, grad);
        if (rc) return rc;
        OT_HIP(hipGetLastError());
    }
    return OT_OK;
}

// One pass over the points with the ops in `ops` (OT_OP_* bits, or the
// gradient with at most one of interpolation and spreading).
int run_pass(const ot_tree *t, int ops, const void *field, const void *force, const void *pos, int dtype, int64_t n,
             int mode, int accumulate, int32_t *ids, void *vel, void *fout, void *grad, hipStream_t s)
{
    int rc = check_common(t, dtype, n, pos);
    if (rc) return rc;
    const bool ops_ok = (ops > 0 && ops <= 7) || ops == kOpGrad || ops == (kOpGrad | kOpInterp) ||
                        ops == (kOpGrad | kOpSpread);
    if (!ops_ok) return fail(OT_ERR_INVALID, "ops must be a non-empty combination of OT_OP_* bits");
    if ((ops & kOpLocate) && n > 0 && !ids) return fail(OT_ERR_INVALID, "ids is NULL");
    if ((ops & kOpInterp) && ((n > 0 && !vel) || !field)) return fail(OT_ERR_INVALID, "field or vel is NULL");
    if ((ops & kOpGrad) && ((n > 0 && (!grad || !force)) || !field))
        return fail(OT_ERR_INVALID, "field, vector or gradient output is NULL");
    if (ops & kOpSpread) {
        if ((n > 0 && !force) || !fout) return fail(OT_ERR_INVALID, "force or field_out is NULL");
        if (mode != OT_SPREAD_ATOMIC && mode != OT_SPREAD_FIXED) return fail(OT_ERR_INVALID, "bad spread mode");
        if ((rc = spread_prologue(t, dtype, mode, accumulate, force, n, fout, s))) return rc;
    }
    if ((rc = launch_ops(t, ops, field, force, pos, dtype, n, mode, ids, vel, fout, grad, s))) return rc;
    if (ops & kOpSpread) return spread_epilogue(t, dtype, mode, accumulate, fout, s);
    return OT_OK;
}

}  // namespace

int track(const ot_tree *t, int ops, const void *field, const void *force, const void *pos, int dtype, int64_t n,
          int mode, int accumulate, int32_t *ids, void *vel, void *fout, hipStream_t s)
{
    if (ops <= 0 || ops > 7) return fail(OT_ERR_INVALID, "ops must be a non-empty combination of OT_OP_* bits");
    return run_pass(t, ops, field, force, pos, dtype, n, mode, accumulate, ids, vel, fout, nullptr, s);
}

}  // namespace ot

using namespace ot;

extern "C" int ot_locate(const ot_tree *t, const void *pos, int32_t dtype, int64_t n, int32_t *ids, void *stream)
{
    return track(t, kOpLocate, nullptr, nullptr, pos, dtype, n, OT_SPREAD_ATOMIC, 0, ids, nullptr, nullptr,
                 (hipStream_t)stream);
}

extern "C" int ot_interpolate(const ot_tree *t, const void *field, const void *pos, int32_t dtype, int64_t n,
                              void *vel, void *stream)
{
    return track(t, kOpInterp, field, nullptr, pos, dtype, n, OT_SPREAD_ATOMIC, 0, nullptr, vel, nullptr,
                 (hipStream_t)stream);
}

extern "C" int ot_spread(const ot_tree *t, const void *force, const void *pos, int32_t dtype, int64_t n, int32_t mode,
                         int32_t accumulate, void *field_out, void *stream)
{
    return track(t, kOpSpread, nullptr, force, pos, dtype, n, mode, accumulate, nullptr, nullptr, field_out,
                 (hipStream_t)stream);
}

extern "C" int ot_track(const ot_tree *t, int32_t ops, const void *field, const void *force, const void *pos,
                        int32_t dtype, int64_t n, int32_t mode, int32_t accumulate, int32_t *ids, void *vel,
                        void *field_out, void *stream)
{
    return track(t, ops, field, force, pos, dtype, n, mode, accumulate, ids, vel, field_out, (hipStream_t)stream);
}

extern "C" int ot_grad_pos(const ot_tree *t, const void *field, const void *vec, const void *pos, int32_t dtype,
                           int64_t n, void *grad, void *stream)
{
    return run_pass(t, kOpGrad, field, vec, pos, dtype, n, OT_SPREAD_ATOMIC, 0, nullptr, nullptr, nullptr, grad,
                    (hipStream_t)stream);
}

extern "C" int ot_interp_backward(const ot_tree *t, const void *field, const void *grad_vel, const void *pos,
                                  int32_t dtype, int64_t n, int32_t mode, int32_t accumulate, void *grad_field,
                                  void *grad_pos, void *stream)
{
    int ops = (grad_field ? (int)kOpSpread : 0) | (grad_pos ? (int)kOpGrad : 0);
    if (n == 0) ops &= ~(int)kOpGrad;   // no points: no position gradient (grad_field is still cleared)
    if (!ops) {
        if (n == 0) return check_common(t, dtype, n, pos);
        return fail(OT_ERR_INVALID, "ot_interp_backward: both outputs are NULL");
    }
    return run_pass(t, ops, field, grad_vel, pos, dtype, n, mode, accumulate, nullptr, nullptr, grad_field, grad_pos,
                    (hipStream_t)stream);
}

extern "C" int ot_spread_backward(const ot_tree *t, const void *grad_field, const void *force, const void *pos,
                                  int32_t dtype, int64_t n, void *grad_force, void *grad_pos, void *stream)
{
    const int ops = (grad_force ? (int)kOpInterp : 0) | (grad_pos ? (int)kOpGrad : 0);
    if (n == 0) return check_common(t, dtype, n, pos);   // both outputs are per point: nothing to do
    if (!ops) return fail(OT_ERR_INVALID, "ot_spread_backward: both outputs are NULL");
    return run_pass(t, ops, grad_field, force, pos, dtype, n, OT_SPREAD_ATOMIC, 0, nullptr, grad_force, nullptr,
                    grad_pos, (hipStream_t)stream);
}
