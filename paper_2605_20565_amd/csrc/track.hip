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

// Launch of the plain kernels for one (precision, mode); instantiated in
// track_inst.hip (track_kernels.h).
template <typename T, int MODE>
int dispatch_ops(int ops, const ot_tree *t, dim3 g, dim3 b, int64_t tile, hipStream_t s, int64_t n, const void *pos,
                 const void *field, const void *force, int32_t *ids, void *vel, void *fout, void *grad,
                 const FxWs &ws, const int32_t *hid);

constexpr int kMaxPointsPerThread = 4;

// Prepare the spreading target before a pass: zero the output (atomic mode,
// overwrite) or the fixed-point accumulators and compute the scale.
namespace {

// Zero n 64-bit words at a and, in block 0, m 32-bit words at b: one launch
// for the fixed-point workspace (its header first, then the accumulators)
// and a batch plan's counters.
__global__ void k_zero2(unsigned long long *__restrict__ a, int64_t n, unsigned *__restrict__ b, int64_t m)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0ull;
    if (b && blockIdx.x == 0)
        for (int64_t i = threadIdx.x; i < m; i += blockDim.x) b[i] = 0u;
}

}  // namespace

int spread_begin(const ot_tree *t, const FxWs &ws, int dtype, int mode, int accumulate, void *fout, hipStream_t s,
                 unsigned *counters, int64_t n_counters)
{
    const int64_t n3 = t->n_leaves * 3;
    if (mode == OT_SPREAD_ATOMIC) {
        if (!accumulate) {
            if (dtype == OT_F32) hipLaunchKernelGGL(k_fill<float>, dim3(1024), dim3(256), 0, s, (float *)fout, n3, 0.0f);
            else hipLaunchKernelGGL(k_fill<double>, dim3(1024), dim3(256), 0, s, (double *)fout, n3, 0.0);
        }
        if (counters) hipLaunchKernelGGL(k_fill<unsigned>, dim3(1), dim3(64), 0, s, counters, n_counters, 0u);
    } else {
        // the whole header (max |F|, the non-finite flag; the scale is set
        // later) and the accumulators after it, and the counters
        hipLaunchKernelGGL(k_zero2, dim3(1024), dim3(256), 0, s, (unsigned long long *)ws.fx,
                           kFxHeader / 8 + n3, counters, n_counters);
    }
    OT_HIP(hipGetLastError());
    return OT_OK;
}

int spread_scale(const ot_tree *t, const FxWs &ws, int dtype, int mode, const void *force, int64_t n, hipStream_t s)
{
    (void)t;
    if (mode != OT_SPREAD_FIXED) return OT_OK;
    const int64_t m = force ? n * 3 : 0;
    if (m > 0) {
        unsigned gb = (unsigned)std::min<int64_t>((m + 1023) / 1024, 1024);
        if (dtype == OT_F32)
            hipLaunchKernelGGL(k_maxabs<float>, dim3(gb), dim3(256), 0, s, (const float *)force, m, &ws.fx->maxbits);
        else
            hipLaunchKernelGGL(k_maxabs<double>, dim3(gb), dim3(256), 0, s, (const double *)force, m, &ws.fx->maxbits);
    }
    if (dtype == OT_F32) hipLaunchKernelGGL(k_fx_prepare<float>, dim3(1), dim3(64), 0, s, ws.fx, n);
    else hipLaunchKernelGGL(k_fx_prepare<double>, dim3(1), dim3(64), 0, s, ws.fx, n);
    OT_HIP(hipGetLastError());
    return OT_OK;
}

int spread_prologue(const ot_tree *t, const FxWs &ws, int dtype, int mode, int accumulate, const void *force,
                    int64_t n, void *fout, hipStream_t s)
{
    int rc = spread_begin(t, ws, dtype, mode, accumulate, fout, s);
    return rc ? rc : spread_scale(t, ws, dtype, mode, force, n, s);
}

int spread_epilogue(const ot_tree *t, const FxWs &ws, int dtype, int mode, int accumulate, void *fout, hipStream_t s)
{
    if (mode != OT_SPREAD_FIXED) return OT_OK;
    const int64_t n3 = t->n_leaves * 3;
    const unsigned gb = (unsigned)std::min<int64_t>((n3 + 255) / 256, 8192);
    if (dtype == OT_F32)
        hipLaunchKernelGGL(k_fx_finalize<float>, dim3(gb), dim3(256), 0, s, ws.acc, (float *)fout, n3, ws.fx, accumulate);
    else
        hipLaunchKernelGGL(k_fx_finalize<double>, dim3(gb), dim3(256), 0, s, ws.acc, (double *)fout, n3, ws.fx, accumulate);
    OT_HIP(hipGetLastError());
    return OT_OK;
}

FxWs fx_ws(void *work)
{
    FxWs w;
    w.fx = (FxState *)work;
    w.acc = work ? (unsigned long long *)((char *)work + kFxHeader) : nullptr;
    return w;
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
               int mode, int32_t *ids, void *vel, void *fout, void *grad, const FxWs &ws, const int32_t *hid,
               hipStream_t s)
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
                     ? dispatch_ops<float, kModeFixed>(ops, t, g, b, tile, s, n, pos, field, force, ids, vel, fout, grad,
                                                       ws, hid)
                     : dispatch_ops<float, kModeAtomic>(ops, t, g, b, tile, s, n, pos, field, force, ids, vel, fout,
                                                        grad, ws, hid);
        else
            rc = mode == OT_SPREAD_FIXED
                     ? dispatch_ops<double, kModeFixed>(ops, t, g, b, tile, s, n, pos, field, force, ids, vel, fout,
                                                        grad, ws, hid)
                     : dispatch_ops<double, kModeAtomic>(ops, t, g, b, tile, s, n, pos, field, force, ids, vel, fout,
                                                         grad, ws, hid);
        if (rc) return rc;
        OT_HIP(hipGetLastError());
    }
    return OT_OK;
}

// One pass over the points with the ops in `ops` (OT_OP_* bits, or the
// gradient with at most one of interpolation and spreading).  hid: the
// caller's host ids (nullable).  work: the fixed-point spreading workspace
// (FIXED spreading only; NULL: allocated on the stream for this call).
int run_pass(const ot_tree *t, int ops, const void *field, const void *force, const void *pos, int dtype, int64_t n,
             int mode, int accumulate, int32_t *ids, void *vel, void *fout, void *grad, const int32_t *hid,
             void *work, hipStream_t s)
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
    const bool spread = (ops & kOpSpread) != 0;
    if (spread) {
        if ((n > 0 && !force) || !fout) return fail(OT_ERR_INVALID, "force or field_out is NULL");
        if (mode != OT_SPREAD_ATOMIC && mode != OT_SPREAD_FIXED) return fail(OT_ERR_INVALID, "bad spread mode");
    }
    if (work && ((uintptr_t)work & 255u)) return fail(OT_ERR_INVALID, "work must be 256-byte aligned");
    void *owned = nullptr;
    if (spread && mode == OT_SPREAD_FIXED && !work) {
        hipError_t e = hipMallocAsync(&owned, (size_t)spread_ws_bytes(t->n_leaves), s);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(OT_ERR_OOM, "fixed-point spreading workspace");
        }
        work = owned;
    }
    const FxWs ws = fx_ws(work);
    if (spread) rc = spread_prologue(t, ws, dtype, mode, accumulate, force, n, fout, s);
    if (!rc) rc = launch_ops(t, ops, field, force, pos, dtype, n, mode, ids, vel, fout, grad, ws, hid, s);
    if (!rc && spread) rc = spread_epilogue(t, ws, dtype, mode, accumulate, fout, s);
    if (owned) (void)hipFreeAsync(owned, s);
    return rc;
}

}  // namespace

}  // namespace ot

using namespace ot;

extern "C" int64_t ot_spread_workspace_bytes(const ot_tree *t)
{
    return t ? spread_ws_bytes(t->n_leaves) : 0;
}

extern "C" int ot_locate(const ot_tree *t, const void *pos, int32_t dtype, int64_t n, int32_t *ids, void *stream)
{
    return run_pass(t, kOpLocate, nullptr, nullptr, pos, dtype, n, OT_SPREAD_ATOMIC, 0, ids, nullptr, nullptr, nullptr,
                    nullptr, nullptr, (hipStream_t)stream);
}

extern "C" int ot_interpolate(const ot_tree *t, const void *field, const void *pos, const int32_t *ids,
                              int32_t dtype, int64_t n, void *vel, void *stream)
{
    return run_pass(t, kOpInterp, field, nullptr, pos, dtype, n, OT_SPREAD_ATOMIC, 0, nullptr, vel, nullptr, nullptr,
                    ids, nullptr, (hipStream_t)stream);
}

extern "C" int ot_spread(const ot_tree *t, const void *force, const void *pos, const int32_t *ids, int32_t dtype,
                         int64_t n, int32_t mode, int32_t accumulate, void *field_out, void *work, void *stream)
{
    return run_pass(t, kOpSpread, nullptr, force, pos, dtype, n, mode, accumulate, nullptr, nullptr, field_out,
                    nullptr, ids, work, (hipStream_t)stream);
}

extern "C" int ot_track(const ot_tree *t, int32_t ops, const void *field, const void *force, const void *pos,
                        int32_t dtype, int64_t n, int32_t mode, int32_t accumulate, int32_t *ids, void *vel,
                        void *field_out, void *work, void *stream)
{
    if (ops <= 0 || ops > 7) return fail(OT_ERR_INVALID, "ops must be a non-empty combination of OT_OP_* bits");
    return run_pass(t, ops, field, force, pos, dtype, n, mode, accumulate, ids, vel, field_out, nullptr, nullptr, work,
                    (hipStream_t)stream);
}

extern "C" int ot_grad_pos(const ot_tree *t, const void *field, const void *vec, const void *pos, const int32_t *ids,
                           int32_t dtype, int64_t n, void *grad, void *stream)
{
    return run_pass(t, kOpGrad, field, vec, pos, dtype, n, OT_SPREAD_ATOMIC, 0, nullptr, nullptr, nullptr, grad, ids,
                    nullptr, (hipStream_t)stream);
}

extern "C" int ot_interp_grad_pos(const ot_tree *t, const void *field, const void *grad_vel, const void *pos,
                                  const int32_t *ids, int32_t dtype, int64_t n, void *grad_pos, void *stream)
{
    return ot_grad_pos(t, field, grad_vel, pos, ids, dtype, n, grad_pos, stream);
}

extern "C" int ot_spread_grad_pos(const ot_tree *t, const void *grad_field, const void *force, const void *pos,
                                  const int32_t *ids, int32_t dtype, int64_t n, void *grad_pos, void *stream)
{
    return ot_grad_pos(t, grad_field, force, pos, ids, dtype, n, grad_pos, stream);
}

extern "C" int ot_interp_backward(const ot_tree *t, const void *field, const void *grad_vel, const void *pos,
                                  const int32_t *ids, int32_t dtype, int64_t n, int32_t mode, int32_t accumulate,
                                  void *grad_field, void *grad_pos, void *work, void *stream)
{
    int ops = (grad_field ? (int)kOpSpread : 0) | (grad_pos ? (int)kOpGrad : 0);
    if (n == 0) ops &= ~(int)kOpGrad;   // no points: no position gradient (grad_field is still cleared)
    if (!ops) {
        if (n == 0) return check_common(t, dtype, n, pos);
        return fail(OT_ERR_INVALID, "ot_interp_backward: both outputs are NULL");
    }
    return run_pass(t, ops, field, grad_vel, pos, dtype, n, mode, accumulate, nullptr, nullptr, grad_field, grad_pos,
                    ids, work, (hipStream_t)stream);
}

extern "C" int ot_spread_backward(const ot_tree *t, const void *grad_field, const void *force, const void *pos,
                                  const int32_t *ids, int32_t dtype, int64_t n, void *grad_force, void *grad_pos,
                                  void *stream)
{
    const int ops = (grad_force ? (int)kOpInterp : 0) | (grad_pos ? (int)kOpGrad : 0);
    if (n == 0) return check_common(t, dtype, n, pos);   // both outputs are per point: nothing to do
    if (!ops) return fail(OT_ERR_INVALID, "ot_spread_backward: both outputs are NULL");
    return run_pass(t, ops, grad_field, force, pos, dtype, n, OT_SPREAD_ATOMIC, 0, nullptr, grad_force, nullptr,
                    grad_pos, ids, nullptr, (hipStream_t)stream);
}
