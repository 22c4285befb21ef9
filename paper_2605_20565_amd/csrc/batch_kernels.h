// The persistent batched kernel and its enqueue sequence, templated on
// precision and spreading mode.  batch_inst.hip instantiates enqueue<T, MODE>
// and kbatch_fn<T, MODE> once per (T, MODE) in its own object file; the host
// code of the plans (batch.hip) calls them.
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "batch_plan.h"
#include "hm_pass.h"
#include "ot_common.h"
#include "point_sort.h"
#include "track_device.h"


namespace ot {


// Tiles handed over by the host-major pass: window indices and their count
// (device), the window size, the number of points and the common ops.
struct FbTiles {
    const uint32_t *list;
    const unsigned *count;
    int64_t pts, n;
    uint32_t ops;
};

// GRAD: the plan's ops are gradient passes (8, 10, 12), else forward (1..7).
// S: slots of the workgroup's spreading table.  fb.list != null: the tiles
// are the windows the host-major pass handed over, not the plan's table.
template <typename T, int MODE, bool PER, bool GRAD, int S>
__global__ __launch_bounds__(512) void k_batch(TreeView tv, const int64_t *__restrict__ tile_start,
                                               const uint32_t *__restrict__ tile_info, int64_t n_tiles,
                                               unsigned *__restrict__ counter, const uint64_t *__restrict__ kv,
                                               int rs, const T *__restrict__ pos,
                                               const T *__restrict__ field, const T *__restrict__ force,
                                               int32_t *__restrict__ ids, T *__restrict__ vel, T *__restrict__ fout,
                                               unsigned long long *__restrict__ facc, const FxState *__restrict__ fx,
                                               T *__restrict__ grad, FbTiles fb)
{
    if (fb.list) n_tiles = *fb.count;
    using Acc = typename AccType<T, MODE>::type;
    __shared__ uint32_t keys[S];
    __shared__ Acc vals[LdsSink<T, MODE, S>::kVals];
    __shared__ unsigned s_tile;
    // the fixed-point state exists only for plans that spread (fx null otherwise)
    const double scale = (MODE == kModeFixed && fx) ? fx->scale : 0.0;
    LdsSink<T, MODE, S> sink{keys, vals, fout, facc, scale};
    sink.clear();
    // The next tile is claimed before the flush, so the queue atomic's round
    // trip overlaps it.  Every thread reads s_tile before the flush's first
    // barrier, and thread 0 writes it again only after the flush's last one.
    unsigned nxt = 0u;
    if (threadIdx.x == 0) nxt = atomicAdd(counter, 1u);
    for (;;) {
        if (threadIdx.x == 0) s_tile = nxt;
        __syncthreads();
        const int64_t tile = s_tile;
        if (tile >= n_tiles) break;   // same value in every thread of the workgroup
        int64_t start, end;
        uint32_t info;
        if (fb.list) {
            start = (int64_t)fb.list[tile] * fb.pts;
            end = start + fb.pts < fb.n ? start + fb.pts : fb.n;
            info = fb.ops << 24;
        } else {
            start = tile_start[tile];
            info = tile_info[tile];
            end = start + (int64_t)(info & kCountMask);
        }
        if constexpr (!GRAD) {
            switch (info >> 24) {
#define OT_CASE(OPSV) \
    case OPSV: track_range<T, OPSV, PER>(tv, start, end, kv, rs, pos, field, force, ids, vel, sink); break;
                OT_CASE(1) OT_CASE(2) OT_CASE(3) OT_CASE(4) OT_CASE(5) OT_CASE(6) OT_CASE(7)
#undef OT_CASE
            default: break;
            }
        } else {
            switch (info >> 24) {
#define OT_CASE(OPSV) \
    case OPSV: track_range<T, OPSV, PER>(tv, start, end, kv, rs, pos, field, force, ids, vel, sink, grad); break;
                OT_CASE(kOpGrad) OT_CASE(kOpGrad | kOpInterp) OT_CASE(kOpGrad | kOpSpread)
#undef OT_CASE
            default: break;
            }
        }
        if (threadIdx.x == 0) nxt = atomicAdd(counter, 1u);
        sink.flush();   // one spatially coherent tile per table fill
    }
}

template <typename T, int MODE>
int enqueue(ot_batch_plan *p, const void *field, const void *force, const void *pos, int32_t *ids, void *vel,
            void *fout, void *grad, hipStream_t s)
{
    const ot_tree *t = p->tree;
    const int64_t n = p->n_points;
    // counter[0]: the pass's tile queue, [1]: the per-point pass over handed-over
    // windows, [2]: how many windows were handed over
    int rc;
    const bool spread = (p->ops_union & kOpSpread) != 0;
    const FxWs ws = fx_ws(p->fxws);
    if (spread) {
        if ((rc = spread_begin(t, ws, p->dtype, p->mode, 0, fout, s, p->counter, 3))) return rc;
    } else {
        hipLaunchKernelGGL(k_fill<unsigned>, dim3(1), dim3(64), 0, s, p->counter, (int64_t)3, 0u);
    }
    const uint64_t *kv = nullptr;
    int rs = 3;
    int32_t *kids = ids;
    const T *kpos = (const T *)pos, *kforce = (const T *)force;
    const void *scale_from = force;   // max |F| still to take (FIXED)
    if (p->sort_points && n > 0) {
        // ids come from the key pass; positions and forces travel with the
        // keys, and the first pass takes max |F| on the way
        const bool carry_force = (p->ops_all & (kOpSpread | kOpGrad)) != 0;
        PointSortBufs<T> b{{p->skv[0], p->skv[1]}, {(T *)p->srec[0], (T *)p->srec[1]}, p->sws};
        PointSortResult<T> r;
        unsigned long long *maxbits = ((p->ops_all & kOpSpread) && p->mode == OT_SPREAD_FIXED)
                                          ? &ws.fx->maxbits
                                          : nullptr;
        point_sort<T>(t->view, n, t->n_leaves, p->sort_shift, p->sort_bits, (const T *)pos,
                      carry_force ? (const T *)force : nullptr, (p->ops_all & kOpLocate) ? ids : nullptr, b, maxbits,
                      s, r);
        kv = r.kv;
        rs = r.stride;
        kpos = r.rec;
        kforce = carry_force ? r.rec + 3 : nullptr;
        kids = nullptr;
        if (maxbits) scale_from = nullptr;
    }
    if (spread && (rc = spread_scale(t, ws, p->dtype, p->mode, scale_from, n, s))) return rc;
    if (p->timing) OT_HIP(hipEventRecord(p->ev[0], s));
    if (p->use_hm && n > 0) {
        const int sops = p->ops_all & (kOpInterp | kOpSpread);
#define OT_KHM(PERV, OPSV)                                                                                         \
    hipLaunchKernelGGL((k_hm<T, MODE, PERV, OPSV>), dim3(p->hm_grid), dim3(kHmThreads), 0, s, t->view, n, p->n_win,  \
                       p->counter, kv, rs, kpos, (const T *)field, (T *)vel, (T *)fout, ws.acc, ws.fx, p->fb_list,  \
                       p->counter + 2)
        if (t->view.periodic) {
            if (sops == kOpInterp) OT_KHM(true, kOpInterp);
            else if (sops == kOpSpread) OT_KHM(true, kOpSpread);
            else OT_KHM(true, kOpInterp | kOpSpread);
        } else {
            if (sops == kOpInterp) OT_KHM(false, kOpInterp);
            else if (sops == kOpSpread) OT_KHM(false, kOpSpread);
            else OT_KHM(false, kOpInterp | kOpSpread);
        }
#undef OT_KHM
        OT_HIP(hipGetLastError());
        // windows the host-major pass handed over, per point
        const FbTiles fb{p->fb_list, p->counter + 2, (int64_t)kHmThreads, n, (uint32_t)sops};
        constexpr int kS = SinkSlots<T, MODE>::value;
        if (t->view.periodic)
            hipLaunchKernelGGL((k_batch<T, MODE, true, false, kS>), dim3(p->grid), dim3(kHmThreads), 0, s, t->view,
                               p->tile_start, p->tile_info, (int64_t)0, p->counter + 1, kv, rs, kpos, (const T *)field,
                               kforce, (int32_t *)nullptr, (T *)vel, (T *)fout, ws.acc, ws.fx, (T *)nullptr, fb);
        else
            hipLaunchKernelGGL((k_batch<T, MODE, false, false, kS>), dim3(p->grid), dim3(kHmThreads), 0, s, t->view,
                               p->tile_start, p->tile_info, (int64_t)0, p->counter + 1, kv, rs, kpos, (const T *)field,
                               kforce, (int32_t *)nullptr, (T *)vel, (T *)fout, ws.acc, ws.fx, (T *)nullptr, fb);
        OT_HIP(hipGetLastError());
        if (p->timing) OT_HIP(hipEventRecord(p->ev[1], s));
        if (spread && (rc = spread_epilogue(t, ws, p->dtype, p->mode, 0, fout, s))) return rc;
        OT_HIP(hipGetLastError());
        return OT_OK;
    }
#define OT_KBATCH_S(PERV, GRADV, SV)                                                                               \
    hipLaunchKernelGGL((k_batch<T, MODE, PERV, GRADV, SV>), dim3(p->grid), dim3(p->block), 0, s, t->view,            \
                       p->tile_start, p->tile_info, p->n_tiles, p->counter, kv, rs, kpos, (const T *)field, kforce,  \
                       kids, (T *)vel, (T *)fout, ws.acc, ws.fx, (T *)grad, FbTiles{})
#define OT_KBATCH(PERV, GRADV)                                                                                     \
    do {                                                                                                           \
        if (p->small_table) OT_KBATCH_S(PERV, GRADV, kSmallSlots);                                                \
        else OT_KBATCH_S(PERV, GRADV, (SinkSlots<T, MODE>::value));                                                \
    } while (0)
    if (p->grad_plan) {
        if (t->view.periodic) OT_KBATCH(true, true);
        else OT_KBATCH(false, true);
    } else {
        if (t->view.periodic) OT_KBATCH(true, false);
        else OT_KBATCH(false, false);
    }
#undef OT_KBATCH
#undef OT_KBATCH_S
    OT_HIP(hipGetLastError());
    if (p->timing) OT_HIP(hipEventRecord(p->ev[1], s));
    if (p->ops_union & kOpSpread)
        if ((rc = spread_epilogue(t, ws, p->dtype, p->mode, 0, fout, s))) return rc;
    OT_HIP(hipGetLastError());
    return OT_OK;
}

// The host-major kernel of a plan (for the occupancy query).
template <typename T, int MODE>
const void *hm_fn(int ops)
{
    if (ops == kOpInterp) return (const void *)k_hm<T, MODE, true, kOpInterp>;
    if (ops == kOpSpread) return (const void *)k_hm<T, MODE, true, kOpSpread>;
    return (const void *)k_hm<T, MODE, true, kOpInterp | kOpSpread>;
}

// The persistent kernel of a plan (for the occupancy query).
template <typename T, int MODE>
const void *kbatch_fn(bool grad, bool small)
{
    constexpr int L = SinkSlots<T, MODE>::value;
    if (grad) return small ? (const void *)k_batch<T, MODE, true, true, kSmallSlots> : (const void *)k_batch<T, MODE, true, true, L>;
    return small ? (const void *)k_batch<T, MODE, true, false, kSmallSlots> : (const void *)k_batch<T, MODE, true, false, L>;
}

}  // namespace ot
