// Batched tracking of many point sets of uneven size in one persistent
// launch.  The paper's bubble/particle workloads mix a few hundred bubbles
// with 10^2..10^4 markers each and particle groups of 10^4..10^6 points
// (bubble-driven load imbalance, Sec. 5.2); launching one kernel per set
// leaves the chip idle on the small ones.  Here the sets are cut into tiles
// that never straddle a set, a fixed grid of workgroups pulls tiles from a
// device counter until none are left, and the whole sequence (clears,
// fixed-point scale, persistent kernel, finalize) is captured once in a HIP
// graph and replayed.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "batch_plan.h"
#include "ot_common.h"
#include "point_sort.h"
#include "track_device.h"


namespace ot {

// Instantiated in batch_inst.hip (batch_kernels.h).
template <typename T, int MODE>
int enqueue(ot_batch_plan *p, const void *field, const void *force, const void *pos, int32_t *ids, void *vel,
            void *fout, void *grad, hipStream_t s);
template <typename T, int MODE>
const void *kbatch_fn(bool grad, bool small);
template <typename T, int MODE>
const void *hm_fn(int ops);
constexpr int kHmWindow = 256;   // points per window of the host-major pass (kHmThreads)

namespace {

int enqueue_any(ot_batch_plan *p, const void *field, const void *force, const void *pos, int32_t *ids, void *vel,
                void *fout, void *grad, hipStream_t s)
{
    if (p->dtype == OT_F32)
        return p->mode == OT_SPREAD_FIXED ? enqueue<float, kModeFixed>(p, field, force, pos, ids, vel, fout, grad, s)
                                          : enqueue<float, kModeAtomic>(p, field, force, pos, ids, vel, fout, grad, s);
    return p->mode == OT_SPREAD_FIXED ? enqueue<double, kModeFixed>(p, field, force, pos, ids, vel, fout, grad, s)
                                      : enqueue<double, kModeAtomic>(p, field, force, pos, ids, vel, fout, grad, s);
}

bool valid_ops(int o)
{
    return (o >= 0 && o <= 7) || o == kOpGrad || o == (kOpGrad | kOpInterp) || o == (kOpGrad | kOpSpread);
}

void drop_graph(ot_batch_plan *p)
{
    if (p->have_graph) {
        (void)hipGraphExecDestroy(p->exec);
        (void)hipGraphDestroy(p->graph);
        p->have_graph = false;
    }
}

}  // namespace
}  // namespace ot

using namespace ot;

extern "C" int ot_batch_plan_create(const ot_tree *tree, const int64_t *offsets, const int32_t *ops, int32_t n_inst,
                                    int32_t dtype, int32_t mode, const ot_tuning *tuning, ot_batch_plan **out)
{
    if (!out) return fail(OT_ERR_INVALID, "ot_batch_plan_create: out is NULL");
    *out = nullptr;
    if (!tree || !offsets || !ops || n_inst <= 0) return fail(OT_ERR_INVALID, "ot_batch_plan_create: bad arguments");
    if (dtype != OT_F32 && dtype != OT_F64) return fail(OT_ERR_INVALID, "dtype must be OT_F32 or OT_F64");
    if (mode != OT_SPREAD_ATOMIC && mode != OT_SPREAD_FIXED) return fail(OT_ERR_INVALID, "bad spread mode");
    int kinds = 0;   // bit 0: forward-only ops, bit 1: gradient ops
    for (int i = 0; i < n_inst; ++i) {
        if (!valid_ops(ops[i])) return fail(OT_ERR_INVALID, "bad per-instance ops");
        if (ops[i]) kinds |= (ops[i] & kOpGrad) ? 2 : 1;
    }
    if (kinds == 3) return fail(OT_ERR_INVALID, "gradient and forward-only ops cannot share a plan");
    const bool sort_points = tuning && (tuning->flags & OT_TUNE_SORT_POINTS);
    // defaults: 256 threads and up to 4 points per thread, narrower and
    // shorter tiles when there are too few points for two workgroups per CU
    // (measured: 256 x 512-1024 beats 512 x 2048 by 15-20% on large sets,
    // where two 56 KiB tables per CU leave 512-thread groups few waves)
    const int64_t want = 2 * (int64_t)tree->cus;
    const int64_t n_all = offsets[n_inst] > 0 ? offsets[n_inst] : 0;
    int block = 256;
    while (block > 64 && (n_all + block - 1) / block < want) block >>= 1;
    if (tuning && tuning->block) block = tuning->block;
    int tile = (int)(block * std::max<int64_t>(1, std::min<int64_t>(4, n_all / ((int64_t)block * want))));
    if (sort_points && tree->n_leaves > 0) {
        // sorted tiles: about 160 points per point-per-leaf of the run, the
        // power of two nearest to it within [block, 4 block], so that a
        // tile's stencil nodes fit the 2048-slot spreading table (autotuned
        // on the workloads: 256 at ~1 point per leaf, 512 at ~4, 1024 at ~5
        // with 26 per finest leaf)
        const double target = 160.0 * (double)n_all / (double)tree->n_leaves;
        int t = block;
        while (t < 4 * block && (double)(2 * t) <= target * 1.41421356) t *= 2;
        tile = std::min(tile, t);
    }
    if (tuning && tuning->tile) tile = tuning->tile;
    if (block < 64 || block > 512 || block % 64) return fail(OT_ERR_INVALID, "block must be a multiple of 64 in [64, 512]");
    if (tile < block || tile % block || tile > (int)kCountMask) return fail(OT_ERR_INVALID, "tile must be a multiple of block");
    if (offsets[0] != 0) return fail(OT_ERR_INVALID, "offsets[0] must be 0");
    if (sort_points && offsets[n_inst] > (int64_t)INT32_MAX)
        return fail(OT_ERR_CAPACITY, "point sorting indexes points with int32: at most 2^31 - 1 points");
    std::vector<int64_t> starts;
    std::vector<uint32_t> infos;
    int ops_union = 0, ops_all = -1;
    for (int i = 0; i < n_inst; ++i) {
        if (offsets[i + 1] < offsets[i]) return fail(OT_ERR_INVALID, "offsets must be ascending");
        // the sorted pass covers every point of the run with the common ops,
        // so it cannot leave an instance's points untouched
        if (sort_points && ops[i] == 0 && offsets[i + 1] > offsets[i])
            return fail(OT_ERR_INVALID, "point sorting cannot skip an instance (ops = 0 with points)");
        if (ops[i] == 0 || offsets[i + 1] == offsets[i]) continue;
        ops_union |= ops[i];
        if (ops_all >= 0 && ops_all != ops[i] && sort_points)
            return fail(OT_ERR_INVALID, "point sorting needs the same ops for every instance");
        ops_all = ops[i];
        if (sort_points) continue;
        for (int64_t a = offsets[i]; a < offsets[i + 1]; a += tile) {
            const int64_t c = std::min<int64_t>(tile, offsets[i + 1] - a);
            starts.push_back(a);
            infos.push_back((uint32_t)c | ((uint32_t)ops[i] << 24));
        }
    }
    if (ops_all < 0) ops_all = 0;
    if (sort_points) {
        // one run of tiles over the sorted points; ids were written by the sort-key pass
        const int sops = ops_all & ~kOpLocate;
        const int64_t n = offsets[n_inst];
        if (sops)
            for (int64_t a = 0; a < n; a += tile) {
                starts.push_back(a);
                infos.push_back((uint32_t)std::min<int64_t>(tile, n - a) | ((uint32_t)sops << 24));
            }
    }
    ot_batch_plan *p = new ot_batch_plan();
    p->tree = tree;
    p->dtype = dtype;
    p->mode = mode;
    p->block = block;
    p->tile = tile;
    p->ops_union = ops_union;
    p->n_points = offsets[n_inst];
    p->n_tiles = (int64_t)starts.size();
    p->have_graph = false;
    p->use_graph = tuning && (tuning->flags & OT_TUNE_GRAPH);
    p->sort_points = sort_points;
    p->ops_all = ops_all;
    p->grad_plan = (ops_union & kOpGrad) != 0;
    if (sort_points && p->n_points > 0) {
        const int64_t n = p->n_points;
        point_sort_key_bits(tree->n_leaves, p->sort_shift, p->sort_bits);
        const size_t rec = ((ops_all & (kOpSpread | kOpGrad)) ? 6 : 3) * (size_t)n * (dtype == OT_F32 ? 4 : 8);
        hipError_t e = hipSuccess;
        for (int i = 0; i < 2 && e == hipSuccess; ++i) {
            e = hipMalloc((void **)&p->skv[i], 8 * (size_t)n);
            if (e == hipSuccess) e = hipMalloc(&p->srec[i], rec);
        }
        if (e == hipSuccess) e = hipMalloc(&p->sws, (size_t)point_sort_ws_bytes(n));

        if (e != hipSuccess) {
            (void)hipGetLastError();
            ot_batch_plan_destroy(p);
            return fail(OT_ERR_OOM, "ot_batch_plan_create: sort buffers");
        }
    }
    // sorted forward plans that interpolate or spread may take the host-major pass
    p->use_hm = sort_points && !p->grad_plan && (ops_all & (kOpInterp | kOpSpread)) != 0 &&
                tuning && (tuning->flags & OT_TUNE_HOST_MAJOR) && p->n_points > 0;
    if (p->use_hm) {
        p->n_win = (p->n_points + kHmWindow - 1) / kHmWindow;
        if (hipMalloc((void **)&p->fb_list, (size_t)p->n_win * 4) != hipSuccess) {
            (void)hipGetLastError();
            p->fb_list = nullptr;
            ot_batch_plan_destroy(p);
            return fail(OT_ERR_OOM, "ot_batch_plan_create: window list");
        }
    }
    if (mode == OT_SPREAD_FIXED && (ops_union & kOpSpread)) {
        if (hipMalloc(&p->fxws, (size_t)spread_ws_bytes(tree->n_leaves)) != hipSuccess) {
            (void)hipGetLastError();
            p->fxws = nullptr;
            ot_batch_plan_destroy(p);
            return fail(OT_ERR_OOM, "ot_batch_plan_create: fixed-point workspace");
        }
    }
    int cus = 0, dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int per_cu = 0;
    p->small_table = tile <= kSmallTile;
    const void *kfn = dtype == OT_F32
                          ? (mode == OT_SPREAD_FIXED ? kbatch_fn<float, kModeFixed>(p->grad_plan, p->small_table)
                                                     : kbatch_fn<float, kModeAtomic>(p->grad_plan, p->small_table))
                          : (mode == OT_SPREAD_FIXED ? kbatch_fn<double, kModeFixed>(p->grad_plan, p->small_table)
                                                     : kbatch_fn<double, kModeAtomic>(p->grad_plan, p->small_table));
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, block, 0);
    if (per_cu <= 0) per_cu = 1;
    int grid = tuning && tuning->grid ? tuning->grid : std::max(1, cus) * per_cu;
    if (p->n_tiles > 0 && grid > p->n_tiles) grid = (int)p->n_tiles;
    p->grid = std::max(1, grid);
    if (p->use_hm) {
        const int hops = ops_all & (kOpInterp | kOpSpread);
        const void *hfn = dtype == OT_F32 ? (mode == OT_SPREAD_FIXED ? hm_fn<float, kModeFixed>(hops)
                                                                     : hm_fn<float, kModeAtomic>(hops))
                                          : (mode == OT_SPREAD_FIXED ? hm_fn<double, kModeFixed>(hops)
                                                                     : hm_fn<double, kModeAtomic>(hops));
        int hper = 0;
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&hper, hfn, kHmWindow, 0);
        if (hper <= 0) hper = 1;
        int hg = tuning && tuning->grid ? tuning->grid : std::max(1, cus) * hper;
        p->hm_grid = (int)std::max<int64_t>(1, std::min<int64_t>(hg, p->n_win));
    }
    hipError_t e1 = hipMalloc((void **)&p->tile_start, std::max<size_t>(8, starts.size() * 8));
    hipError_t e2 = hipMalloc((void **)&p->tile_info, std::max<size_t>(4, infos.size() * 4));
    hipError_t e3 = hipMalloc((void **)&p->counter, 64);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
        (void)hipGetLastError();
        ot_batch_plan_destroy(p);
        return fail(OT_ERR_OOM, "ot_batch_plan_create: device allocation failed");
    }
    if (!starts.empty()) {
        hipError_t e = hipMemcpy(p->tile_start, starts.data(), starts.size() * 8, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(p->tile_info, infos.data(), infos.size() * 4, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            ot_batch_plan_destroy(p);
            return hip_fail(e, "ot_batch_plan_create: upload");
        }
    }
    hipError_t e = hipStreamCreateWithFlags(&p->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        p->capture_stream = nullptr;
        ot_batch_plan_destroy(p);
        return hip_fail(e, "ot_batch_plan_create: stream");
    }
    *out = p;
    return OT_OK;
}

namespace ot {
namespace {

int run_plan(ot_batch_plan *p, const void *field, const void *force, const void *pos, int32_t *ids, void *vel,
             void *field_out, void *grad, void *stream)
{
    const int u = p->ops_union;
    if (p->n_points > 0 && !pos) return fail(OT_ERR_INVALID, "pos is NULL");
    if ((u & kOpLocate) && !ids) return fail(OT_ERR_INVALID, "ids is NULL");
    if ((u & kOpInterp) && (!field || !vel)) return fail(OT_ERR_INVALID, "field or vel is NULL");
    if ((u & kOpSpread) && (!force || !field_out)) return fail(OT_ERR_INVALID, "force or field_out is NULL");
    if ((u & kOpGrad) && (!field || !force || !grad)) return fail(OT_ERR_INVALID, "field, force or grad is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (p->timing || !p->use_graph) {
        // Plans enqueue their kernels on the caller's stream unless they were
        // made with OT_TUNE_GRAPH; events recorded inside a captured graph
        // cannot be timed, so a timed run does the same.
        return enqueue_any(p, field, force, pos, ids, vel, field_out, grad, s);
    }
    const void *key[7] = {field, force, pos, ids, vel, field_out, grad};
    if (!p->have_graph || std::memcmp(key, p->key, sizeof(key)) != 0) {
        drop_graph(p);
        OT_HIP(hipStreamBeginCapture(p->capture_stream, hipStreamCaptureModeThreadLocal));
        int rc = enqueue_any(p, field, force, pos, ids, vel, field_out, grad, p->capture_stream);
        hipGraph_t g = nullptr;
        hipError_t ec = hipStreamEndCapture(p->capture_stream, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (ec != hipSuccess) return hip_fail(ec, "hipStreamEndCapture");
        hipGraphExec_t ex = nullptr;
        hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            (void)hipGraphDestroy(g);
            return hip_fail(ei, "hipGraphInstantiate");
        }
        p->graph = g;
        p->exec = ex;
        p->have_graph = true;
        std::memcpy(p->key, key, sizeof(key));
    }
    OT_HIP(hipGraphLaunch(p->exec, s));
    return OT_OK;
}

}  // namespace
}  // namespace ot

extern "C" int ot_batch_run(ot_batch_plan *p, const void *field, const void *force, const void *pos, int32_t *ids,
                            void *vel, void *field_out, void *stream)
{
    if (!p) return fail(OT_ERR_INVALID, "plan is NULL");
    if (p->grad_plan) return fail(OT_ERR_INVALID, "plan has gradient ops: run it with ot_batch_run_grad");
    return run_plan(p, field, force, pos, ids, vel, field_out, nullptr, stream);
}

extern "C" int ot_batch_run_grad(ot_batch_plan *p, const void *field, const void *force, const void *pos,
                                 int32_t *ids, void *vel, void *field_out, void *grad, void *stream)
{
    if (!p) return fail(OT_ERR_INVALID, "plan is NULL");
    if (!p->grad_plan) return fail(OT_ERR_INVALID, "plan has no gradient ops: run it with ot_batch_run");
    return run_plan(p, field, force, pos, ids, vel, field_out, grad, stream);
}

extern "C" int ot_batch_plan_shape(const ot_batch_plan *p, int64_t *n_tiles, int32_t *grid)
{
    if (!p) return fail(OT_ERR_INVALID, "plan is NULL");
    if (n_tiles) *n_tiles = p->n_tiles;
    if (grid) *grid = p->grid;
    return OT_OK;
}

extern "C" int ot_batch_plan_timing(ot_batch_plan *p, int32_t enable)
{
    if (!p) return fail(OT_ERR_INVALID, "plan is NULL");
    const bool on = enable != 0;
    if (on == p->timing) return OT_OK;
    if (on && !p->ev[0]) {
        OT_HIP(hipEventCreate(&p->ev[0]));
        OT_HIP(hipEventCreate(&p->ev[1]));
    }
    p->timing = on;
    return OT_OK;
}

extern "C" int ot_batch_last_kernel_ms(const ot_batch_plan *p, float *ms)
{
    if (!p || !ms) return fail(OT_ERR_INVALID, "NULL argument");
    if (!p->timing) return fail(OT_ERR_INVALID, "timing is off for this plan");
    OT_HIP(hipEventElapsedTime(ms, p->ev[0], p->ev[1]));
    return OT_OK;
}

extern "C" int ot_batch_plan_windows(const ot_batch_plan *p, int64_t *n_windows, int64_t *handed_over)
{
    if (!p) return fail(OT_ERR_INVALID, "plan is NULL");
    const int64_t nw = p->use_hm ? p->n_win : 0;
    if (n_windows) *n_windows = nw;
    if (handed_over) {
        *handed_over = 0;
        if (nw > 0) {
            unsigned c = 0;
            OT_HIP(hipMemcpy(&c, p->counter + 2, sizeof(c), hipMemcpyDeviceToHost));
            *handed_over = c;
        }
    }
    return OT_OK;
}

extern "C" int ot_batch_plan_destroy(ot_batch_plan *p)
{
    if (!p) return OT_OK;
    (void)hipDeviceSynchronize();
    drop_graph(p);
    if (p->ev[0]) (void)hipEventDestroy(p->ev[0]);
    if (p->ev[1]) (void)hipEventDestroy(p->ev[1]);
    for (void *q : {(void *)p->skv[0], (void *)p->skv[1], p->srec[0], p->srec[1], p->sws, p->fxws, (void *)p->fb_list})
        if (q) (void)hipFree(q);
    if (p->tile_start) (void)hipFree(p->tile_start);
    if (p->tile_info) (void)hipFree(p->tile_info);
    if (p->counter) (void)hipFree(p->counter);
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    delete p;
    return OT_OK;
}
