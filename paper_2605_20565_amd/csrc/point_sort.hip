// Sorting the points of a batched run by host leaf, carrying their
// positions, forces and original indices with them.
//
// Neighbouring threads of the tracking pass then work on neighbouring host
// cells: their stencil nodes share cache lines and the workgroup's spreading
// table, and positions and forces are read with coalesced loads.  The key of a
// point is its host leaf id; the passes order by bits [shift, shift + bits)
// only (groups of 2^shift consecutive leaves, at most two 8-bit LSD passes),
// and the tracking pass finishes the order inside each tile.  Each pass stages a
// tile of 2048 keys in LDS with coalesced loads, ranks them stably by the
// digit with eight 1-bit splits, and writes every digit's run contiguously;
// the payload of a key is gathered from inside the tile and written once.
#include <hip/hip_runtime.h>

#include "ot_common.h"
#include "point_sort.h"

namespace ot {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;
constexpr int kBits = 8;
constexpr int kBuckets = 1 << kBits;

__device__ __forceinline__ uint32_t exscan_256(uint32_t v, uint32_t *sh_w, uint32_t &total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh_w[wid] = x;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        const uint32_t s = sh_w[w];
        if (w < wid) pre += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return pre + x - v;
}

// Host-leaf keys (and ids when asked) of all points.
template <typename T>
__global__ __launch_bounds__(256) void k_point_keys(TreeView tv, int64_t n, const T *__restrict__ pos,
                                                    int32_t *__restrict__ ids, uint32_t *__restrict__ keys,
                                                    uint32_t none)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    uint32_t I[3];
    const bool ok = point_cell<T>(tv, pos[3 * k], pos[3 * k + 1], pos[3 * k + 2], I);
    const uint32_t host = ok ? (descend(tv, I[0], I[1], I[2]) & kIdMask) : none;
    if (ids) ids[k] = ok ? (int32_t)host : -1;
    keys[k] = host;
}

__global__ __launch_bounds__(kThreads) void k_point_hist(const uint32_t *__restrict__ keys, int64_t n, int shift,
                                                         uint32_t *__restrict__ counts, int nblocks)
{
    __shared__ uint32_t hist[kBuckets];
    for (int i = threadIdx.x; i < kBuckets; i += kThreads) hist[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int j = threadIdx.x; j < kTile; j += kThreads) {
        const int64_t i = base + j;
        if (i < n) atomicAdd(&hist[(keys[i] >> shift) & (kBuckets - 1)], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kBuckets; d += kThreads) counts[(int64_t)d * nblocks + blockIdx.x] = hist[d];
}

// One stable counting pass.  vin == nullptr: the values are the input
// indices themselves (first pass).  fin may be null (no forces carried).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_point_scatter(
    const uint32_t *__restrict__ kin, const int32_t *__restrict__ vin, const T *__restrict__ pin,
    const T *__restrict__ fin, uint32_t *__restrict__ kout, int32_t *__restrict__ vout, T *__restrict__ pout,
    T *__restrict__ fout, int64_t n, int shift, const uint32_t *__restrict__ offs, int nblocks)
{
    __shared__ uint32_t sk[kTile];
    __shared__ uint16_t si[kTile];
    __shared__ uint32_t sh_w[kThreads / 64];
    __shared__ uint32_t dstart[kBuckets];
    __shared__ uint32_t dcount[kBuckets];

    const int64_t base = (int64_t)blockIdx.x * kTile;
    const int64_t rem = n - base;
    const int valid = rem < kTile ? (int)rem : kTile;
    for (int d = threadIdx.x; d < kBuckets; d += kThreads) dcount[d] = 0;
    // coalesced load of the tile's keys; padding sorts last
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int li = j * kThreads + threadIdx.x;
        sk[li] = li < valid ? kin[base + li] : 0xFFFFFFFFu;
        si[li] = (uint16_t)li;
    }
    __syncthreads();
    uint32_t k[kItems];
    uint32_t x[kItems];
    const int t0 = threadIdx.x * kItems;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        k[j] = sk[t0 + j];
        x[j] = si[t0 + j];
        if (t0 + j < valid) atomicAdd(&dcount[(k[j] >> shift) & (kBuckets - 1)], 1u);
    }
    __syncthreads();
    for (int b = 0; b < kBits; ++b) {
        uint32_t zeros = 0;
#pragma unroll
        for (int j = 0; j < kItems; ++j) zeros += 1u - ((k[j] >> (shift + b)) & 1u);
        uint32_t total_zeros;
        uint32_t zb = exscan_256(zeros, sh_w, total_zeros);
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const uint32_t bit = (k[j] >> (shift + b)) & 1u;
            const uint32_t g = (uint32_t)(t0 + j);
            const uint32_t p = bit ? total_zeros + (g - zb) : zb;
            zb += 1u - bit;
            sk[p] = k[j];
            si[p] = (uint16_t)x[j];
        }
        __syncthreads();
        if (b + 1 < kBits) {
#pragma unroll
            for (int j = 0; j < kItems; ++j) {
                k[j] = sk[t0 + j];
                x[j] = si[t0 + j];
            }
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int d = 0; d < kBuckets; ++d) {
            dstart[d] = acc;
            acc += dcount[d];
        }
    }
    __syncthreads();
    // coalesced write: sorted position i -> its digit's run; payload gathered from the tile
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int i = j * kThreads + threadIdx.x;
        if (i < valid) {
            const uint32_t key = sk[i];
            const int64_t src = base + si[i];
            const uint32_t d = (key >> shift) & (kBuckets - 1);
            const int64_t dst = (int64_t)offs[(int64_t)d * nblocks + blockIdx.x] + (i - (int)dstart[d]);
            kout[dst] = key;
            vout[dst] = vin ? vin[src] : (int32_t)src;
            pout[3 * dst] = pin[3 * src];
            pout[3 * dst + 1] = pin[3 * src + 1];
            pout[3 * dst + 2] = pin[3 * src + 2];
            if (fin) {
                fout[3 * dst] = fin[3 * src];
                fout[3 * dst + 1] = fin[3 * src + 1];
                fout[3 * dst + 2] = fin[3 * src + 2];
            }
        }
    }
}

}  // namespace

int64_t point_sort_ws_bytes(int64_t n)
{
    const int64_t nb = (n + kTile - 1) / kTile;
    const int64_t nc = (int64_t)kBuckets * nb;
    return 4 * (2 * nc + scan_tmp_words(nc)) + 256;
}

template <typename T>
void point_sort(const TreeView &tv, int64_t n, int64_t n_leaves, int shift, int bits, const T *pos, const T *force,
                int32_t *ids, PointSortBufs<T> &b, hipStream_t s, PointSortResult<T> &out)
{
    const unsigned gb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_point_keys<T>, dim3(gb), dim3(256), 0, s, tv, n, pos, ids, b.key[0], (uint32_t)n_leaves);
    const int nb = (int)((n + kTile - 1) / kTile);
    const int64_t nc = (int64_t)kBuckets * nb;
    uint32_t *counts = (uint32_t *)b.ws, *offs = counts + nc, *tmp = offs + nc;
    const uint32_t *kin = b.key[0];
    const int32_t *vin = nullptr;
    const T *pin = pos, *fin = force;
    int cur = 0;
    for (int sh = 0; sh < bits; sh += kBits) {
        const int o = cur ^ 1;   // write buffer: 1, 0, 1, ...
        hipLaunchKernelGGL(k_point_hist, dim3(nb), dim3(kThreads), 0, s, kin, n, shift + sh, counts, nb);
        exclusive_scan(counts, offs, nc, tmp, s);
        hipLaunchKernelGGL(k_point_scatter<T>, dim3(nb), dim3(kThreads), 0, s, kin, vin, pin, fin, b.key[o], b.val[o],
                           b.pos[o], force ? b.force[o] : (T *)nullptr, n, shift + sh, (const uint32_t *)offs, nb);
        kin = b.key[o];
        vin = b.val[o];
        pin = b.pos[o];
        fin = force ? b.force[o] : nullptr;
        cur = o;
    }
    out.host = kin;
    out.perm = vin;
    out.pos = pin;
    out.force = fin;
}

template void point_sort<float>(const TreeView &, int64_t, int64_t, int, int, const float *, const float *, int32_t *,
                                PointSortBufs<float> &, hipStream_t, PointSortResult<float> &);
template void point_sort<double>(const TreeView &, int64_t, int64_t, int, int, const double *, const double *,
                                 int32_t *, PointSortBufs<double> &, hipStream_t, PointSortResult<double> &);

}  // namespace ot
