// Sorting the points of a batched run by host leaf, carrying their
// positions and forces with them.
//
// Neighbouring threads of the tracking pass then work on neighbouring host
// cells: their stencil nodes share cache lines and the workgroup's spreading
// table, and positions and forces are read with coalesced loads.  Each point
// is one 64-bit word (host's leaf entry) << 32 | input index plus one record of R values
// (position, then force when spreading).  The passes order by key bits
// [shift, shift + bits) only (groups of 2^shift consecutive leaves; 8-bit
// LSD passes, see point_sort_key_bits).
//
// A pass takes tiles of 2048 points: the keys are staged in LDS with
// coalesced loads, ranked by the digit (stably, with eight 1-bit splits,
// except in the first pass, whose order no later pass relies on: there each
// key takes the next slot of its digit from an LDS counter), and every
// digit's run is written contiguously; the records, read once in
// input order, move to their sorted slots through LDS in small chunks.  (Tiles of 4096 and 8192
// points give longer runs but fewer workgroups in flight, and were slower.)  The
// first pass's digit counts come from the key kernel, and the first pass also
// takes max |F| for the fixed-point scale, since it reads every force anyway.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "ot_common.h"
#include "point_sort.h"

namespace ot {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;   // 2048
constexpr int kBits = 8;
constexpr int kBuckets = 1 << kBits;
static_assert(kThreads == kBuckets, "one digit per thread in the digit scan");

// CW consecutive record values as one LDS word of the staging buffer.
template <typename T, int CW>
struct Chunk2;
template <>
struct Chunk2<float, 2> {
    using type = float2;
    static __device__ __forceinline__ float2 pack(const float *v, int c) { return make_float2(v[c], v[c + 1]); }
};
template <>
struct Chunk2<double, 2> {
    using type = double2;
    static __device__ __forceinline__ double2 pack(const double *v, int c) { return make_double2(v[c], v[c + 1]); }
};
template <typename T>
struct Chunk2<T, 1> {
    using type = T;
    static __device__ __forceinline__ T pack(const T *v, int c) { return v[c]; }
};

// Four floats at a 4-byte aligned address (one 16-byte store).
struct __attribute__((aligned(4))) F4u {
    float x, y, z, w;
};

// Tile of workgroup blockIdx.x.  Workgroups go round-robin over the 8 XCDs;
// each XCD takes a contiguous range of tiles, so that what neighbouring
// tiles write next to each other (the digit counts of one digit, the ends of
// one digit's runs) meets in the same L2 instead of in partial lines of up
// to eight.
__device__ __forceinline__ int xcd_tile(int nblocks)
{
    const int xg = (int)(blockIdx.x & 7u), xk = (int)(blockIdx.x >> 3), xq = nblocks >> 3, xr = nblocks & 7;
    return xg * xq + (xg < xr ? xg : xr) + xk;
}

// LDS index with one pad word per 32: the blocked reads (stride kItems) and
// the striped writes both spread over the banks.
__device__ __forceinline__ int pad(int i) { return i + (i >> 5); }
constexpr int kPadded = kTile + kTile / 32;

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

__device__ __forceinline__ unsigned long long abs_bits_of(float v)
{
    return (unsigned long long)(__float_as_uint(v) & 0x7FFFFFFFu);
}
__device__ __forceinline__ unsigned long long abs_bits_of(double v)
{
    return (unsigned long long)__double_as_longlong(v) & 0x7FFFFFFFFFFFFFFFull;
}

// Block-wide max, one atomic per workgroup (same-address atomics serialise).
__device__ __forceinline__ void block_max_to(unsigned long long v, unsigned long long *sh, unsigned long long *out)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = std::max(v, (unsigned long long)__shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kThreads / 64; ++w) v = std::max(v, sh[w]);
        if (v) atomicMax(out, v);
    }
}

// Host leaf of every point (and ids when asked): kv = entry << 32 | index
// with the host's leaf entry (level << 26 | id); points without a host get
// n_leaves.  Digits are taken from the id bits only.  Workgroup b covers the first
// pass's tile b and leaves its digit counts in counts[d * nblocks + b].
// A thread's kItems points go through the descent together: all positions,
// then all root-table loads, then the deeper levels, so that the table loads
// (the pass's latency) are in flight at once rather than one after another.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_point_keys(TreeView tv, int64_t n, const T *__restrict__ pos,
                                                         int32_t *__restrict__ ids, uint64_t *__restrict__ kv,
                                                         uint32_t none, int shift, uint32_t *__restrict__ counts,
                                                         int nblocks)
{
    __shared__ uint32_t hist[kBuckets];
    for (int i = threadIdx.x; i < kBuckets; i += kThreads) hist[i] = 0;
    __syncthreads();
    const int tile = xcd_tile(nblocks);
    const int64_t base = (int64_t)tile * kTile;
    uint32_t I[kItems][3];
    uint32_t e[kItems];
    bool ok[kItems];
    // loads at clamped indices, so that no item's load sits behind a branch
    // (a load inside a branch is waited for at the branch's end)
    T X[kItems][3];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int64_t k = base + j * kThreads + threadIdx.x;
        const int64_t kc = k < n ? k : n - 1;
#pragma unroll
        for (int d = 0; d < 3; ++d) X[j][d] = pos[3 * kc + d];
    }
    const int sh = tv.L - tv.lev[0];
    // root summary first (small enough for L2); the root itself only where
    // the summary has no answer (other lanes load entry 0)
    uint32_t root[kItems], sm[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int64_t k = base + j * kThreads + threadIdx.x;
        ok[j] = point_cell<T>(tv, X[j][0], X[j][1], X[j][2], I[j]) && k < n;
        root[j] = ok[j] ? interleave3(I[j][0] >> sh, I[j][1] >> sh, I[j][2] >> sh) : 0u;
        sm[j] = tv.summary ? ld_summary(tv, root[j] >> 3) : kSplit;
    }
#pragma unroll
    for (int j = 0; j < kItems; ++j) e[j] = ld_table(tv, (sm[j] & kSplit) ? root[j] : 0u);
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        if (!(sm[j] & kSplit)) e[j] = sm[j] + (root[j] & 7u);
        if (!ok[j]) e[j] = none;
    }
    // the level-1 step of every split entry at once, then deeper levels (rare)
    uint32_t e1[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) e1[j] = ld_table(tv, step1_index(tv, e[j], I[j][0], I[j][1], I[j][2]));
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        if (e[j] & kSplit) e[j] = e1[j];
        if (e[j] & kSplit) e[j] = descend_from_level2(tv, e[j], I[j][0], I[j][1], I[j][2]);
    }
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int64_t k = base + j * kThreads + threadIdx.x;
        if (k < n) {
            // the host's whole leaf entry (level << 26 | id): the tracking pass
            // takes it from here instead of searching again
            if (ids) ids[k] = ok[j] ? (int32_t)(e[j] & kIdMask) : -1;
            kv[k] = ((uint64_t)e[j] << 32) | (uint32_t)k;
            atomicAdd(&hist[((e[j] & kIdMask) >> shift) & (kBuckets - 1)], 1u);
        }
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kBuckets; d += kThreads) counts[(int64_t)d * nblocks + tile] = hist[d];
}

__global__ __launch_bounds__(kThreads) void k_point_hist(const uint64_t *__restrict__ kv, int64_t n, int shift,
                                                         uint32_t *__restrict__ counts, int nblocks)
{
    __shared__ uint32_t hist[kBuckets];
    for (int i = threadIdx.x; i < kBuckets; i += kThreads) hist[i] = 0;
    __syncthreads();
    const int tile = xcd_tile(nblocks);
    const int64_t base = (int64_t)tile * kTile;
    // all of a thread's words loaded (clamped indices) before any is counted
    uint32_t hk[kItems];
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int64_t i = base + j * kThreads + threadIdx.x;
        hk[j] = (uint32_t)(kv[i < n ? i : base] >> 32);
    }
#pragma unroll
    for (int j = 0; j < kItems; ++j)
        if (base + j * kThreads + threadIdx.x < n) atomicAdd(&hist[((hk[j] & kIdMask) >> shift) & (kBuckets - 1)], 1u);
    __syncthreads();
    for (int d = threadIdx.x; d < kBuckets; d += kThreads) counts[(int64_t)d * nblocks + tile] = hist[d];
}

// One counting pass over tiles of kTile points, stable except the first
// (first != 0).  Records come from rin (R values per point) or, in the first
// pass, from pos (3 per point) and force (3 per point, R = 6 only).
// maxbits != null: also max |F| over the finite force components.
template <typename T, int R>
__global__ __launch_bounds__(kThreads) void k_point_scatter(
    const uint64_t *__restrict__ kin, const T *__restrict__ rin, const T *__restrict__ pos,
    const T *__restrict__ force, uint64_t *__restrict__ kout, T *__restrict__ rout, int64_t n, int shift,
    const uint32_t *__restrict__ offs, const uint32_t *__restrict__ offs_hi, int nblocks,
    unsigned long long *__restrict__ maxbits, int first)
{
    __shared__ uint32_t sk[kPadded];
    __shared__ uint16_t si[kPadded];
    __shared__ uint32_t sh_w[kThreads / 64];
    __shared__ uint32_t dstart[kBuckets];
    __shared__ uint32_t dcount[kBuckets];
    __shared__ uint32_t dcur[kBuckets];
    __shared__ unsigned long long sh_max[kThreads / 64];

    const int tile = xcd_tile(nblocks);
    const int64_t base = (int64_t)tile * kTile;
    const int64_t rem = n - base;
    const int valid = rem < kTile ? (int)rem : kTile;
    // The tile's words and records, read once in input order (coalesced) and
    // before the ranking, so that their latency overlaps it.
    // Every item loads at a clamped index (the tile's first point stands in
    // for the padding), with no branch around the loads: a load inside a
    // branch is waited for where the branch joins, which had put the eight
    // items' round trips one after another.
    T rv[kItems][R];
    uint32_t lo[kItems], kk[kItems];
    uint64_t wv[kItems];
    if (rin) {
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const int li = j * kThreads + threadIdx.x;
            const int64_t src = base + (li < valid ? li : 0);
            wv[j] = kin[src];
#pragma unroll
            for (int c = 0; c < R; ++c) rv[j][c] = rin[R * src + c];
        }
    } else {
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const int li = j * kThreads + threadIdx.x;
            const int64_t src = base + (li < valid ? li : 0);
            wv[j] = kin[src];
#pragma unroll
            for (int c = 0; c < 3; ++c) rv[j][c] = pos[3 * src + c];
#pragma unroll
            for (int c = 3; c < R; ++c) rv[j][c] = force[3 * src + (c - 3)];
        }
    }
    unsigned long long mx = 0;
    bool bad = false;
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const bool in = j * kThreads + (int)threadIdx.x < valid;
        kk[j] = in ? (uint32_t)(wv[j] >> 32) : 0xFFFFFFFFu;   // padding sorts last
        lo[j] = in ? (uint32_t)wv[j] : 0u;
        if (maxbits && in) {
#pragma unroll
            for (int c = 3; c < R; ++c) {
                if (isfinite(rv[j][c])) mx = std::max(mx, abs_bits_of(rv[j][c]));
                else bad = true;
            }
        }
    }
    for (int d = threadIdx.x; d < kBuckets; d += kThreads) {
        dcount[d] = 0;
        dcur[d] = 0;
    }
    __syncthreads();
    for (int j = 0; j < kItems; ++j) {
        const int li = j * kThreads + threadIdx.x;
        const uint32_t key = kk[j];
        if (li < valid) atomicAdd(&dcount[((key & kIdMask) >> shift) & (kBuckets - 1)], 1u);
        sk[pad(li)] = key;
        si[pad(li)] = (uint16_t)li;
    }
    __syncthreads();
    {
        uint32_t tot;
        const uint32_t c = dcount[threadIdx.x];
        dstart[threadIdx.x] = exscan_256(c, sh_w, tot);
    }
    __syncthreads();
    if (first) {
        // The first pass need not be stable (the later, stable passes keep
        // its order only inside groups of equal key, where any order will
        // do): each item takes the next slot of its digit's run from an LDS
        // counter, instead of eight one-bit split rounds.
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const int li = j * kThreads + threadIdx.x;
            if (li < valid) {
                const uint32_t d = ((kk[j] & kIdMask) >> shift) & (kBuckets - 1);
                const uint32_t p = dstart[d] + atomicAdd(&dcur[d], 1u);
                sk[pad((int)p)] = kk[j];
                si[pad((int)p)] = (uint16_t)li;
            }
        }
        __syncthreads();
    } else {
        // stable: eight one-bit splits, each a block-wide scan of the zeros
        uint32_t k[kItems];
        uint32_t x[kItems];
        const int t0 = threadIdx.x * kItems;
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            k[j] = sk[pad(t0 + j)];
            x[j] = si[pad(t0 + j)];
        }
        __syncthreads();
        for (int b = 0; b < kBits; ++b) {
            uint32_t zeros = 0;
#pragma unroll
            for (int j = 0; j < kItems; ++j) zeros += 1u - (((k[j] & kIdMask) >> (shift + b)) & 1u);
            uint32_t total_zeros;
            uint32_t zb = exscan_256(zeros, sh_w, total_zeros);
#pragma unroll
            for (int j = 0; j < kItems; ++j) {
                const uint32_t bit = ((k[j] & kIdMask) >> (shift + b)) & 1u;
                const uint32_t g = (uint32_t)(t0 + j);
                const uint32_t p = bit ? total_zeros + (g - zb) : zb;
                zb += 1u - bit;
                sk[pad((int)p)] = k[j];
                si[pad((int)p)] = (uint16_t)x[j];
            }
            __syncthreads();
            if (b + 1 < kBits) {
#pragma unroll
                for (int j = 0; j < kItems; ++j) {
                    k[j] = sk[pad(t0 + j)];
                    x[j] = si[pad(t0 + j)];
                }
                __syncthreads();
            }
        }
    }
    // Records are read once, in input order (coalesced), into registers and
    // reach their sorted positions through LDS in chunks of CW values (the
    // whole tile's records at once would take too much LDS: fewer
    // workgroups in flight); words and records are then written in sorted
    // order, contiguously within each digit's run.  (Gathering each record
    // from global memory instead, at its source inside the tile, fetched
    // about 4x its bytes past L2 and took 319 against 232 us per pass on
    // 10^7 points.)
    // FP32 records of 6 values move as one 16-byte and one 8-byte chunk;
    // otherwise in chunks of CW values
    constexpr bool kF6 = std::is_same<T, float>::value && R == 6;
    constexpr int CW = (R % 2 == 0) ? 2 : 1;
    constexpr int kChunks = kF6 ? 2 : R / CW;
    using Chunk = typename std::conditional<kF6, float4, typename Chunk2<T, CW>::type>::type;
    __shared__ Chunk stg[kPadded];
    // the words' low halves (input indices) travel in the second FP32 chunk
    __shared__ uint32_t slo[kF6 ? 1 : kPadded];
    // sorted position i = j * kThreads + thread: its destination and source slot
    int64_t dstv[kItems];
    int srcv[kItems];
    // (no branch around the offset loads either: the padding's keys, sorted
    // last, also name a digit, so their loads stay in bounds)
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
        const int i = j * kThreads + threadIdx.x;
        const uint32_t key = sk[pad(i)];
        const uint32_t d = ((key & kIdMask) >> shift) & (kBuckets - 1);
        const int64_t oi = (int64_t)d * nblocks + tile;
        const int64_t o = (int64_t)offs[oi] + (offs_hi ? (int64_t)offs_hi[oi / kScanBlock] : 0);
        dstv[j] = i < valid ? o + (i - (int)dstart[d]) : -1;
        srcv[j] = i < valid ? (int)si[pad(i)] : 0;
    }
#pragma unroll
    for (int ch = 0; ch < kChunks; ++ch) {
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            const int li = j * kThreads + threadIdx.x;
            if constexpr (kF6) {
                const float *v = reinterpret_cast<const float *>(rv[j]);
                stg[pad(li)] = ch == 0 ? make_float4(v[0], v[1], v[2], v[3])
                                       : make_float4(v[4], v[5], __uint_as_float(lo[j]), 0.f);
            } else {
                stg[pad(li)] = Chunk2<T, CW>::pack(rv[j], CW * ch);
                if (ch == 0) slo[pad(li)] = lo[j];
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kItems; ++j) {
            // LDS reads outside the branch, stores inside it
            const int i = j * kThreads + threadIdx.x;
            const Chunk c = stg[pad(srcv[j])];
            const uint32_t key = sk[pad(i)];
            if constexpr (kF6) {
                if (dstv[j] < 0) continue;
                // a record starts at 24 dst bytes: 8-byte aligned
                float *dst = reinterpret_cast<float *>(rout) + 6 * dstv[j];
                if (ch == 0) {
                    *reinterpret_cast<F4u *>(dst) = F4u{c.x, c.y, c.z, c.w};
                } else {
                    *reinterpret_cast<float2 *>(dst + 4) = make_float2(c.x, c.y);
                    kout[dstv[j]] = ((uint64_t)key << 32) | __float_as_uint(c.z);
                }
            } else {
                const uint32_t lw = ch == 0 ? slo[pad(srcv[j])] : 0u;
                if (dstv[j] < 0) continue;
                if (ch == 0) kout[dstv[j]] = ((uint64_t)key << 32) | lw;
                reinterpret_cast<Chunk *>(rout)[(R * dstv[j]) / CW + ch] = c;
            }
        }
        __syncthreads();
    }
    if (maxbits) {
        if (bad) atomicOr(maxbits + 1, 1ull);   // the non-finite flag next to max |F|
        block_max_to(mx, sh_max, maxbits);
    }
}

template <typename T, int R>
void sort_passes(const TreeView &tv, int64_t n, int64_t n_leaves, int shift, int bits, const T *pos, const T *force,
                 int32_t *ids, PointSortBufs<T> &b, unsigned long long *maxbits, hipStream_t s,
                 PointSortResult<T> &out)
{
    const int nb = (int)((n + kTile - 1) / kTile);
    const int64_t nc = (int64_t)kBuckets * nb;
    uint32_t *counts = (uint32_t *)b.ws, *offs = counts + nc, *tmp = offs + nc;
    hipLaunchKernelGGL(k_point_keys<T>, dim3(nb), dim3(kThreads), 0, s, tv, n, pos, ids, b.kv[0],
                       (uint32_t)n_leaves, shift, counts, nb);
    const uint64_t *kin = b.kv[0];
    const T *rin = nullptr;
    int cur = 0;
    for (int sh = 0; sh < bits; sh += kBits) {
        const int o = cur ^ 1;   // write buffer: 1, 0, 1, ...
        if (sh > 0) hipLaunchKernelGGL(k_point_hist, dim3(nb), dim3(kThreads), 0, s, kin, n, shift + sh, counts, nb);
        // the digit offsets: each 2048-count block's own scan, plus the
        // blocks' scanned sums, which the scatter adds (one launch less)
        const uint32_t *offs_hi = exclusive_scan_split(counts, offs, nc, tmp, s);
        hipLaunchKernelGGL((k_point_scatter<T, R>), dim3(nb), dim3(kThreads), 0, s, kin, rin, pos, force, b.kv[o],
                           b.rec[o], n, shift + sh, (const uint32_t *)offs, offs_hi, nb,
                           sh == 0 ? maxbits : (unsigned long long *)nullptr, sh == 0 ? 1 : 0);
        kin = b.kv[o];
        rin = b.rec[o];
        cur = o;
    }
    out.kv = kin;
    out.rec = rin;
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
                int32_t *ids, PointSortBufs<T> &b, unsigned long long *maxbits, hipStream_t s,
                PointSortResult<T> &out)
{
    if (force) sort_passes<T, 6>(tv, n, n_leaves, shift, bits, pos, force, ids, b, maxbits, s, out);
    else sort_passes<T, 3>(tv, n, n_leaves, shift, bits, pos, nullptr, ids, b, nullptr, s, out);
    out.stride = force ? 6 : 3;
}

template void point_sort<float>(const TreeView &, int64_t, int64_t, int, int, const float *, const float *, int32_t *,
                                PointSortBufs<float> &, unsigned long long *, hipStream_t, PointSortResult<float> &);
template void point_sort<double>(const TreeView &, int64_t, int64_t, int, int, const double *, const double *,
                                 int32_t *, PointSortBufs<double> &, unsigned long long *, hipStream_t,
                                 PointSortResult<double> &);

}  // namespace ot
