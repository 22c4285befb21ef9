// Tree construction on the GPU: Morton keys of leaf anchors, an LSD radix
// sort of the keys staged in LDS, validation that the sorted leaves tile the
// unit cube, and the descent table used by every lookup.
//
// Sec. 3.1 of the paper keeps the leaves of each tree in an array sorted by
// Morton (Z-order) index; Algorithm 1 binary-searches that array once per
// level.  Here the sorted array is built once per tree and indexed by a radix
// table over groups of three Morton digits, so a lookup is one dependent
// load per three levels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "ot_common.h"

namespace ot {

namespace {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;   // 2048 keys per workgroup
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;

__global__ void k_encode_keys(const uint32_t *__restrict__ a, int64_t n, uint64_t *__restrict__ keys)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    // Anchors at or above 2^21 keep their high bits so that validation sees them.
    uint64_t x = a[3 * i], y = a[3 * i + 1], z = a[3 * i + 2];
    uint64_t k = split3_21(x) | (split3_21(y) << 1) | (split3_21(z) << 2);
    if ((x | y | z) >> 21) k |= 0x8000000000000000ull;
    keys[i] = k;
}

// -- block-wide exclusive scan over 256 threads (4 waves of 64) -------------
__device__ __forceinline__ uint32_t block_exscan_256(uint32_t v, uint32_t *sh_w, uint32_t &total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh_w[wid] = x;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kSortThreads / 64; ++w) {
        uint32_t s = sh_w[w];
        if (w < wid) pre += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return pre + x - v;
}

}  // namespace

// -- device-wide exclusive scan of uint32 (reduce/scan per 2048 + recursion) -
__global__ __launch_bounds__(kSortThreads) void k_scan_tiles(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                             int64_t n, uint32_t *__restrict__ sums)
{
    __shared__ uint32_t sh_w[kSortThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)threadIdx.x * kSortItems;
    uint32_t v[kSortItems], s = 0;
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        v[j] = (base + j < n) ? in[base + j] : 0u;
        s += v[j];
    }
    uint32_t tot;
    uint32_t pre = block_exscan_256(s, sh_w, tot);
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        if (base + j < n) out[base + j] = pre;
        pre += v[j];
    }
    if (threadIdx.x == 0 && sums) sums[blockIdx.x] = tot;
}

__global__ void k_scan_add(uint32_t *__restrict__ out, int64_t n, const uint32_t *__restrict__ offs)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] += offs[i / kSortTile];
}

// Exclusive scan of n uint32 values (n < 2^32 total).  tmp must hold
// scan_tmp_words(n) words.
int64_t scan_tmp_words(int64_t n)
{
    int64_t w = 0;
    while (n > kSortTile) {
        n = (n + kSortTile - 1) / kSortTile;
        w += 2 * n;
    }
    return w + 1;
}

void exclusive_scan(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp, hipStream_t s)
{
    if (n <= 0) return;
    int64_t nb = (n + kSortTile - 1) / kSortTile;
    if (nb == 1) {
        hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kSortThreads), 0, s, in, out, n, (uint32_t *)nullptr);
        return;
    }
    uint32_t *sums = tmp, *sums_scan = tmp + nb;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nb), dim3(kSortThreads), 0, s, in, out, n, sums);
    exclusive_scan(sums, sums_scan, nb, tmp + 2 * nb, s);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n, sums_scan);
}

const uint32_t *exclusive_scan_split(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp, hipStream_t s)
{
    static_assert(kScanBlock == kSortTile, "the split scan's block is the scan tile");
    const int64_t nb = (n + kSortTile - 1) / kSortTile;
    if (nb <= 1 || nb > kSortTile) {
        exclusive_scan(in, out, n, tmp, s);
        return nullptr;
    }
    uint32_t *sums = tmp, *sums_scan = tmp + nb;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nb), dim3(kSortThreads), 0, s, in, out, n, sums);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kSortThreads), 0, s, sums, sums_scan, nb, (uint32_t *)nullptr);
    return sums_scan;
}

// -- LSD radix sort of (uint64 key, int32 value), 8 bits per pass ------------
__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint64_t *__restrict__ keys, int64_t n, int shift,
                                                             uint32_t *__restrict__ counts, int nblocks)
{
    __shared__ uint32_t hist[kRadix];
    for (int i = threadIdx.x; i < kRadix; i += kSortThreads) hist[i] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int j = threadIdx.x; j < kSortTile; j += kSortThreads) {
        int64_t i = base + j;
        if (i < n) atomicAdd(&hist[(keys[i] >> shift) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kRadix; d += kSortThreads)
        counts[(int64_t)d * nblocks + blockIdx.x] = hist[d];
}

// Stable scatter of one tile: the tile is first sorted by the digit in LDS
// with eight stable 1-bit splits, then every key goes to
// offset[digit][tile] + (its rank among the tile's keys with that digit).
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const uint64_t *__restrict__ kin, const int32_t *__restrict__ vin,
                                                                uint64_t *__restrict__ kout, int32_t *__restrict__ vout,
                                                                int64_t n, int shift, const uint32_t *__restrict__ offs,
                                                                int nblocks)
{
    __shared__ uint64_t sk[kSortTile];
    __shared__ int32_t sv[kSortTile];
    __shared__ uint32_t sh_w[kSortThreads / 64];
    __shared__ uint32_t dstart[kRadix];
    __shared__ uint32_t dcount[kRadix];

    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const int64_t rem = n - base;
    const int valid = rem < kSortTile ? (int)rem : kSortTile;
    for (int d = threadIdx.x; d < kRadix; d += kSortThreads) dcount[d] = 0;

    uint64_t k[kSortItems];
    int32_t v[kSortItems];
    const int t0 = threadIdx.x * kSortItems;
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        int li = t0 + j;
        if (li < valid) {
            k[j] = kin[base + li];
            v[j] = vin[base + li];
        } else {
            k[j] = ~0ull;   // padding sorts last (all digit bits set) and stays after real keys
            v[j] = -1;
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSortItems; ++j)
        if (t0 + j < valid) atomicAdd(&dcount[(k[j] >> shift) & (kRadix - 1)], 1u);

    for (int b = 0; b < kRadixBits; ++b) {
        uint32_t zeros = 0;
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) zeros += 1u - (uint32_t)((k[j] >> (shift + b)) & 1u);
        uint32_t total_zeros;
        uint32_t zb = block_exscan_256(zeros, sh_w, total_zeros);
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            uint32_t bit = (uint32_t)((k[j] >> (shift + b)) & 1u);
            uint32_t g = (uint32_t)(t0 + j);
            uint32_t pos = bit ? total_zeros + (g - zb) : zb;
            zb += 1u - bit;
            sk[pos] = k[j];
            sv[pos] = v[j];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kSortItems; ++j) {
            k[j] = sk[t0 + j];
            v[j] = sv[t0 + j];
        }
        __syncthreads();
    }
    // local start of each digit inside the sorted tile
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int d = 0; d < kRadix; ++d) {
            dstart[d] = acc;
            acc += dcount[d];
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        int li = t0 + j;
        if (li < valid) {
            uint32_t d = (uint32_t)((k[j] >> shift) & (kRadix - 1));
            int64_t dst = (int64_t)offs[(int64_t)d * nblocks + blockIdx.x] + (li - (int)dstart[d]);
            kout[dst] = k[j];
            vout[dst] = v[j];
        }
    }
}

namespace {

__global__ void k_iota(int32_t *v, int64_t n)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) v[i] = (int32_t)i;
}

__global__ void k_gather_levels(const uint8_t *__restrict__ lin, const int32_t *__restrict__ perm,
                                uint8_t *__restrict__ lout, int64_t n)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) lout[i] = lin[perm[i]];
}

// -- validation: the sorted leaves tile the cube exactly --------------------
enum : unsigned { kErrPartition = 1u, kErrDup = 2u, kErrLevel = 4u };

__global__ void k_validate(const uint64_t *__restrict__ keys, const uint8_t *__restrict__ lv, int64_t n,
                           int l_min, int L, unsigned *__restrict__ err)
{
    int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    unsigned e = 0;
    const uint64_t k = keys[j];
    const int l = lv[j];
    if (l < l_min || l > L || (k >> (3 * L)) != 0) {
        e |= kErrLevel;
    } else {
        const uint64_t vol = 1ull << (3 * (L - l));
        if (k & (vol - 1)) e |= kErrPartition;
        if (j == 0 && k != 0) e |= kErrPartition;
        if (j + 1 < n) {
            const uint64_t kn = keys[j + 1];
            if (kn == k) e |= kErrDup;
            else if (k + vol != kn) e |= kErrPartition;
        } else if (k + vol != (1ull << (3 * L))) {
            e |= kErrPartition;
        }
    }
    if (e) atomicOr(err, e);
}

// -- descent table ------------------------------------------------------------
// Number of split cells at each table level t (cells of level lev[t] covered
// by finer leaves): counted at the first leaf inside each such cell.
__global__ void k_count_splits(const uint64_t *__restrict__ keys, const uint8_t *__restrict__ lv, int64_t n,
                               TreeView tv, unsigned long long *__restrict__ counts)
{
    __shared__ unsigned sc[kMaxTabLevels];
    if (threadIdx.x < kMaxTabLevels) sc[threadIdx.x] = 0;
    __syncthreads();
    int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j < n) {
        const uint64_t k = keys[j];
        const int l = lv[j];
        for (int t = 0; t + 1 < tv.nlev; ++t) {
            const uint64_t cell = 1ull << (3 * (tv.L - tv.lev[t]));
            if (l > tv.lev[t] && (k & (cell - 1)) == 0) atomicAdd(&sc[t], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < kMaxTabLevels && sc[threadIdx.x]) atomicAdd(&counts[threadIdx.x], (unsigned long long)sc[threadIdx.x]);
}

__global__ void k_split_flags(const uint64_t *__restrict__ keys, const uint8_t *__restrict__ lv, int64_t n, int L,
                              int lev_t, uint32_t *__restrict__ flags)
{
    int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    const uint64_t cell = 1ull << (3 * (L - lev_t));
    flags[j] = (lv[j] > lev_t && (keys[j] & (cell - 1)) == 0) ? 1u : 0u;
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Write the entries of table level t.  Leaves with lev[t-1] < level <= lev[t]
// fill the 8^(lev[t]-level) entries they cover; the first leaf of each split
// level-lev[t] cell writes the pointer to its sub-table.
__global__ void k_write_level(const uint64_t *__restrict__ keys, const uint8_t *__restrict__ lv, int64_t n,
                              TreeView tv, uint32_t *__restrict__ table, int t, const uint32_t *__restrict__ sub_ids)
{
    int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int l = lv[j];
    if (t > 0 && l <= tv.lev[t - 1]) return;
    const uint64_t k = keys[j];
    const uint32_t ax = compact3_21(k), ay = compact3_21(k >> 1), az = compact3_21(k >> 2);
    const int L = tv.L;
    int64_t base;
    uint32_t digit;
    if (t == 0) {
        const int s = L - tv.lev[0];
        base = 0;
        digit = interleave3(ax >> s, ay >> s, az >> s);
    } else {
        // walk the already written levels 0..t-1; the leaf lies in a split cell at each
        const int s0 = L - tv.lev[0];
        uint32_t e = table[interleave3(ax >> s0, ay >> s0, az >> s0)];
        for (int u = 1; u < t; ++u) {
            const int d = tv.lev[u] - tv.lev[u - 1];
            const int s = L - tv.lev[u];
            const uint32_t m = (1u << d) - 1u;
            e = table[tv.off[u] + (int64_t)(e & ~kSplit) * (int64_t(1) << (3 * d)) +
                      interleave3((ax >> s) & m, (ay >> s) & m, (az >> s) & m)];
        }
        const int d = tv.lev[t] - tv.lev[t - 1];
        const int s = L - tv.lev[t];
        const uint32_t m = (1u << d) - 1u;
        base = tv.off[t] + (int64_t)(e & ~kSplit) * (int64_t(1) << (3 * d));
        digit = interleave3((ax >> s) & m, (ay >> s) & m, (az >> s) & m);
    }
    if (l <= tv.lev[t]) {
        const uint32_t ent = ((uint32_t)l << kLevelShift) | (uint32_t)j;
        const int64_t cnt = int64_t(1) << (3 * (tv.lev[t] - l));
        for (int64_t c = 0; c < cnt; ++c) table[base + digit + c] = ent;
    } else {
        const uint64_t cell = 1ull << (3 * (L - tv.lev[t]));
        if ((k & (cell - 1)) == 0) table[base + digit] = kSplit | sub_ids[j];
    }
}

// Summary of the root one level up: entry m describes the 8 root cells of
// the level-(r-1) cell m.  When all 8 are leaves of level r, they are 8
// consecutive leaves in Z-order and the entry is the first one's (so the
// leaf of child c is entry + c); otherwise it is kSplit.
__global__ void k_root_summary(const uint32_t *__restrict__ root, int64_t m_cells, int r, uint32_t *__restrict__ sum)
{
    const int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (m >= m_cells) return;
    bool uniform = true;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const uint32_t e = root[8 * m + c];
        uniform = uniform && !(e & kSplit) && (int)((e >> kLevelShift) & 31u) == r;
    }
    sum[m] = uniform ? root[8 * m] : kSplit;
}

__global__ void k_count_value(const uint32_t *__restrict__ p, int64_t n, uint32_t v, unsigned *__restrict__ out)
{
    unsigned c = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        c += (p[i] == v);
    if (c) atomicAdd(out, c);
}

inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
    void *release() { void *q = p; p = nullptr; return q; }
};

int dalloc(DevBuf &b, size_t bytes)
{
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return fail(OT_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    return OT_OK;
}

}  // namespace

// Device workspace (bytes) of radix_sort_pairs for n keys.
int64_t radix_ws_bytes(int64_t n)
{
    const int64_t nb = (n + kSortTile - 1) / kSortTile;
    const int64_t nc = (int64_t)kRadix * nb;
    return 4 * (2 * nc + scan_tmp_words(nc)) + 256;
}

// LSD radix sort of (key, value) pairs over the low `bits` bits, 8 bits per
// pass, without allocating (ws: radix_ws_bytes(n) bytes).  After an even
// number of passes the result is in (k0, v0), after an odd number in (k1, v1);
// *k_res / *v_res point at it.
void radix_sort_pairs(uint64_t *k0, int32_t *v0, uint64_t *k1, int32_t *v1, int64_t n, int bits, void *ws,
                      uint64_t **k_res, int32_t **v_res, hipStream_t s)
{
    const int nb = (int)((n + kSortTile - 1) / kSortTile);
    const int64_t ncounts = (int64_t)kRadix * nb;
    uint32_t *counts = (uint32_t *)ws, *offs = counts + ncounts, *tmp = offs + ncounts;
    uint64_t *ka = k0, *kb = k1;
    int32_t *va = v0, *vb = v1;
    for (int shift = 0; shift < bits && n > 0; shift += kRadixBits) {
        hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(kSortThreads), 0, s, ka, n, shift, counts, nb);
        exclusive_scan(counts, offs, ncounts, tmp, s);
        hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(kSortThreads), 0, s, ka, va, kb, vb, n, shift,
                           (const uint32_t *)offs, nb);
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    *k_res = ka;
    *v_res = va;
}

}  // namespace ot

using namespace ot;

extern "C" int ot_encode_keys(const uint32_t *anchors, int64_t n, int32_t l_max, uint64_t *keys, void *stream)
{
    if (n < 0 || (n > 0 && (!anchors || !keys))) return fail(OT_ERR_INVALID, "ot_encode_keys: bad arguments");
    if (l_max < 0 || l_max > 21) return fail(OT_ERR_LEVEL_RANGE, "ot_encode_keys: l_max must be in [0, 21]");
    if (n == 0) return OT_OK;
    hipLaunchKernelGGL(k_encode_keys, dim3(nblk(n)), dim3(256), 0, (hipStream_t)stream, anchors, n, keys);
    OT_HIP(hipGetLastError());
    return OT_OK;
}

extern "C" int ot_build_tree(const uint64_t *keys, const uint8_t *levels, int64_t n, const ot_tree_desc *desc,
                             int32_t *perm_out, void *stream, ot_tree **out)
{
    if (!out) return fail(OT_ERR_INVALID, "ot_build_tree: out is NULL");
    *out = nullptr;
    if (!desc || !keys || !levels || n <= 0) return fail(OT_ERR_INVALID, "ot_build_tree: bad arguments");
    const int L = desc->l_max, l_min = desc->l_min;
    if (L < 0 || L > 21 || l_min < 0 || l_min > L)
        return fail(OT_ERR_LEVEL_RANGE, "ot_build_tree: need 0 <= l_min <= l_max <= 21");
    if (n > kMaxLeaves) return fail(OT_ERR_CAPACITY, "ot_build_tree: more than 2^26 leaves");
    hipStream_t s = (hipStream_t)stream;
    int rc;

    DevBuf ka, kb, va, vb, lvs, scratch;
    if ((rc = dalloc(ka, n * 8)) || (rc = dalloc(kb, n * 8)) || (rc = dalloc(va, n * 4)) || (rc = dalloc(vb, n * 4)) ||
        (rc = dalloc(lvs, n)) || (rc = dalloc(scratch, 256)))
        return rc;
    OT_HIP(hipMemcpyAsync(ka.p, keys, n * 8, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_iota, dim3(nblk(n)), dim3(256), 0, s, (int32_t *)va.p, n);
    uint64_t *ks;
    int32_t *perm;
    DevBuf sws;
    if ((rc = dalloc(sws, radix_ws_bytes(n)))) return rc;
    // Keys of a valid tree use 3L bits; sort on those (others fail validation).
    radix_sort_pairs((uint64_t *)ka.p, (int32_t *)va.p, (uint64_t *)kb.p, (int32_t *)vb.p, n, 3 * L, sws.p, &ks,
                     &perm, s);
    OT_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_gather_levels, dim3(nblk(n)), dim3(256), 0, s, levels, perm, (uint8_t *)lvs.p, n);

    // Table layout: root level r = min(l_min, 8), then steps of <= 3 levels.
    TreeView tv{};
    tv.L = L;
    tv.periodic = desc->periodic ? 1 : 0;
    tv.lev[0] = std::min(l_min, kMaxRootLevel);
    tv.nlev = 1;
    while (tv.lev[tv.nlev - 1] < L) {
        tv.lev[tv.nlev] = std::min(tv.lev[tv.nlev - 1] + 3, L);
        tv.nlev++;
    }

    unsigned *err = (unsigned *)scratch.p;
    unsigned long long *cnt = (unsigned long long *)((char *)scratch.p + 64);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, (uint32_t *)scratch.p, (int64_t)64, 0u);
    hipLaunchKernelGGL(k_validate, dim3(nblk(n)), dim3(256), 0, s, ks, (const uint8_t *)lvs.p, n, l_min, L, err);
    hipLaunchKernelGGL(k_count_splits, dim3(nblk(n)), dim3(256), 0, s, ks, (const uint8_t *)lvs.p, n, tv, cnt);
    OT_HIP(hipGetLastError());
    unsigned herr = 0;
    unsigned long long hcnt[kMaxTabLevels] = {0};
    OT_HIP(hipMemcpyAsync(&herr, err, sizeof(herr), hipMemcpyDeviceToHost, s));
    OT_HIP(hipMemcpyAsync(hcnt, cnt, sizeof(hcnt), hipMemcpyDeviceToHost, s));
    OT_HIP(hipStreamSynchronize(s));
    if (herr & kErrLevel) return fail(OT_ERR_LEVEL_RANGE, "ot_build_tree: leaf level outside [l_min, l_max] or key above 3*l_max bits");
    if (herr & kErrDup) return fail(OT_ERR_UNSORTED_DUP, "ot_build_tree: two leaves share a Morton key");
    if (herr & kErrPartition) return fail(OT_ERR_NOT_PARTITION, "ot_build_tree: leaves do not tile the unit cube");

    int64_t entries = int64_t(1) << (3 * tv.lev[0]);
    tv.off[0] = 0;
    for (int t = 1; t < tv.nlev; ++t) {
        tv.off[t] = entries;
        entries += (int64_t)hcnt[t - 1] << (3 * (tv.lev[t] - tv.lev[t - 1]));
    }
    if (entries >= (int64_t(1) << 40)) return fail(OT_ERR_CAPACITY, "ot_build_tree: descent table too large");
    // the pool offsets follow the entries, 8-byte aligned, then the root's
    // summary one level up (an eighth of the root: most lookups of points in
    // random order then hit a table small enough for one XCD's L2)
    const int64_t off_at = (entries + 1) & ~int64_t(1);
    const int64_t sum_at = off_at + 2 * kMaxTabLevels;
    const int64_t sum_cells = tv.lev[0] >= 1 ? (int64_t(1) << (3 * (tv.lev[0] - 1))) : 0;
    DevBuf table, flags, ids, stmp;
    if ((rc = dalloc(table, (sum_at + sum_cells) * 4)) || (rc = dalloc(flags, n * 4)) || (rc = dalloc(ids, n * 4)) ||
        (rc = dalloc(stmp, scan_tmp_words(n) * 4)))
        return rc;
    hipLaunchKernelGGL(k_fill_u32, dim3(2048), dim3(256), 0, s, (uint32_t *)table.p, entries, 0xFFFFFFFFu);
    OT_HIP(hipMemcpyAsync((uint32_t *)table.p + off_at, tv.off, sizeof(tv.off), hipMemcpyHostToDevice, s));
    for (int t = 0; t < tv.nlev; ++t) {
        if (t + 1 < tv.nlev) {
            hipLaunchKernelGGL(k_split_flags, dim3(nblk(n)), dim3(256), 0, s, ks, (const uint8_t *)lvs.p, n, L,
                               tv.lev[t], (uint32_t *)flags.p);
            exclusive_scan((uint32_t *)flags.p, (uint32_t *)ids.p, n, (uint32_t *)stmp.p, s);
        }
        hipLaunchKernelGGL(k_write_level, dim3(nblk(n)), dim3(256), 0, s, ks, (const uint8_t *)lvs.p, n, tv,
                           (uint32_t *)table.p, t, (const uint32_t *)ids.p);
    }
    if (sum_cells)
        hipLaunchKernelGGL(k_root_summary, dim3(nblk(sum_cells)), dim3(256), 0, s, (const uint32_t *)table.p, sum_cells,
                           tv.lev[0], (uint32_t *)table.p + sum_at);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, (uint32_t *)scratch.p, (int64_t)1, 0u);
    hipLaunchKernelGGL(k_count_value, dim3(1024), dim3(256), 0, s, (const uint32_t *)table.p, entries, 0xFFFFFFFFu, err);
    OT_HIP(hipGetLastError());
    OT_HIP(hipMemcpyAsync(&herr, err, sizeof(herr), hipMemcpyDeviceToHost, s));
    if (perm_out) OT_HIP(hipMemcpyAsync(perm_out, perm, n * 4, hipMemcpyDeviceToDevice, s));
    OT_HIP(hipStreamSynchronize(s));
    if (herr) return fail(OT_ERR_NOT_PARTITION, "ot_build_tree: descent table has unfilled entries");

    ot_tree *tr = new ot_tree();
    OT_HIP(hipGetDevice(&tr->device));
    tr->cus = 0;
    (void)hipDeviceGetAttribute(&tr->cus, hipDeviceAttributeMultiprocessorCount, tr->device);
    if (tr->cus <= 0) tr->cus = 1;
    tr->l_min = l_min;
    tr->l_max = L;
    tr->periodic = tv.periodic;
    tr->n_leaves = n;
    // keep the sorted keys in whichever buffer holds them
    if (ks == (uint64_t *)ka.p) tr->keys = (uint64_t *)ka.release();
    else tr->keys = (uint64_t *)kb.release();
    tr->levels = (uint8_t *)lvs.release();
    tr->table = (uint32_t *)table.release();
    tr->table_entries = entries;
    tv.table = tr->table;
    tv.pool_off = (const int64_t *)(tr->table + off_at);
    tv.summary = sum_cells ? tr->table + sum_at : nullptr;
    tv.levels = tr->levels;
    tv.nleaf = (int32_t)n;
    tr->view = tv;
    *out = tr;
    return OT_OK;
}

extern "C" int ot_destroy_tree(ot_tree *t)
{
    if (!t) return OT_OK;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(t->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(t->keys);
    (void)hipFree(t->levels);
    (void)hipFree(t->table);
    (void)hipSetDevice(cur);
    delete t;
    return OT_OK;
}

extern "C" int ot_tree_info_get(const ot_tree *t, ot_tree_info *info)
{
    if (!t || !info) return fail(OT_ERR_INVALID, "ot_tree_info_get: NULL argument");
    info->n_leaves = t->n_leaves;
    info->l_min = t->l_min;
    info->l_max = t->l_max;
    info->periodic = t->periodic;
    info->table_levels = t->view.nlev;
    info->table_bytes = t->table_entries * 4;
    info->workspace_bytes = spread_ws_bytes(t->n_leaves);
    return OT_OK;
}

extern "C" int ot_tree_leaves(const ot_tree *t, uint64_t *keys_out, uint8_t *levels_out, void *stream)
{
    if (!t) return fail(OT_ERR_INVALID, "ot_tree_leaves: NULL tree");
    hipStream_t s = (hipStream_t)stream;
    if (keys_out) OT_HIP(hipMemcpyAsync(keys_out, t->keys, t->n_leaves * 8, hipMemcpyDeviceToDevice, s));
    if (levels_out) OT_HIP(hipMemcpyAsync(levels_out, t->levels, t->n_leaves, hipMemcpyDeviceToDevice, s));
    return OT_OK;
}
