// Internal definitions shared by the library's HIP sources (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/octrack.h"

namespace ot {

// ---------------------------------------------------------------------------
// Descent table.
//
// The Z-sorted leaf array (Sec. 3.1) is searched through a radix table over
// Morton digits instead of per-level binary searches: the root holds one
// entry per cell of level r = min(l_min, 8); a cell that is split into finer
// leaves points to a sub-table holding the cells up to 3 levels deeper
// (512 entries), and so on down to L.  Every entry is either
//   LEAF : bit 31 = 0, bits 26..30 = leaf level, bits 0..25 = leaf id
//   SPLIT: bit 31 = 1, bits 0..30 = sub-table index at the next table level.
// A lookup costs one dependent load per table level (2 for trees that span
// at most 3 levels below the root), and returns the leaf and its level at
// once.  It returns the same leaf as Algorithm 1 for every point: both find
// the unique leaf whose half-open box contains the point.
// ---------------------------------------------------------------------------
constexpr uint32_t kSplit = 0x80000000u;
constexpr uint32_t kIdMask = 0x03FFFFFFu;
constexpr int kLevelShift = 26;
constexpr int kMaxTabLevels = 9;
constexpr int kMaxRootLevel = 8;
constexpr int64_t kMaxLeaves = int64_t(1) << 26;

struct TreeView {
    const uint32_t *table;
    const uint8_t *levels;   // leaf levels in id order (hosts given by id)
    int32_t L;         // finest level
    int32_t periodic;
    int32_t nlev;      // table levels (root included)
    int32_t nleaf;     // leaves (ids are 0 .. nleaf - 1)
    int32_t lev[kMaxTabLevels];   // cell level of each table level; lev[0] = root level
    int64_t off[kMaxTabLevels];   // entry offset of each level's pool; off[0] = 0
    // The same pool offsets in device memory, after the table's entries.
    // Kernels index them by a level number that varies by lane: a dynamic
    // index into the by-value kernel argument above would put a copy of the
    // whole struct in per-lane scratch memory.  Level t's cells are at level
    // min(lev[0] + 3t, L), so lev[] itself is never indexed on the device.
    const int64_t *pool_off;
    // Root summary one level up (NULL when the root is level 0): entry m is
    // the leaf entry of the first of the 8 root cells of level-(lev[0]-1)
    // cell m when all 8 are leaves of level lev[0] (then child c's leaf is
    // entry + c), kSplit otherwise.
    const uint32_t *summary;
};

// Spread the low 10 bits of v so that bit b lands on bit 3b.
__host__ __device__ __forceinline__ uint32_t part1by2(uint32_t v)
{
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__host__ __device__ __forceinline__ uint32_t interleave3(uint32_t x, uint32_t y, uint32_t z)
{
    return part1by2(x) | (part1by2(y) << 1) | (part1by2(z) << 2);
}

// 64-bit Morton keys at 21 bits per axis (x lowest): spread the low 21 bits
// of v so that bit b lands on bit 3b, and the inverse.
__host__ __device__ __forceinline__ uint64_t split3_21(uint64_t v)
{
    v &= 0x1FFFFFull;
    v = (v | (v << 32)) & 0x1F00000000FFFFull;
    v = (v | (v << 16)) & 0x1F0000FF0000FFull;
    v = (v | (v << 8)) & 0x100F00F00F00F00Full;
    v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__host__ __device__ __forceinline__ uint32_t compact3_21(uint64_t v)
{
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10C30C30C30C30C3ull;
    v = (v ^ (v >> 4)) & 0x100F00F00F00F00Full;
    v = (v ^ (v >> 8)) & 0x1F0000FF0000FFull;
    v = (v ^ (v >> 16)) & 0x1F00000000FFFFull;
    v = (v ^ (v >> 32)) & 0x1FFFFFull;
    return (uint32_t)v;
}

// Descent-table entry i.  The table pointer reaches kernels inside
// TreeView, where the compiler cannot tell its address space and emits flat
// loads; a flat load counts against the LDS counter as well, so every wait
// for an LDS result would also wait for the table loads in flight.  Read it
// as global memory.
__device__ __forceinline__ uint32_t ld_table(const TreeView &tv, int64_t i)
{
    return ((const __attribute__((address_space(1))) uint32_t *)tv.table)[i];
}

// Index of the level-1 pool entry below root entry e for the finest-level
// cell (ix, iy, iz), or 0 when e is a leaf: callers issue many of these
// loads at once, at valid addresses and without branches, and keep the
// loaded entry only where e was split.  The level-1 pool offset is read at
// a constant index of the tree view (a scalar kernel argument).
__device__ __forceinline__ int64_t step1_index(const TreeView &tv, uint32_t e, uint32_t ix, uint32_t iy, uint32_t iz)
{
    const int l0 = tv.lev[0];
    const int l1 = min(l0 + 3, tv.L);
    const int d = l1 - l0, s = tv.L - l1;
    const uint32_t m = (1u << d) - 1u;
    const uint32_t sub = interleave3((ix >> s) & m, (iy >> s) & m, (iz >> s) & m);
    return (e & kSplit) ? tv.off[1] + (int64_t)(e & ~kSplit) * (int64_t(1) << (3 * d)) + sub : int64_t(0);
}

// Continue a descent from a level-1 table entry e down to the leaf entry of
// the finest-level cell (ix, iy, iz) (trees more than 3 levels deeper than
// the root).  The level of each table step is computed and its pool offset
// read from device memory: a lane-dependent index into the by-value tree
// view would put a copy of the struct in per-lane scratch memory.
__device__ __forceinline__ uint32_t descend_from_level2(const TreeView &tv, uint32_t e, uint32_t ix, uint32_t iy,
                                                        uint32_t iz)
{
    int lv = min(tv.lev[0] + 3, tv.L);
    for (int t = 2; t < tv.nlev && (e & kSplit); ++t) {
        const int nl = min(lv + 3, tv.L);
        const int d = nl - lv, s = tv.L - nl;
        const uint32_t m = (1u << d) - 1u;
        const uint32_t sub = interleave3((ix >> s) & m, (iy >> s) & m, (iz >> s) & m);
        const int64_t po = ((const __attribute__((address_space(1))) int64_t *)tv.pool_off)[t];
        e = ld_table(tv, po + (int64_t)(e & ~kSplit) * (int64_t(1) << (3 * d)) + sub);
        lv = nl;
    }
    return e;
}

// Continue a descent from root entry e down to the leaf entry of the
// finest-level cell (ix, iy, iz).
__device__ __forceinline__ uint32_t descend_below_root(const TreeView &tv, uint32_t e, uint32_t ix, uint32_t iy,
                                                       uint32_t iz)
{
    if (!(e & kSplit)) return e;
    e = ld_table(tv, step1_index(tv, e, ix, iy, iz));
    return (e & kSplit) ? descend_from_level2(tv, e, ix, iy, iz) : e;
}

__device__ __forceinline__ uint32_t ld_summary(const TreeView &tv, uint32_t m)
{
    return ((const __attribute__((address_space(1))) uint32_t *)tv.summary)[m];
}

// Table entry of the leaf containing the finest-level cell (ix, iy, iz).
// Points in random order look up the root summary first: a root an eighth
// the size, which one XCD's L2 holds; only cells whose 8 root children are
// not all root-level leaves continue to the root itself.
__device__ __forceinline__ uint32_t descend(const TreeView &tv, uint32_t ix, uint32_t iy,
                                            uint32_t iz)
{
    const int sh = tv.L - tv.lev[0];
    const uint32_t root = interleave3(ix >> sh, iy >> sh, iz >> sh);
    if (tv.summary) {
        const uint32_t sm = ld_summary(tv, root >> 3);
        if (!(sm & kSplit)) return sm + (root & 7u);
    }
    const uint32_t e = ld_table(tv, root);
    return descend_below_root(tv, e, ix, iy, iz);
}

// Integer coordinates at level L: floor(x 2^L) in FP64, wrapped (periodic)
// or range-checked.  False when the point has no host cell.  Branch-free:
// the periodic wrap is the floor-mod f - floor(f 2^-L) 2^L, exact in FP64
// for |f| < 2^52, so no 64-bit integer conversion is needed, and the axes'
// checks combine without short-circuits (which had compiled to a branch and
// an exec-mask update per test).
template <typename T>
__device__ __forceinline__ bool point_cell(const TreeView &tv, T x, T y, T z, uint32_t I[3])
{
    const double sc = (double)(int64_t(1) << tv.L);
    const double inv = 1.0 / sc;   // a power of two: exact
    const double v[3] = {(double)x * sc, (double)y * sc, (double)z * sc};
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const bool fin = fabs(v[d]) < 4503599627370496.0;   // 2^52; false for NaN
        double f = floor(fin ? v[d] : 0.0);
        if (tv.periodic) f -= floor(f * inv) * sc;          // floor-mod into [0, 2^L)
        const bool in = fin & (f >= 0.0) & (f < sc);
        ok = ok & in;
        I[d] = in ? (uint32_t)f : 0u;
    }
    return ok;
}

// Offsets of a point inside its level-l cell along one axis, from the scaled
// coordinate s = x 2^l: t = s - floor(s) in [0,1] and r = 1 - t, each formed
// from s itself.  Whichever is at most 1/2 is then exact (Sterbenz's lemma),
// negative s (a periodic wrap) included, where 1 - (s - floor(s)) would lose
// the digits of a small r and with them the relative accuracy of the weight
// r^2/... of the node at the far edge of the support.  For t <= 1/2 the
// plain 1 - t is kept: it lies in [1/2, 1], and (floor(s) + 1) could round
// for |s| beyond the significand.
template <typename T>
__device__ __forceinline__ void cell_offsets(T s, T &t, T &r)
{
    const T f = floor(s);
    t = s - f;
    r = t > T(0.5) ? (f + T(1)) - s : T(1) - t;
}

// 1-D weights of the three stencil nodes i0-1, i0, i0+1 for a point at
// fractional offset t in [0,1) inside its level-l cell, r = 1 - t.  With u = t - 1/2
// the node distances are u+1, u, u-1, and all three branches of phi share
// q = sqrt(1 - 3u^2) (substitute |r| = 1+u, |u|, 1-u into the phi equation of
// Sec. 2.2; -2 + 6|r| - 3r^2 = 1 - 3u^2 for |r| = 1 -+ u):
//   phi(u+1) = (2 - 3u - q)/6,  phi(u) = (1 + q)/3,  phi(u-1) = (2 + 3u - q)/6.
// The outer two lose all their digits to cancellation near the edge of the
// support; multiplying by the conjugate gives forms without cancellation,
//   (2 -+ 3u - q)/6 = (1 -+ 2u)^2 / (2 (2 -+ 3u + q)),  1 + 2u = 2t, 1 - 2u = 2(1-t),
// so every weight is accurate to a few ulp relative.  Derivatives d/du:
//   (u - q)/(2q),  -u/q,  (u + q)/(2q),
// with u -+ q rewritten the same way where it cancels
// (u - q = -4t(1-t)/(u+q) for u >= 0, u + q = 4t(1-t)/(q-u) for u < 0).
template <typename T>
__device__ __forceinline__ void delta3(T t, T s, T w[3])
{
    const T u = t - T(0.5);
    const T q = sqrt(T(1) - T(3) * u * u);
    w[0] = T(2) * s * s / (T(2) - T(3) * u + q);
    w[1] = (T(1) + q) * T(1.0 / 3.0);
    w[2] = T(2) * t * t / (T(2) + T(3) * u + q);
}

// FP32: the hardware square root and reciprocal (about 1 ulp each) instead
// of the correctly rounded sequences; 1 - 3u^2 lies in [1/4, 1] and the two
// denominators in [1, 9/2], so neither meets a special case.
template <>
__device__ __forceinline__ void delta3<float>(float t, float s, float w[3])
{
    const float u = t - 0.5f;
    const float q = __builtin_amdgcn_sqrtf(1.0f - 3.0f * u * u);
    w[0] = 2.0f * s * s * __builtin_amdgcn_rcpf(2.0f - 3.0f * u + q);
    w[1] = (1.0f + q) * (1.0f / 3.0f);
    w[2] = 2.0f * t * t * __builtin_amdgcn_rcpf(2.0f + 3.0f * u + q);
}

template <typename T>
__device__ __forceinline__ void delta3_grad(T t, T s, T w[3], T dw[3])
{
    const T u = t - T(0.5);
    const T q = sqrt(T(1) - T(3) * u * u);
    w[0] = T(2) * s * s / (T(2) - T(3) * u + q);
    w[1] = (T(1) + q) * T(1.0 / 3.0);
    w[2] = T(2) * t * t / (T(2) + T(3) * u + q);
    const T ts = t * s;
    dw[0] = u < T(0) ? (u - q) / (T(2) * q) : T(-2) * ts / (q * (u + q));
    dw[1] = -u / q;
    dw[2] = u < T(0) ? T(2) * ts / (q * (q - u)) : (u + q) / (T(2) * q);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);

// Device-wide helpers (tree_build.hip): exclusive scan of uint32 and the
// LDS-staged LSD radix sort of (uint64 key, int32 value) pairs.
int64_t scan_tmp_words(int64_t n);
void exclusive_scan(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp, hipStream_t s);
// The same scan without its last pass: out holds every 2048-value block's
// own exclusive scan and the result the blocks' scanned sums (element i's
// prefix is out[i] + result[i / 2048]); nullptr when out already holds the
// whole scan (one block, or more than 2048 blocks).
const uint32_t *exclusive_scan_split(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp, hipStream_t s);
constexpr int64_t kScanBlock = 2048;
int64_t radix_ws_bytes(int64_t n);
void radix_sort_pairs(uint64_t *k0, int32_t *v0, uint64_t *k1, int32_t *v1, int64_t n, int bits, void *ws,
                      uint64_t **k_res, int32_t **v_res, hipStream_t s);
int fail(int code, const std::string &msg);

// Fixed-point spreading workspace: a 256-byte header (FxState) followed by
// the n_leaves x 3 int64 accumulators.
constexpr int64_t kFxHeader = 256;
inline int64_t spread_ws_bytes(int64_t n_leaves) { return kFxHeader + n_leaves * 3 * 8; }
int hip_fail(hipError_t e, const char *what);

#define OT_HIP(call)                                      \
    do {                                                  \
        hipError_t _e = (call);                           \
        if (_e != hipSuccess) return ot::hip_fail(_e, #call); \
    } while (0)

}  // namespace ot

struct ot_tree {
    int device;
    int cus;             // compute units of that device
    int32_t l_min, l_max, periodic;
    int64_t n_leaves;
    uint64_t *keys;      // sorted Morton keys
    uint8_t *levels;     // levels in sorted order
    uint32_t *table;     // descent table (root + pools)
    int64_t table_entries;
    ot::TreeView view;
    // Read-only after the build: the workspace of fixed-point spreading
    // belongs to each call (or batch plan), so calls on one tree may run on
    // several streams at once.
};
