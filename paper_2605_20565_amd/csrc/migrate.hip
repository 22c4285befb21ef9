// Phase I of the migration of Lagrangian points (Algorithm 2) on one device.
//
// relocate: the host of every moved point and the number of points whose
// host changed (the leavers of phase I).  The paper checks the previous host
// first because its search is a binary search; here a fresh descent is one
// or two loads from the (cached) descent table, cheaper than fetching the
// previous leaf's key and level (measured: 0.12 against 0.25 ms for 10^7
// points), so every point descends and is compared with its previous id.
// find_owner: under a partition of the leaves into contiguous Morton ranges
// (Sec. 3.1), the owner of a point is the range holding the Morton key of
// its finest-level cell, found by a binary search over the P + 1 splitters;
// the per-owner counts are the sizes of the send buffers of phase II.
#include <hip/hip_runtime.h>

#include "ot_common.h"
#include "track_device.h"

namespace ot {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxOwners = 4096;

__device__ __forceinline__ void block_count_to(unsigned long long v, unsigned long long *sh, unsigned long long *out)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += (unsigned long long)__shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kThreads / 64; ++w) v += sh[w];
        if (v) atomicAdd(out, v);
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_relocate(TreeView tv, const T *__restrict__ pos, int64_t n,
                                                       int32_t *__restrict__ ids,
                                                       unsigned long long *__restrict__ moved)
{
    __shared__ unsigned long long sh[kThreads / 64];
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    unsigned long long changed = 0;
    if (k < n) {
        const int32_t prev = ids[k];
        uint32_t I[3];
        const bool ok = point_cell<T>(tv, pos[3 * k], pos[3 * k + 1], pos[3 * k + 2], I);
        const int32_t id = ok ? (int32_t)(descend(tv, I[0], I[1], I[2]) & kIdMask) : -1;
        ids[k] = id;
        changed = id != prev ? 1ull : 0ull;
    }
    if (moved) block_count_to(changed, sh, moved);
}

__global__ void k_leaf_splitters(const uint64_t *__restrict__ keys, int64_t n_leaves, int P, int L,
                                 int64_t *__restrict__ split)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r > P) return;
    if (r == 0) split[0] = 0;
    else if (r == P) split[P] = (int64_t)1 << (3 * L);
    else split[r] = (int64_t)keys[((int64_t)r * n_leaves) / P];
}

// Splitters staged in LDS; each thread takes kOwnerItems points.  Counts:
// for up to kBallotOwners owners every wave counts each owner with one
// ballot (no same-address atomics), else LDS atomics.
constexpr int kOwnerItems = 8;
constexpr int kBallotOwners = 32;

template <typename T>
__global__ __launch_bounds__(kThreads) void k_find_owner(TreeView tv, const int64_t *__restrict__ split, int P,
                                                         const T *__restrict__ pos, int64_t n,
                                                         int32_t *__restrict__ owner,
                                                         unsigned long long *__restrict__ counts)
{
    __shared__ int64_t s_split[kMaxOwners + 1];
    __shared__ unsigned int hist[kMaxOwners];
    for (int i = threadIdx.x; i <= P; i += kThreads) s_split[i] = split[i];
    for (int i = threadIdx.x; i < P; i += kThreads) hist[i] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kThreads * kOwnerItems;
    for (int j = 0; j < kOwnerItems; ++j) {
        const int64_t k = base + (int64_t)j * kThreads + threadIdx.x;
        int32_t o = -1;
        if (k < n) {
            uint32_t I[3];
            const bool ok = point_cell<T>(tv, pos[3 * k], pos[3 * k + 1], pos[3 * k + 2], I);
            if (ok) {
                const int64_t key = (int64_t)(split3_21(I[0]) | (split3_21(I[1]) << 1) | (split3_21(I[2]) << 2));
                // largest r in [0, P) with split[r] <= key
                int lo = 0, hi = P;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_split[mid] <= key) lo = mid;
                    else hi = mid;
                }
                o = lo;
            }
            owner[k] = o;
        }
        if (counts) {
            if (P <= kBallotOwners) {
                for (int r = 0; r < P; ++r) {
                    const unsigned long long m = __ballot(o == r);
                    if ((threadIdx.x & 63) == 0 && m) atomicAdd(&hist[r], (unsigned)__popcll(m));
                }
            } else if (o >= 0) {
                atomicAdd(&hist[o], 1u);
            }
        }
    }
    if (counts) {
        __syncthreads();
        for (int i = threadIdx.x; i < P; i += kThreads)
            if (hist[i]) atomicAdd(&counts[i], (unsigned long long)hist[i]);
    }
}

}  // namespace
}  // namespace ot

using namespace ot;

extern "C" int ot_relocate(const ot_tree *t, const void *pos, int32_t dtype, int64_t n, int32_t *ids, int64_t *moved,
                           void *stream)
{
    if (!t) return fail(OT_ERR_INVALID, "ot_relocate: tree is NULL");
    if (dtype != OT_F32 && dtype != OT_F64) return fail(OT_ERR_INVALID, "dtype must be OT_F32 or OT_F64");
    if (n < 0) return fail(OT_ERR_INVALID, "n < 0");
    if (n > 0 && (!pos || !ids)) return fail(OT_ERR_INVALID, "ot_relocate: pos or ids is NULL");
    hipStream_t s = (hipStream_t)stream;
    unsigned long long *mv = (unsigned long long *)moved;
    if (mv) hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(1), dim3(64), 0, s, mv, (int64_t)1, 0ull);
    if (n > 0) {
        const dim3 g((unsigned)((n + kThreads - 1) / kThreads)), b(kThreads);
        if (dtype == OT_F32)
            hipLaunchKernelGGL(k_relocate<float>, g, b, 0, s, t->view, (const float *)pos, n, ids, mv);
        else
            hipLaunchKernelGGL(k_relocate<double>, g, b, 0, s, t->view, (const double *)pos, n, ids, mv);
    }
    OT_HIP(hipGetLastError());
    return OT_OK;
}

extern "C" int ot_leaf_splitters(const ot_tree *t, int32_t P, int64_t *splitters, void *stream)
{
    if (!t || !splitters) return fail(OT_ERR_INVALID, "ot_leaf_splitters: NULL argument");
    if (P < 1 || P > kMaxOwners || P > t->n_leaves) return fail(OT_ERR_INVALID, "ot_leaf_splitters: need 1 <= P <= min(4096, n_leaves)");
    hipLaunchKernelGGL(k_leaf_splitters, dim3((unsigned)((P + 1 + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       t->keys, t->n_leaves, (int)P, (int)t->l_max, splitters);
    OT_HIP(hipGetLastError());
    return OT_OK;
}

extern "C" int ot_find_owner(const int64_t *splitters, int32_t P, int32_t l_max, int32_t periodic, const void *pos,
                             int32_t dtype, int64_t n, int32_t *owner, int64_t *counts, void *stream)
{
    if (P < 1 || P > kMaxOwners) return fail(OT_ERR_INVALID, "ot_find_owner: need 1 <= P <= 4096");
    if (l_max < 0 || l_max > 21) return fail(OT_ERR_LEVEL_RANGE, "ot_find_owner: l_max outside [0, 21]");
    if (dtype != OT_F32 && dtype != OT_F64) return fail(OT_ERR_INVALID, "dtype must be OT_F32 or OT_F64");
    if (n < 0) return fail(OT_ERR_INVALID, "n < 0");
    if (!splitters || (n > 0 && (!pos || !owner))) return fail(OT_ERR_INVALID, "ot_find_owner: NULL array");
    hipStream_t s = (hipStream_t)stream;
    unsigned long long *cnt = (unsigned long long *)counts;
    if (cnt) hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(16), dim3(256), 0, s, cnt, (int64_t)P, 0ull);
    TreeView tv{};
    tv.L = l_max;
    tv.periodic = periodic ? 1 : 0;
    if (n > 0) {
        const int64_t per_block = (int64_t)kThreads * kOwnerItems;
        const dim3 g((unsigned)((n + per_block - 1) / per_block)), b(kThreads);
        if (dtype == OT_F32)
            hipLaunchKernelGGL(k_find_owner<float>, g, b, 0, s, tv, splitters, (int)P, (const float *)pos, n, owner,
                               cnt);
        else
            hipLaunchKernelGGL(k_find_owner<double>, g, b, 0, s, tv, splitters, (int)P, (const double *)pos, n,
                               owner, cnt);
    }
    OT_HIP(hipGetLastError());
    return OT_OK;
}
