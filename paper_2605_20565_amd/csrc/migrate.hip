// Phase I of the migration of Lagrangian points (Algorithm 2) on one device.
//
// relocate: after the points moved (usually by less than a cell, Sec. 3.2),
// each keeps its previous host leaf when that leaf still contains it (one
// key + level load and an integer compare) and otherwise descends the table
// again; the points whose host changed are counted.
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
__global__ __launch_bounds__(kThreads) void k_relocate(TreeView tv, const uint64_t *__restrict__ keys,
                                                       const uint8_t *__restrict__ levels, int64_t n_leaves,
                                                       const T *__restrict__ pos, int64_t n, int32_t *__restrict__ ids,
                                                       unsigned long long *__restrict__ moved)
{
    __shared__ unsigned long long sh[kThreads / 64];
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    unsigned long long changed = 0;
    if (k < n) {
        const int32_t prev = ids[k];
        uint32_t I[3];
        const bool ok = point_cell<T>(tv, pos[3 * k], pos[3 * k + 1], pos[3 * k + 2], I);
        int32_t id = -1;
        if (ok) {
            bool inside = false;
            if (prev >= 0 && prev < n_leaves) {
                const uint64_t key = keys[prev];
                const int sh_l = tv.L - (int)levels[prev];
                inside = ((I[0] >> sh_l) == (compact3_21(key) >> sh_l)) &&
                         ((I[1] >> sh_l) == (compact3_21(key >> 1) >> sh_l)) &&
                         ((I[2] >> sh_l) == (compact3_21(key >> 2) >> sh_l));
            }
            id = inside ? prev : (int32_t)(descend(tv, I[0], I[1], I[2]) & kIdMask);
        }
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

template <typename T>
__global__ __launch_bounds__(kThreads) void k_find_owner(TreeView tv, const int64_t *__restrict__ split, int P,
                                                         const T *__restrict__ pos, int64_t n,
                                                         int32_t *__restrict__ owner,
                                                         unsigned long long *__restrict__ counts)
{
    __shared__ unsigned int hist[kMaxOwners];
    if (counts) {
        for (int i = threadIdx.x; i < P; i += kThreads) hist[i] = 0u;
        __syncthreads();
    }
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < n) {
        uint32_t I[3];
        const bool ok = point_cell<T>(tv, pos[3 * k], pos[3 * k + 1], pos[3 * k + 2], I);
        int32_t o = -1;
        if (ok) {
            const int64_t key = (int64_t)(split3_21(I[0]) | (split3_21(I[1]) << 1) | (split3_21(I[2]) << 2));
            // largest r in [0, P) with split[r] <= key
            int lo = 0, hi = P;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (split[mid] <= key) lo = mid;
                else hi = mid;
            }
            o = lo;
            if (counts) atomicAdd(&hist[o], 1u);
        }
        owner[k] = o;
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
            hipLaunchKernelGGL(k_relocate<float>, g, b, 0, s, t->view, t->keys, t->levels, t->n_leaves,
                               (const float *)pos, n, ids, mv);
        else
            hipLaunchKernelGGL(k_relocate<double>, g, b, 0, s, t->view, t->keys, t->levels, t->n_leaves,
                               (const double *)pos, n, ids, mv);
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
        const dim3 g((unsigned)((n + kThreads - 1) / kThreads)), b(kThreads);
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
