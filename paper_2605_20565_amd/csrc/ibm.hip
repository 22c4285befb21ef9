// Multi-direct forcing of the immersed-boundary method (IBM subsection of
// Sec. 2.2): per iteration, interpolate the leaf velocity to the markers,
// form the marker force from the slip against the prescribed marker
// velocity, spread it back to the leaves and correct the leaf velocity.
//
// The markers do not move during the iterations, so once per call every
// marker's stencil is computed and kept: its 27 node leaves and weights, as
// the tracking kernel forms them (its own lookups and products, so the same
// values).  The leaves the stencils reach are listed, and the (marker, node)
// pairs grouped by listed leaf.  An iteration is then two passes without
// atomic adds: one over the markers (interpolation by gathering through the
// kept stencils, slip force, max |F|), one over the listed leaves (each sums
// its pairs' contributions, in FIXED mode as the rounded integers of plain
// spreading, and applies u += f / rho).  Every marker's and every leaf's
// arithmetic is that of the plain composition of the library's
// interpolation and spreading (FIXED: bit for bit; ATOMIC: each leaf's sum
// in FP64, rounded once).  Everything is enqueued on the caller's stream;
// the caller provides the workspace; no memset nodes, so the call can be
// captured in a graph.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "ot_common.h"
#include "track_device.h"

namespace ot {
namespace {

constexpr int kNodes = 27;

// Sink of the stencil pass: keeps one point's node leaves and weights and
// flags the leaves.
template <typename T>
struct StencilSink {
    int32_t *leaf;   // the point's kNodes entries
    T *wt;           // the point's kNodes entries
    uint32_t *flags;
    __device__ __forceinline__ void add27(const uint32_t (&ent)[27], uint32_t live, const T (&w)[3][3], const T *,
                                          const uint32_t (&)[3][3], int)
    {
#pragma unroll
        for (int q = 0; q < kNodes; ++q) {
            if ((live >> q) & 1u) {
                const uint32_t l = ent[q] & kIdMask;
                leaf[q] = (int32_t)l;
                wt[q] = w[0][q % 3] * w[1][(q / 3) % 3] * w[2][q / 9];
                flags[l] = 1u;
            }
        }
    }
};

// Node leaves (-1: dropped at a wall, or no host) and weights of every marker.
template <typename T, bool PER>
__global__ __launch_bounds__(256) void k_mdf_stencil(TreeView tv, int64_t n, const T *__restrict__ pos,
                                                     int32_t *__restrict__ leaf, T *__restrict__ wt,
                                                     uint32_t *__restrict__ flags)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    int32_t *lk = leaf + kNodes * k;
    for (int q = 0; q < kNodes; ++q) lk[q] = -1;
    StencilSink<T> sink{lk, wt + kNodes * k, flags};
    // the positions stand in for the forces: the sink reads no values
    track_point<T, kOpSpread, PER>(tv, k, nullptr, 3, pos, nullptr, pos, nullptr, nullptr, sink);
}

__global__ __launch_bounds__(256) void k_compact(const uint32_t *__restrict__ flags, const uint32_t *__restrict__ offs,
                                                 int64_t m, int32_t *__restrict__ list, uint32_t *__restrict__ count)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        if (flags[i]) list[offs[i]] = (int32_t)i;
        if (i == m - 1) *count = offs[i] + flags[i];
    }
}

// Pairs per listed leaf (offs maps a flagged leaf to its list index).
__global__ __launch_bounds__(256) void k_pair_count(const int32_t *__restrict__ leaf, int64_t m,
                                                    const uint32_t *__restrict__ offs, uint32_t *__restrict__ cnt)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t l = leaf[i];
        if (l >= 0) atomicAdd(&cnt[offs[l]], 1u);
    }
}

// pairs[start[li] ..] = marker * kNodes + node of every pair reaching listed leaf li.
__global__ __launch_bounds__(256) void k_pair_fill(const int32_t *__restrict__ leaf, int64_t m,
                                                   const uint32_t *__restrict__ offs, const uint32_t *__restrict__ start,
                                                   uint32_t *__restrict__ cursor, uint32_t *__restrict__ pairs)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t l = leaf[i];
        if (l >= 0) {
            const uint32_t li = offs[l];
            pairs[start[li] + atomicAdd(&cursor[li], 1u)] = (uint32_t)i;
        }
    }
}

// Per marker: U = sum over its kept nodes of w u[leaf] (the tracking
// kernel's order and operations), F = (target - U) / dt into fk, f_lag
// (nullable) += F, and max |F| (finite components) into *maxbits (nullable).
template <typename T>
__global__ __launch_bounds__(256) void k_mdf_markers(int64_t n, const int32_t *__restrict__ leaf,
                                                     const T *__restrict__ wt, const T *__restrict__ u,
                                                     const T *__restrict__ target, T *__restrict__ fk,
                                                     T *__restrict__ f_lag, T dt, unsigned long long *__restrict__ maxbits)
{
    __shared__ unsigned long long wmax[4];
    unsigned long long best = 0;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        // all 27 leaf ids and weights first, then the gathers: independent loads
        int32_t lq[kNodes];
        T wq[kNodes];
#pragma unroll
        for (int q = 0; q < kNodes; ++q) {
            lq[q] = leaf[kNodes * k + q];
            wq[q] = wt[kNodes * k + q];
        }
        T U[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int q = 0; q < kNodes; ++q) {
            if (lq[q] < 0) continue;
            const int64_t j = 3 * (int64_t)lq[q];
            U[0] = fma(wq[q], u[j], U[0]);
            U[1] = fma(wq[q], u[j + 1], U[1]);
            U[2] = fma(wq[q], u[j + 2], U[2]);
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const T F = (target[3 * k + d] - U[d]) / dt;
            fk[3 * k + d] = F;
            if (f_lag) f_lag[3 * k + d] += F;
            if (isfinite(F)) best = std::max(best, abs_bits(F));
        }
    }
    if (!maxbits) return;   // the same for every thread
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) best = std::max(best, (unsigned long long)__shfl_xor(best, o, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) best = std::max(best, wmax[w]);
        if (best) atomicMax(maxbits, best);
    }
}

// Per listed leaf: f = the sum of its pairs' contributions w F (FIXED: the
// rounded integers rint(w F 2^s) of plain spreading, with its scale;
// ATOMIC: FP64), then u += f / rho and f_eul (nullable) += f.  FIXED also
// clears the next iteration's max |F| slot (next_max, not read here).
template <typename T, bool FIXED>
__global__ __launch_bounds__(256) void k_mdf_leaves(const int32_t *__restrict__ list, const uint32_t *__restrict__ count,
                                                    const uint32_t *__restrict__ start, const uint32_t *__restrict__ pairs,
                                                    const T *__restrict__ wt, const T *__restrict__ fk,
                                                    const unsigned long long *__restrict__ maxbits,
                                                    unsigned long long *__restrict__ next_max, int64_t n,
                                                    T *__restrict__ u, T *__restrict__ f_eul, T rho)
{
    const int64_t c = *count;
    double scale = 0.0, inv = 0.0;
    if constexpr (FIXED) {
        const int s = fx_shift<T>(*maxbits, n);
        scale = ldexp(1.0, s);
        inv = ldexp(1.0, -s);
        if (blockIdx.x == 0 && threadIdx.x == 0) *next_max = 0ull;
    }
    using Acc = typename std::conditional<FIXED, unsigned long long, double>::type;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < c; i += (int64_t)gridDim.x * blockDim.x) {
        Acc a[3] = {Acc(0), Acc(0), Acc(0)};
#pragma unroll 4
        for (uint32_t p = start[i]; p < start[i + 1]; ++p) {
            const uint32_t pr = pairs[p];
            const int64_t k = pr / kNodes;
            const T w = wt[pr];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                if constexpr (FIXED) a[d] += fx_round_fma((double)w, (double)fk[3 * k + d] * scale);
                else a[d] += (double)w * (double)fk[3 * k + d];
            }
        }
        const int64_t j = 3 * (int64_t)list[i];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const T fi = FIXED ? (T)((double)(long long)a[d] * inv) : (T)a[d];
            u[j + d] += fi / rho;
            if (f_eul) f_eul[j + d] += fi;
        }
    }
}

unsigned grid_for(int64_t m) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((m + 255) / 256, 4096)); }

// Workspace layout (bytes, each part 256-aligned): kept node leaves and
// weights (27n each), marker forces (3n T), flags, offsets and list
// (n_leaves words each), count, scan scratch, pair counts and starts
// (min(n_leaves, 27n) + 1 words each), pairs (27n words), two max |F| slots.
struct MdfWork {
    int32_t *leaf, *list;
    void *wt, *fk;
    uint32_t *flags, *offs, *count, *tmp, *cnt, *start, *pairs;
    unsigned long long *maxb;
    int64_t lmax;
};

int64_t align256(int64_t b) { return (b + 255) & ~int64_t(255); }

int64_t mdf_layout(int64_t n, int64_t n_leaves, int64_t tsize, char *base, MdfWork *w)
{
    int64_t o = 0;
    auto take = [&](int64_t bytes) {
        char *p = base ? base + o : nullptr;
        o += align256(bytes);
        return p;
    };
    const int64_t lmax = std::min<int64_t>(n_leaves, kNodes * n);
    char *leaf = take(4 * kNodes * n), *wt = take(tsize * kNodes * n), *fk = take(3 * n * tsize);
    char *flags = take(4 * n_leaves), *offs = take(4 * n_leaves), *list = take(4 * n_leaves);
    char *count = take(4), *tmp = take(4 * scan_tmp_words(n_leaves + 1));
    char *cnt = take(4 * (lmax + 1)), *start = take(4 * (lmax + 1)), *pairs = take(4 * kNodes * n);
    char *maxb = take(16);
    if (w)
        *w = MdfWork{(int32_t *)leaf,      (int32_t *)list,  wt,
                     fk,                   (uint32_t *)flags, (uint32_t *)offs,
                     (uint32_t *)count,    (uint32_t *)tmp,   (uint32_t *)cnt,
                     (uint32_t *)start,    (uint32_t *)pairs, (unsigned long long *)maxb,
                     lmax};
    return o;
}

template <typename T>
int mdf(const ot_tree *t, T *field, const T *pos, const T *target, int64_t n, int n_iter, T dt, T rho, int mode,
        T *f_lag, T *f_eul, void *work, hipStream_t s)
{
    const int64_t m_pts = 3 * n, m_leaves = 3 * t->n_leaves, m_nodes = kNodes * n;
    MdfWork w;
    mdf_layout(n, t->n_leaves, sizeof(T), (char *)work, &w);
    T *wt = (T *)w.wt, *fk = (T *)w.fk;
    if (f_lag) hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(m_pts)), dim3(256), 0, s, f_lag, m_pts, T(0));
    if (f_eul) hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(m_leaves)), dim3(256), 0, s, f_eul, m_leaves, T(0));
    if (n_iter == 0 || n == 0) {
        OT_HIP(hipGetLastError());
        return OT_OK;
    }
    // stencils kept, leaves listed, pairs grouped by listed leaf: once
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(t->n_leaves)), dim3(256), 0, s, w.flags, t->n_leaves, 0u);
    const dim3 gm((unsigned)((n + 255) / 256));
    if (t->view.periodic)
        hipLaunchKernelGGL((k_mdf_stencil<T, true>), gm, dim3(256), 0, s, t->view, n, pos, w.leaf, wt, w.flags);
    else
        hipLaunchKernelGGL((k_mdf_stencil<T, false>), gm, dim3(256), 0, s, t->view, n, pos, w.leaf, wt, w.flags);
    exclusive_scan(w.flags, w.offs, t->n_leaves, w.tmp, s);
    hipLaunchKernelGGL(k_compact, dim3(grid_for(t->n_leaves)), dim3(256), 0, s, w.flags, w.offs, t->n_leaves, w.list,
                       w.count);
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(w.lmax + 1)), dim3(256), 0, s, w.cnt, w.lmax + 1, 0u);
    hipLaunchKernelGGL(k_pair_count, dim3(grid_for(m_nodes)), dim3(256), 0, s, w.leaf, m_nodes, w.offs, w.cnt);
    exclusive_scan(w.cnt, w.start, w.lmax + 1, w.tmp, s);
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(w.lmax + 1)), dim3(256), 0, s, w.cnt, w.lmax + 1, 0u);
    hipLaunchKernelGGL(k_pair_fill, dim3(grid_for(m_nodes)), dim3(256), 0, s, w.leaf, m_nodes, w.offs, w.start,
                       w.cnt, w.pairs);
    OT_HIP(hipGetLastError());
    const bool fixed = mode == OT_SPREAD_FIXED;
    if (fixed) hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(1), dim3(64), 0, s, w.maxb, (int64_t)2, 0ull);
    const unsigned gl = grid_for(w.lmax);
    for (int it = 0; it < n_iter; ++it) {
        unsigned long long *mx = fixed ? w.maxb + (it & 1) : nullptr;
        hipLaunchKernelGGL(k_mdf_markers<T>, dim3(grid_for(n)), dim3(256), 0, s, n, (const int32_t *)w.leaf,
                           (const T *)wt, (const T *)field, target, fk, f_lag, dt, mx);
        if (fixed)
            hipLaunchKernelGGL((k_mdf_leaves<T, true>), dim3(gl), dim3(256), 0, s, (const int32_t *)w.list,
                               (const uint32_t *)w.count, (const uint32_t *)w.start, (const uint32_t *)w.pairs,
                               (const T *)wt, (const T *)fk, (const unsigned long long *)mx, w.maxb + ((it + 1) & 1),
                               n, field, f_eul, rho);
        else
            hipLaunchKernelGGL((k_mdf_leaves<T, false>), dim3(gl), dim3(256), 0, s, (const int32_t *)w.list,
                               (const uint32_t *)w.count, (const uint32_t *)w.start, (const uint32_t *)w.pairs,
                               (const T *)wt, (const T *)fk, (const unsigned long long *)nullptr,
                               (unsigned long long *)nullptr, n, field, f_eul, rho);
        OT_HIP(hipGetLastError());
    }
    return OT_OK;
}

}  // namespace
}  // namespace ot

using namespace ot;

extern "C" int64_t ot_mdf_workspace_bytes(const ot_tree *tree, int64_t n, int32_t dtype)
{
    if (!tree || n < 0 || (dtype != OT_F32 && dtype != OT_F64)) return -1;
    return mdf_layout(n, tree->n_leaves, dtype == OT_F32 ? 4 : 8, nullptr, nullptr);
}

extern "C" int ot_mdf(const ot_tree *tree, void *field, const void *pos, const void *target, int32_t dtype, int64_t n,
                      int32_t n_iter, double dt, double rho, int32_t mode, void *force_lag, void *force_eul,
                      void *work, void *stream)
{
    if (!tree) return fail(OT_ERR_INVALID, "ot_mdf: tree is NULL");
    if (dtype != OT_F32 && dtype != OT_F64) return fail(OT_ERR_INVALID, "dtype must be OT_F32 or OT_F64");
    if (n < 0 || n_iter < 0) return fail(OT_ERR_INVALID, "ot_mdf: n and n_iter must be >= 0");
    if (mode != OT_SPREAD_ATOMIC && mode != OT_SPREAD_FIXED) return fail(OT_ERR_INVALID, "bad spread mode");
    if (!(dt > 0.0) || !(rho > 0.0)) return fail(OT_ERR_INVALID, "ot_mdf: dt and rho must be positive");
    if (!field || !work || (n > 0 && (!pos || !target)))
        return fail(OT_ERR_INVALID, "ot_mdf: field, work, pos or target is NULL");
    if ((uintptr_t)work & 7) return fail(OT_ERR_INVALID, "ot_mdf: work must be 8-byte aligned");
    if (n > (int64_t)(UINT32_MAX / kNodes)) return fail(OT_ERR_CAPACITY, "ot_mdf: at most 159,072,862 markers");
    hipStream_t s = (hipStream_t)stream;
    if (dtype == OT_F32)
        return mdf<float>(tree, (float *)field, (const float *)pos, (const float *)target, n, n_iter, (float)dt,
                          (float)rho, mode, (float *)force_lag, (float *)force_eul, work, s);
    return mdf<double>(tree, (double *)field, (const double *)pos, (const double *)target, n, n_iter, dt, rho, mode,
                       (double *)force_lag, (double *)force_eul, work, s);
}
