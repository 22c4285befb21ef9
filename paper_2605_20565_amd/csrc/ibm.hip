// Multi-direct forcing of the immersed-boundary method (IBM subsection of
// Sec. 2.2): per iteration, interpolate the leaf velocity to the markers,
// form the marker force from the slip against the prescribed marker
// velocity, spread it back to the leaves and correct the leaf velocity.
// The interpolation and spreading are the library's own (any spreading mode).
//
// The markers do not move during the iterations, so once per call they are
// sorted by host leaf (the library's point sort; a bubble's markers come in
// an order that spreads each workgroup's tile over the whole surface, which
// overflows the spreading table) and the leaves their stencils reach are
// found (a marking pass that runs the spreading kernel's own node lookup)
// and compacted into a list; each iteration then works on the sorted
// markers and clears, converts and updates only the listed leaves instead
// of sweeping all of them.  Every marker's arithmetic and every leaf's is
// that of the plain composition in input order (leaves that no marker
// reaches receive nothing; FIXED sums do not depend on the order).
// Everything is enqueued on the caller's stream; the caller provides the
// workspace; no memset nodes, so the call can be captured in a graph.
#include <hip/hip_runtime.h>

#include "ot_common.h"
#include "point_sort.h"
#include "track_device.h"

namespace ot {
int track(const ot_tree *t, int ops, const void *field, const void *force, const void *pos, int dtype, int64_t n,
          int mode, int accumulate, int32_t *ids, void *vel, void *fout, hipStream_t s);
int spread_kernel(const ot_tree *t, int dtype, int mode, const void *force, const void *pos, int64_t n, void *fout,
                  hipStream_t s);

namespace {

// Sink of the marking pass: flags every leaf a marker's stencil reaches.
struct MarkSink {
    uint32_t *flags;
    template <typename T>
    __device__ __forceinline__ void add27(const uint32_t (&ent)[27], uint32_t live, const T (&)[3][3], const T *)
    {
#pragma unroll
        for (int q = 0; q < 27; ++q)
            if ((live >> q) & 1u) flags[ent[q] & kIdMask] = 1u;
    }
};

template <typename T, bool PER>
__global__ __launch_bounds__(256) void k_mark(TreeView tv, int64_t n, const T *__restrict__ pos,
                                              uint32_t *__restrict__ flags)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    MarkSink sink{flags};
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

// Zero the three components of every listed leaf.
template <typename A>
__global__ __launch_bounds__(256) void k_clear_listed(const int32_t *__restrict__ list, const uint32_t *__restrict__ count,
                                                      A *__restrict__ a)
{
    const int64_t c = *count;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < c; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = 3 * (int64_t)list[i];
        a[j] = A(0);
        a[j + 1] = A(0);
        a[j + 2] = A(0);
    }
}

// u += f / rho and f_eul += f on the listed leaves; f from the spread sums
// (ATOMIC) or converted from the fixed-point sums as the finalisation of
// plain spreading does (FIXED).  The sums are cleared for the next
// iteration, and so is max |F| (FIXED; the scale has been taken from it).
template <typename T, bool FIXED>
__global__ __launch_bounds__(256) void k_mdf_update_listed(const int32_t *__restrict__ list,
                                                           const uint32_t *__restrict__ count, T *__restrict__ u,
                                                           T *__restrict__ f, unsigned long long *__restrict__ acc,
                                                           FxState *__restrict__ fx, T *__restrict__ f_eul, T rho)
{
    const int64_t c = *count;
    const double inv = FIXED ? fx->inv : 0.0;
    if (FIXED && blockIdx.x == 0 && threadIdx.x == 0) fx->maxbits = 0ull;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < c; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = 3 * (int64_t)list[i];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            T fi;
            if constexpr (FIXED) {
                fi = (T)((double)(long long)acc[j + d] * inv);
                acc[j + d] = 0ull;
            } else {
                fi = f[j + d];
                f[j + d] = T(0);
            }
            u[j + d] += fi / rho;
            if (f_eul) f_eul[j + d] += fi;
        }
    }
}

// In sorted order: buf holds the interpolated marker velocity u_k on entry
// and the marker force F_k = (U_k - u_k) / dt on exit; f_lag (nullable, input
// order) accumulates F_k at the marker's input index.  maxbits != null: the
// bit pattern of max |F| over the finite components is maxed into it (the
// fixed-point scale's input, as the plain spreading takes it).
template <typename T>
__global__ __launch_bounds__(256) void k_mdf_force(int64_t m, const T *__restrict__ target, T *__restrict__ buf,
                                                   const uint64_t *__restrict__ kv, T *__restrict__ f_lag, T dt,
                                                   unsigned long long *__restrict__ maxbits)
{
    __shared__ unsigned long long wmax[4];
    unsigned long long best = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const T F = (target[i] - buf[i]) / dt;
        buf[i] = F;
        if (f_lag) f_lag[3 * (int64_t)(uint32_t)kv[i / 3] + i % 3] += F;
        if (isfinite(F)) best = std::max(best, abs_bits(F));
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

// Prescribed marker velocities in sorted order.
template <typename T>
__global__ __launch_bounds__(256) void k_gather_rows(int64_t m, const T *__restrict__ in, const uint64_t *__restrict__ kv,
                                                     T *__restrict__ out)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[3 * (int64_t)(uint32_t)kv[i / 3] + i % 3];
}

unsigned grid_for(int64_t m) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((m + 255) / 256, 4096)); }

// Workspace layout (bytes, each part 256-aligned): marker values and
// sorted targets (3n T each), leaf sums (3 n_leaves T), flags, offsets and
// list (n_leaves words each), count, scan scratch, the point sort's two key
// and two record buffers and its counting workspace.
struct MdfWork {
    void *fk, *tg, *f;
    uint32_t *flags, *offs, *count, *tmp;
    int32_t *list;
    uint64_t *kv[2];
    void *rec[2], *sws;
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
    char *fk = take(3 * n * tsize), *tg = take(3 * n * tsize), *f = take(3 * n_leaves * tsize);
    char *flags = take(4 * n_leaves), *offs = take(4 * n_leaves), *list = take(4 * n_leaves);
    char *count = take(4), *tmp = take(4 * scan_tmp_words(n_leaves));
    char *kv0 = take(8 * n), *kv1 = take(8 * n), *rec0 = take(3 * n * tsize), *rec1 = take(3 * n * tsize);
    char *sws = take(point_sort_ws_bytes(n));
    if (w)
        *w = MdfWork{fk,       tg, f, (uint32_t *)flags, (uint32_t *)offs, (uint32_t *)count, (uint32_t *)tmp,
                     (int32_t *)list, {(uint64_t *)kv0, (uint64_t *)kv1}, {rec0, rec1}, sws};
    return o;
}

template <typename T>
int mdf(const ot_tree *t, T *field, const T *pos, const T *target, int64_t n, int n_iter, T dt, T rho, int mode,
        T *f_lag, T *f_eul, void *work, hipStream_t s)
{
    const int64_t m_pts = 3 * n, m_leaves = 3 * t->n_leaves;
    MdfWork w;
    mdf_layout(n, t->n_leaves, sizeof(T), (char *)work, &w);
    T *fk = (T *)w.fk;   // (n, 3): u_k, then F_k
    T *f = (T *)w.f;     // (n_leaves, 3): this iteration's spread force (ATOMIC)
    if (f_lag) hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(m_pts)), dim3(256), 0, s, f_lag, m_pts, T(0));
    if (f_eul) hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(m_leaves)), dim3(256), 0, s, f_eul, m_leaves, T(0));
    if (n_iter == 0 || n == 0) {
        OT_HIP(hipGetLastError());
        return OT_OK;
    }
    const int dtype = sizeof(T) == 4 ? OT_F32 : OT_F64;
    // markers sorted by host leaf, once
    int shift, bits;
    point_sort_key_bits(t->n_leaves, shift, bits);
    PointSortBufs<T> sb{{w.kv[0], w.kv[1]}, {(T *)w.rec[0], (T *)w.rec[1]}, w.sws};
    PointSortResult<T> sr;
    point_sort<T>(t->view, n, t->n_leaves, shift, bits, pos, (const T *)nullptr, (int32_t *)nullptr, sb,
                  (unsigned long long *)nullptr, s, sr);
    const uint64_t *kv = sr.kv;
    pos = sr.rec;   // sorted positions, (n, 3)
    T *tg = (T *)w.tg;
    hipLaunchKernelGGL(k_gather_rows<T>, dim3(grid_for(m_pts)), dim3(256), 0, s, m_pts, target, kv, tg);
    // leaves the markers reach, once
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(t->n_leaves)), dim3(256), 0, s, w.flags, t->n_leaves, 0u);
    const dim3 gm((unsigned)((n + 255) / 256));
    if (t->view.periodic) hipLaunchKernelGGL((k_mark<T, true>), gm, dim3(256), 0, s, t->view, n, pos, w.flags);
    else hipLaunchKernelGGL((k_mark<T, false>), gm, dim3(256), 0, s, t->view, n, pos, w.flags);
    exclusive_scan(w.flags, w.offs, t->n_leaves, w.tmp, s);
    hipLaunchKernelGGL(k_compact, dim3(grid_for(t->n_leaves)), dim3(256), 0, s, w.flags, w.offs, t->n_leaves, w.list,
                       w.count);
    OT_HIP(hipGetLastError());
    // listed leaves at most min(n_leaves, 27 n): the grid covers them
    const unsigned gl = grid_for(std::min<int64_t>(t->n_leaves, 27 * n));
    FxState *fx = (FxState *)t->scratch;
    const bool fixed = mode == OT_SPREAD_FIXED;
    // the sums start cleared; each update clears them (and max |F|) again
    if (fixed) {
        hipLaunchKernelGGL(k_clear_listed<unsigned long long>, dim3(gl), dim3(256), 0, s, w.list, w.count, t->fx_acc);
        hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(1), dim3(64), 0, s, &fx->maxbits, (int64_t)1, 0ull);
    } else {
        hipLaunchKernelGGL(k_clear_listed<T>, dim3(gl), dim3(256), 0, s, w.list, w.count, f);
    }
    for (int it = 0; it < n_iter; ++it) {
        int rc = track(t, kOpInterp, field, nullptr, pos, dtype, n, OT_SPREAD_ATOMIC, 0, nullptr, fk, nullptr, s);
        if (rc) return rc;
        hipLaunchKernelGGL(k_mdf_force<T>, dim3(grid_for(m_pts)), dim3(256), 0, s, m_pts, (const T *)tg, fk, kv, f_lag,
                           dt, fixed ? &fx->maxbits : (unsigned long long *)nullptr);
        if (fixed) {
            hipLaunchKernelGGL(k_fx_prepare<T>, dim3(1), dim3(64), 0, s, fx, n);
            if ((rc = spread_kernel(t, dtype, mode, fk, pos, n, nullptr, s))) return rc;
            hipLaunchKernelGGL((k_mdf_update_listed<T, true>), dim3(gl), dim3(256), 0, s, w.list, w.count, field,
                               (T *)nullptr, t->fx_acc, fx, f_eul, rho);
        } else {
            if ((rc = spread_kernel(t, dtype, mode, fk, pos, n, f, s))) return rc;
            hipLaunchKernelGGL((k_mdf_update_listed<T, false>), dim3(gl), dim3(256), 0, s, w.list, w.count, field, f,
                               (unsigned long long *)nullptr, (FxState *)nullptr, f_eul, rho);
        }
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
    if (n > (int64_t)INT32_MAX) return fail(OT_ERR_CAPACITY, "ot_mdf: at most 2^31 - 1 markers");
    hipStream_t s = (hipStream_t)stream;
    if (dtype == OT_F32)
        return mdf<float>(tree, (float *)field, (const float *)pos, (const float *)target, n, n_iter, (float)dt,
                          (float)rho, mode, (float *)force_lag, (float *)force_eul, work, s);
    return mdf<double>(tree, (double *)field, (const double *)pos, (const double *)target, n, n_iter, dt, rho, mode,
                       (double *)force_lag, (double *)force_eul, work, s);
}
