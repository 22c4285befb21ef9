// Point-particle step (Sec. 2.3, point-like particles), one thread per
// particle: host leaf, fluid velocity by trilinear interpolation at the host
// level (8 nodes, each read from the leaf containing the node's centre),
// Schiller-Naumann drag and buoyancy, second-order Adams-Bashforth with the
// host level's time step dt0 / 2^(l - l_min), and the host after the move.
// Physical units throughout: the paper's rescale of the previous acceleration
// when a particle changes level (a_c = 2 a_f in lattice units) is the unit
// change itself, so the previous acceleration carries over unchanged.
#include <hip/hip_runtime.h>

#include "ot_common.h"
#include "track_device.h"

namespace ot {
namespace {

template <typename T, bool PER>
__global__ __launch_bounds__(256) void k_particle_step(TreeView tv, int l_min, int64_t n, const T *__restrict__ field,
                                                       T *__restrict__ pos, T *__restrict__ vel,
                                                       T *__restrict__ vel_prev, T *__restrict__ acc_prev,
                                                       int32_t *__restrict__ ids, ot_particle_params p)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    const T X[3] = {pos[3 * k], pos[3 * k + 1], pos[3 * k + 2]};
    const T V[3] = {vel[3 * k], vel[3 * k + 1], vel[3 * k + 2]};
    const T Vp[3] = {vel_prev[3 * k], vel_prev[3 * k + 1], vel_prev[3 * k + 2]};
    const T Ap[3] = {acc_prev[3 * k], acc_prev[3 * k + 1], acc_prev[3 * k + 2]};
    uint32_t I[3];
    const bool ok = point_cell<T>(tv, X[0], X[1], X[2], I);
    T U[3] = {T(0), T(0), T(0)};
    double dt = 0.0;
    if (ok) {
        const uint32_t e = descend(tv, I[0], I[1], I[2]);
        const int l = (int)((e >> kLevelShift) & 31u);
        const int sh = tv.L - l;
        const int64_t M = int64_t(1) << l;
        const uint32_t half = sh > 0 ? (1u << (sh - 1)) : 0u;
        int64_t i0[3];
        T t[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double s = (double)X[d] * (double)M - 0.5;
            const double f = floor(s);
            i0[d] = (int64_t)f;
            t[d] = (T)(s - f);
        }
        // the 8 nodes: root-summary entries issued together, root entries
        // where the summary has no answer, the deeper descent only under
        // split root cells, then the gathers (independent loads instead of
        // one search after another)
        uint32_t nc[8][3];
        uint32_t ent[8], root[8], sm[8];
        T wq[8];
        uint32_t inside = 0u;
        const int rsh = tv.L - tv.lev[0];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int o[3] = {q & 1, (q >> 1) & 1, (q >> 2) & 1};
            bool in = true;
            T w = T(1);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                int64_t c = i0[d] + o[d];
                if (PER) c &= (M - 1);
                else in = in && c >= 0 && c < M;
                nc[q][d] = (uint32_t)(((c < 0 ? 0 : c) << sh) | half);
                w *= o[d] ? t[d] : T(1) - t[d];
            }
            wq[q] = w;
            inside |= (in ? 1u : 0u) << q;
            // a node outside the walls is dropped with its weight; its lookups
            // go to entry 0
            root[q] = in ? interleave3(nc[q][0] >> rsh, nc[q][1] >> rsh, nc[q][2] >> rsh) : 0u;
            sm[q] = tv.summary ? ld_summary(tv, root[q] >> 3) : kSplit;
        }
        // the root itself only where the summary has no answer
#pragma unroll
        for (int q = 0; q < 8; ++q) ent[q] = ld_table(tv, (sm[q] & kSplit) ? root[q] : 0u);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            if (!(sm[q] & kSplit)) ent[q] = sm[q] + (root[q] & 7u);
            if (!((inside >> q) & 1u)) ent[q] = 0u;
        }
        // the level-1 step of every split node at once, then deeper levels (rare)
        uint32_t e1[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) e1[q] = ld_table(tv, step1_index(tv, ent[q], nc[q][0], nc[q][1], nc[q][2]));
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            if (ent[q] & kSplit) ent[q] = e1[q];
            if (ent[q] & kSplit) ent[q] = descend_from_level2(tv, ent[q], nc[q][0], nc[q][1], nc[q][2]);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            if (!((inside >> q) & 1u)) continue;
            const int64_t j = 3 * (int64_t)(ent[q] & kIdMask);
            U[0] = fma(wq[q], field[j], U[0]);
            U[1] = fma(wq[q], field[j + 1], U[1]);
            U[2] = fma(wq[q], field[j + 2], U[2]);
        }
        dt = ldexp(p.dt0, -(l - l_min));
    }
    // drag (Schiller-Naumann) and buoyancy
    const T rel[3] = {U[0] - V[0], U[1] - V[1], U[2] - V[2]};
    const T mag = sqrt(rel[0] * rel[0] + rel[1] * rel[1] + rel[2] * rel[2]);
    const T re = (T)(2.0 * p.r_p / p.nu) * mag;
    const T fd = T(1) + T(0.15) * pow(re, T(0.687));
    const T inv_tau = (T)(9.0 * p.rho_f * p.nu / (2.0 * p.rho_p * p.r_p * p.r_p));
    const T buoy = (T)(1.0 - p.rho_f / p.rho_p);
    T A[3], Vn[3], Xn[3];
    const T h = (T)dt;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        A[d] = fd * rel[d] * inv_tau + buoy * (T)p.g[d];
        if (p.first) {
            Vn[d] = V[d] + h * A[d];
            Xn[d] = X[d] + h * V[d];
        } else {
            Vn[d] = V[d] + h * (T(1.5) * A[d] - T(0.5) * Ap[d]);
            Xn[d] = X[d] + h * (T(1.5) * V[d] - T(0.5) * Vp[d]);
        }
        if (PER) Xn[d] = Xn[d] - floor(Xn[d]);
    }
    uint32_t In[3];
    const bool okn = point_cell<T>(tv, Xn[0], Xn[1], Xn[2], In);
    ids[k] = okn ? (int32_t)(descend(tv, In[0], In[1], In[2]) & kIdMask) : -1;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        pos[3 * k + d] = Xn[d];
        vel[3 * k + d] = Vn[d];
        vel_prev[3 * k + d] = V[d];
        acc_prev[3 * k + d] = A[d];
    }
}

// Host ordering of point particles.  Sort key of each particle: its host
// leaf id, or n_leaves when it has none (those go last); value: its index.
template <typename T>
__global__ __launch_bounds__(256) void k_particle_keys(TreeView tv, int64_t n, const T *__restrict__ pos,
                                                       uint64_t *__restrict__ key, int32_t *__restrict__ val)
{
    const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= n) return;
    uint32_t I[3];
    const bool ok = point_cell<T>(tv, pos[3 * k], pos[3 * k + 1], pos[3 * k + 2], I);
    key[k] = ok ? (uint64_t)(descend(tv, I[0], I[1], I[2]) & kIdMask) : (uint64_t)tv.nleaf;
    val[k] = (int32_t)k;
}

// Row i of the outputs is input row src[i] of each state array.
template <typename T>
__global__ __launch_bounds__(256) void k_particle_gather(int64_t n, const uint64_t *__restrict__ key,
                                                         const int32_t *__restrict__ src, uint64_t nleaf,
                                                         const T *__restrict__ pos, const T *__restrict__ vel,
                                                         const T *__restrict__ vel_prev,
                                                         const T *__restrict__ acc_prev, T *__restrict__ pos_o,
                                                         T *__restrict__ vel_o, T *__restrict__ vel_prev_o,
                                                         T *__restrict__ acc_prev_o, int32_t *__restrict__ ids_o,
                                                         int32_t *__restrict__ perm_o)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t j = src[i];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        pos_o[3 * i + d] = pos[3 * j + d];
        vel_o[3 * i + d] = vel[3 * j + d];
        vel_prev_o[3 * i + d] = vel_prev[3 * j + d];
        acc_prev_o[3 * i + d] = acc_prev[3 * j + d];
    }
    if (ids_o) ids_o[i] = key[i] < nleaf ? (int32_t)key[i] : -1;
    if (perm_o) perm_o[i] = (int32_t)j;
}

// Workspace layout: two key and two value buffers, then the radix sort's.
int64_t psort_align(int64_t b) { return (b + 255) & ~int64_t(255); }

}  // namespace
}  // namespace ot

using namespace ot;

extern "C" int ot_particle_step(const ot_tree *t, const void *field, void *pos, void *vel, void *vel_prev,
                                void *acc_prev, int32_t *ids, int32_t dtype, int64_t n,
                                const ot_particle_params *params, void *stream)
{
    if (!t || !params) return fail(OT_ERR_INVALID, "ot_particle_step: tree or params is NULL");
    if (dtype != OT_F32 && dtype != OT_F64) return fail(OT_ERR_INVALID, "dtype must be OT_F32 or OT_F64");
    if (n < 0) return fail(OT_ERR_INVALID, "n < 0");
    if (n > 0 && (!field || !pos || !vel || !vel_prev || !acc_prev || !ids))
        return fail(OT_ERR_INVALID, "ot_particle_step: NULL array");
    const ot_particle_params &p = *params;
    if (!(p.dt0 >= 0.0) || !(p.r_p > 0.0) || !(p.rho_p > 0.0) || !(p.rho_f >= 0.0) || !(p.nu > 0.0))
        return fail(OT_ERR_INVALID, "ot_particle_step: need dt0 >= 0, r_p, rho_p, nu > 0, rho_f >= 0");
    if (n == 0) return OT_OK;
    const dim3 g((unsigned)((n + 255) / 256)), b(256);
    hipStream_t s = (hipStream_t)stream;
#define OT_PSTEP(TT, PERV)                                                                                      \
    hipLaunchKernelGGL((k_particle_step<TT, PERV>), g, b, 0, s, t->view, (int)t->l_min, n, (const TT *)field, \
                       (TT *)pos, (TT *)vel, (TT *)vel_prev, (TT *)acc_prev, ids, p)
    if (dtype == OT_F32) {
        if (t->view.periodic) OT_PSTEP(float, true);
        else OT_PSTEP(float, false);
    } else {
        if (t->view.periodic) OT_PSTEP(double, true);
        else OT_PSTEP(double, false);
    }
#undef OT_PSTEP
    OT_HIP(hipGetLastError());
    return OT_OK;
}

extern "C" int64_t ot_particle_sort_workspace_bytes(int64_t n)
{
    if (n < 0) n = 0;
    return 2 * psort_align(8 * n) + 2 * psort_align(4 * n) + psort_align(radix_ws_bytes(n));
}

extern "C" int ot_particle_sort(const ot_tree *t, int32_t dtype, int64_t n, const void *pos, const void *vel,
                                const void *vel_prev, const void *acc_prev, void *pos_out, void *vel_out,
                                void *vel_prev_out, void *acc_prev_out, int32_t *ids_out, int32_t *perm_out,
                                void *work, void *stream)
{
    if (!t) return fail(OT_ERR_INVALID, "ot_particle_sort: tree is NULL");
    if (dtype != OT_F32 && dtype != OT_F64) return fail(OT_ERR_INVALID, "dtype must be OT_F32 or OT_F64");
    if (n < 0 || n > INT32_MAX) return fail(OT_ERR_INVALID, "ot_particle_sort: need 0 <= n < 2^31");
    if (n > 0 && (!pos || !vel || !vel_prev || !acc_prev || !pos_out || !vel_out || !vel_prev_out || !acc_prev_out))
        return fail(OT_ERR_INVALID, "ot_particle_sort: NULL array");
    if ((uintptr_t)work & 255u) return fail(OT_ERR_INVALID, "ot_particle_sort: work must be 256-byte aligned");
    {
        const void *in[4] = {pos, vel, vel_prev, acc_prev};
        const void *out_[4] = {pos_out, vel_out, vel_prev_out, acc_prev_out};
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
                if (n > 0 && (out_[a] == in[b] || (a < b && out_[a] == out_[b])))
                    return fail(OT_ERR_INVALID, "ot_particle_sort: the output arrays must be distinct from each other "
                                                "and from the inputs");
    }
    if (n == 0) return OT_OK;
    hipStream_t s = (hipStream_t)stream;
    void *owned = nullptr;
    if (!work) {
        if (hipMallocAsync(&owned, (size_t)ot_particle_sort_workspace_bytes(n), s) != hipSuccess) {
            (void)hipGetLastError();
            return fail(OT_ERR_OOM, "ot_particle_sort: workspace");
        }
        work = owned;
    }
    char *w = (char *)work;
    uint64_t *k0 = (uint64_t *)w;
    uint64_t *k1 = (uint64_t *)(w + psort_align(8 * n));
    int32_t *v0 = (int32_t *)(w + 2 * psort_align(8 * n));
    int32_t *v1 = (int32_t *)(w + 2 * psort_align(8 * n) + psort_align(4 * n));
    void *rws = w + 2 * psort_align(8 * n) + 2 * psort_align(4 * n);
    // keys span 0 .. n_leaves (n_leaves: no host)
    int bits = 1;
    while (bits < 31 && ((int64_t)1 << bits) <= t->n_leaves) ++bits;
    const dim3 g((unsigned)((n + 255) / 256)), b(256);
    if (dtype == OT_F32)
        hipLaunchKernelGGL(k_particle_keys<float>, g, b, 0, s, t->view, n, (const float *)pos, k0, v0);
    else
        hipLaunchKernelGGL(k_particle_keys<double>, g, b, 0, s, t->view, n, (const double *)pos, k0, v0);
    uint64_t *ks = nullptr;
    int32_t *vs = nullptr;
    radix_sort_pairs(k0, v0, k1, v1, n, bits, rws, &ks, &vs, s);
#define OT_PGATHER(TT)                                                                                           \
    hipLaunchKernelGGL(k_particle_gather<TT>, g, b, 0, s, n, (const uint64_t *)ks, (const int32_t *)vs,          \
                       (uint64_t)t->n_leaves, (const TT *)pos, (const TT *)vel, (const TT *)vel_prev,            \
                       (const TT *)acc_prev, (TT *)pos_out, (TT *)vel_out, (TT *)vel_prev_out, (TT *)acc_prev_out, \
                       ids_out, perm_out)
    if (dtype == OT_F32) OT_PGATHER(float);
    else OT_PGATHER(double);
#undef OT_PGATHER
    hipError_t e = hipGetLastError();
    if (owned) (void)hipFreeAsync(owned, s);
    if (e != hipSuccess) return hip_fail(e, "ot_particle_sort");
    return OT_OK;
}
