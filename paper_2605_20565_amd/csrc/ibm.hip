// Multi-direct forcing of the immersed-boundary method (IBM subsection of
// Sec. 2.2): per iteration, interpolate the leaf velocity to the markers,
// form the marker force from the slip against the prescribed marker
// velocity, spread it back to the leaves and correct the leaf velocity.
// The interpolation and spreading are the library's own (any spreading mode);
// the two elementwise steps are small kernels here.  Everything is enqueued
// on the caller's stream; the caller provides the workspace.
#include <hip/hip_runtime.h>

#include "ot_common.h"
#include "track_device.h"

namespace ot {
int track(const ot_tree *t, int ops, const void *field, const void *force, const void *pos, int dtype, int64_t n,
          int mode, int accumulate, int32_t *ids, void *vel, void *fout, hipStream_t s);

namespace {

// buf holds the interpolated marker velocity u_k on entry and the marker
// force F_k = (U_k - u_k) / dt on exit; f_lag (nullable) accumulates F_k.
template <typename T>
__global__ __launch_bounds__(256) void k_mdf_force(int64_t m, const T *__restrict__ target, T *__restrict__ buf,
                                                   T *__restrict__ f_lag, T dt)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const T F = (target[i] - buf[i]) / dt;
        buf[i] = F;
        if (f_lag) f_lag[i] += F;
    }
}

// u += f / rho over all leaf components; f_eul (nullable) accumulates f.
template <typename T>
__global__ __launch_bounds__(256) void k_mdf_update(int64_t m, T *__restrict__ u, const T *__restrict__ f,
                                                    T *__restrict__ f_eul, T rho)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const T fi = f[i];
        u[i] += fi / rho;
        if (f_eul) f_eul[i] += fi;
    }
}

unsigned grid_for(int64_t m) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((m + 255) / 256, 4096)); }

template <typename T>
int mdf(const ot_tree *t, T *field, const T *pos, const T *target, int64_t n, int n_iter, T dt, T rho, int mode,
        T *f_lag, T *f_eul, T *work, hipStream_t s)
{
    const int64_t m_pts = 3 * n, m_leaves = 3 * t->n_leaves;
    T *fk = work;           // (n, 3): u_k, then F_k
    T *f = work + m_pts;    // (n_leaves, 3): this iteration's spread force
    if (f_lag) hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(m_pts)), dim3(256), 0, s, f_lag, m_pts, T(0));
    if (f_eul) hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(m_leaves)), dim3(256), 0, s, f_eul, m_leaves, T(0));
    const int dtype = sizeof(T) == 4 ? OT_F32 : OT_F64;
    for (int it = 0; it < n_iter; ++it) {
        int rc = track(t, kOpInterp, field, nullptr, pos, dtype, n, OT_SPREAD_ATOMIC, 0, nullptr, fk, nullptr, s);
        if (rc) return rc;
        hipLaunchKernelGGL(k_mdf_force<T>, dim3(grid_for(m_pts)), dim3(256), 0, s, m_pts, target, fk, f_lag, dt);
        rc = track(t, kOpSpread, nullptr, fk, pos, dtype, n, mode, 0, nullptr, nullptr, f, s);
        if (rc) return rc;
        hipLaunchKernelGGL(k_mdf_update<T>, dim3(grid_for(m_leaves)), dim3(256), 0, s, m_leaves, field,
                           (const T *)f, f_eul, rho);
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
    return (3 * n + 3 * tree->n_leaves) * (dtype == OT_F32 ? 4 : 8);
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
    hipStream_t s = (hipStream_t)stream;
    if (dtype == OT_F32)
        return mdf<float>(tree, (float *)field, (const float *)pos, (const float *)target, n, n_iter, (float)dt,
                          (float)rho, mode, (float *)force_lag, (float *)force_eul, (float *)work, s);
    return mdf<double>(tree, (double *)field, (const double *)pos, (const double *)target, n, n_iter, dt, rho, mode,
                       (double *)force_lag, (double *)force_eul, (double *)work, s);
}
