// Per-body sums of the IBM coupling (Sec. 2.3, fully resolved bodies): for
// each body b, a contiguous segment of points k,
//     S_b = sum_k v_k dV_k,   M_b = sum_k (X_k - x_b) x v_k dV_k,
// the force and torque on the body up to sign when v are the marker forces,
// or the enclosed fluid's linear and angular momentum when v is the velocity
// at points inside the body.  One workgroup per body; every thread sums a
// fixed stride of the segment in FP64 and the workgroup combines the partial
// sums in a fixed tree order, so the result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ot_common.h"

namespace ot {
namespace {

constexpr int kThreads = 256;

template <typename T>
__global__ __launch_bounds__(kThreads) void k_body_sums(const T *__restrict__ vec, const T *__restrict__ pos,
                                                        const int64_t *__restrict__ offsets, int64_t n,
                                                        const T *__restrict__ centres, const T *__restrict__ dv,
                                                        double dv_all, int periodic, double *__restrict__ S,
                                                        double *__restrict__ M)
{
    __shared__ double part[6][kThreads];
    const int b = blockIdx.x;
    // clamp the segment to the points that exist
    const int64_t lo = min(max(offsets[b], (int64_t)0), n);
    const int64_t hi = min(max(offsets[b + 1], lo), n);
    const double c[3] = {(double)centres[3 * b], (double)centres[3 * b + 1], (double)centres[3 * b + 2]};
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t k = lo + threadIdx.x; k < hi; k += kThreads) {
        double r[3], v[3];
        const double w = dv ? (double)dv[k] : dv_all;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            r[d] = (double)pos[3 * k + d] - c[d];
            if (periodic) r[d] -= floor(r[d] + 0.5);   // nearest periodic image
            v[d] = (double)vec[3 * k + d] * w;
        }
        acc[0] += v[0];
        acc[1] += v[1];
        acc[2] += v[2];
        acc[3] += r[1] * v[2] - r[2] * v[1];
        acc[4] += r[2] * v[0] - r[0] * v[2];
        acc[5] += r[0] * v[1] - r[1] * v[0];
    }
#pragma unroll
    for (int j = 0; j < 6; ++j) part[j][threadIdx.x] = acc[j];
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
#pragma unroll
            for (int j = 0; j < 6; ++j) part[j][threadIdx.x] += part[j][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x < 3) {
        S[3 * b + threadIdx.x] = part[threadIdx.x][0];
        M[3 * b + threadIdx.x] = part[3 + threadIdx.x][0];
    }
}

// Domain average of a leaf field (Sec. 5.2: the IBM forcing's mean over the
// periodic box is removed every step): mean = sum_j f_j 2^(-3 l_j) over the
// unit cube.  A fixed grid of kMeanBlocks workgroups takes fixed contiguous
// leaf ranges, every thread a fixed stride of its range, and the partial
// sums combine in a fixed tree order, so the result is the same bits on
// every run.  The products f_j 2^(-3 l_j) are exact in FP64.
constexpr int kMeanBlocks = 512;

template <typename T>
__global__ __launch_bounds__(kThreads) void k_mean_partial(const T *__restrict__ f, const uint8_t *__restrict__ levels,
                                                           int64_t n, double *__restrict__ part)
{
    __shared__ double sh[3][kThreads];
    const int64_t lo = n * blockIdx.x / kMeanBlocks, hi = n * (blockIdx.x + 1) / kMeanBlocks;
    double a[3] = {0.0, 0.0, 0.0};
    for (int64_t j = lo + threadIdx.x; j < hi; j += kThreads) {
        const int e = -3 * (int)levels[j];
#pragma unroll
        for (int c = 0; c < 3; ++c) a[c] += ldexp((double)f[3 * j + c], e);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] = a[c];
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
#pragma unroll
            for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x < 3) part[3 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(kMeanBlocks) void k_mean_finish(const double *__restrict__ part, double *__restrict__ mean)
{
    __shared__ double sh[3][kMeanBlocks];
#pragma unroll
    for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] = part[3 * threadIdx.x + c];
    __syncthreads();
    for (int h = kMeanBlocks / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
#pragma unroll
            for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x < 3) mean[threadIdx.x] = sh[threadIdx.x][0];
}

// f_j - mean, formed in FP64 and rounded once to the field's precision.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_subtract_mean(T *__restrict__ f, int64_t n3,
                                                            const double *__restrict__ mean)
{
    const double m[3] = {mean[0], mean[1], mean[2]};
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n3; i += (int64_t)gridDim.x * kThreads)
        f[i] = (T)((double)f[i] - m[i % 3]);
}

}  // namespace
}  // namespace ot

using namespace ot;

extern "C" int64_t ot_force_mean_workspace_bytes(void)
{
    return (int64_t)kMeanBlocks * 3 * 8;
}

extern "C" int ot_force_mean(const ot_tree *t, void *field, int32_t dtype, int32_t subtract, double *mean_out,
                             void *work, void *stream)
{
    if (!t) return fail(OT_ERR_INVALID, "tree is NULL");
    if (dtype != OT_F32 && dtype != OT_F64) return fail(OT_ERR_INVALID, "dtype must be OT_F32 or OT_F64");
    if (!field || !mean_out) return fail(OT_ERR_INVALID, "ot_force_mean: field or mean_out is NULL");
    if ((uintptr_t)work & 7u) return fail(OT_ERR_INVALID, "ot_force_mean: work must be 8-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    void *owned = nullptr;
    if (!work) {
        if (hipMallocAsync(&owned, (size_t)ot_force_mean_workspace_bytes(), s) != hipSuccess) {
            (void)hipGetLastError();
            return fail(OT_ERR_OOM, "ot_force_mean: workspace");
        }
        work = owned;
    }
    const int64_t n = t->n_leaves;
    double *part = (double *)work;
    if (dtype == OT_F32)
        hipLaunchKernelGGL(k_mean_partial<float>, dim3(kMeanBlocks), dim3(kThreads), 0, s, (const float *)field,
                           t->levels, n, part);
    else
        hipLaunchKernelGGL(k_mean_partial<double>, dim3(kMeanBlocks), dim3(kThreads), 0, s, (const double *)field,
                           t->levels, n, part);
    hipLaunchKernelGGL(k_mean_finish, dim3(1), dim3(kMeanBlocks), 0, s, (const double *)part, mean_out);
    if (subtract) {
        const unsigned gb = (unsigned)std::min<int64_t>((3 * n + kThreads - 1) / kThreads, 8192);
        if (dtype == OT_F32)
            hipLaunchKernelGGL(k_subtract_mean<float>, dim3(gb), dim3(kThreads), 0, s, (float *)field, 3 * n,
                               (const double *)mean_out);
        else
            hipLaunchKernelGGL(k_subtract_mean<double>, dim3(gb), dim3(kThreads), 0, s, (double *)field, 3 * n,
                               (const double *)mean_out);
    }
    const hipError_t e = hipGetLastError();
    if (owned) (void)hipFreeAsync(owned, s);
    if (e != hipSuccess) return hip_fail(e, "ot_force_mean");
    return OT_OK;
}

extern "C" int ot_body_sums(const void *vec, const void *pos, int64_t n, const int64_t *offsets, int32_t n_body,
                            const void *centres, const void *dv, double dv_all, int32_t dtype, int32_t periodic,
                            double *sum_out, double *moment_out, void *stream)
{
    if (dtype != OT_F32 && dtype != OT_F64) return fail(OT_ERR_INVALID, "dtype must be OT_F32 or OT_F64");
    if (n < 0 || n_body < 0) return fail(OT_ERR_INVALID, "ot_body_sums: n and n_body must be >= 0");
    if (n_body == 0) return OT_OK;
    if (!offsets || !centres || !sum_out || !moment_out || (n > 0 && (!vec || !pos)))
        return fail(OT_ERR_INVALID, "ot_body_sums: NULL array");
    hipStream_t s = (hipStream_t)stream;
    if (dtype == OT_F32)
        hipLaunchKernelGGL(k_body_sums<float>, dim3((unsigned)n_body), dim3(kThreads), 0, s, (const float *)vec,
                           (const float *)pos, offsets, n, (const float *)centres, (const float *)dv, dv_all,
                           periodic ? 1 : 0, sum_out, moment_out);
    else
        hipLaunchKernelGGL(k_body_sums<double>, dim3((unsigned)n_body), dim3(kThreads), 0, s, (const double *)vec,
                           (const double *)pos, offsets, n, (const double *)centres, (const double *)dv, dv_all,
                           periodic ? 1 : 0, sum_out, moment_out);
    OT_HIP(hipGetLastError());
    return OT_OK;
}
