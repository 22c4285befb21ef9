// Per-body sums of the IBM coupling (Sec. 2.3, fully resolved bodies): for
// each body b, a contiguous segment of points k,
//     S_b = sum_k v_k dV_k,   M_b = sum_k (X_k - x_b) x v_k dV_k,
// the force and torque on the body up to sign when v are the marker forces,
// or the enclosed fluid's linear and angular momentum when v is the velocity
// at points inside the body.  One workgroup per body; every thread sums a
// fixed stride of the segment in FP64 and the workgroup combines the partial
// sums in a fixed tree order, so the result does not depend on scheduling.
#include <hip/hip_runtime.h>

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

}  // namespace
}  // namespace ot

using namespace ot;

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
