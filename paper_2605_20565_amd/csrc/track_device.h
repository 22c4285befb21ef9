// Per-point device code of the tracking step, shared by the plain launches
// and the batched persistent kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "ot_common.h"

namespace ot {

enum : int { kOpLocate = OT_OP_LOCATE, kOpInterp = OT_OP_INTERPOLATE, kOpSpread = OT_OP_SPREAD };
enum : int { kModeAtomic = OT_SPREAD_ATOMIC, kModeFixed = OT_SPREAD_FIXED };

// Fixed-point spreading state (lives in the tree's scratch buffer).
struct FxState {
    unsigned long long maxbits;   // bit pattern of max |F| (IEEE order == value order for >= 0)
    double scale;                 // 2^s
    double inv;                   // 2^-s
    unsigned long long pad;
};

__device__ __forceinline__ void atomic_add(float *p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }

// Stencil of one point: host entry, 1-D weights and the node-centre integer
// coordinates (finest level) of the three node cells per axis.
template <typename T>
struct Stencil {
    T w[3][3];
    uint32_t N[3][3];
    uint32_t valid;      // bit (d*3 + o) set when node o of axis d exists
    int level;
    uint32_t host;
};

template <typename T>
__device__ __forceinline__ void make_stencil(const TreeView &tv, const T X[3], const uint32_t I[3], uint32_t e,
                                             Stencil<T> &st)
{
    const int l = (int)((e >> kLevelShift) & 31u);
    const int sh = tv.L - l;
    const int32_t Ml = 1 << l;
    const uint32_t half = sh > 0 ? (1u << (sh - 1)) : 0u;
    const T sc = (T)Ml;   // 2^l, exact
    st.level = l;
    st.host = e & kIdMask;
    st.valid = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T s = X[d] * sc;
        delta3<T>(s - floor(s), st.w[d]);
        const int32_t c = (int32_t)(I[d] >> sh);
#pragma unroll
        for (int o = 0; o < 3; ++o) {
            int32_t nn = c + o - 1;
            bool ok = true;
            if (tv.periodic) nn &= (Ml - 1);
            else ok = (nn >= 0) && (nn < Ml);
            st.N[d][o] = ((uint32_t)nn << sh) | half;
            st.valid |= (ok ? 1u : 0u) << (d * 3 + o);
        }
    }
}

template <typename T, int OPS, int MODE>
__device__ __forceinline__ void track_point(const TreeView &tv, int64_t k, const T *__restrict__ pos,
                                            const T *__restrict__ field, const T *__restrict__ force,
                                            int32_t *__restrict__ ids, T *__restrict__ vel, T *__restrict__ fout,
                                            unsigned long long *__restrict__ facc, double fx_scale)
{
    const T X[3] = {pos[3 * k], pos[3 * k + 1], pos[3 * k + 2]};
    uint32_t I[3];
    const bool ok = point_cell<T>(tv, X[0], X[1], X[2], I);
    const uint32_t e = ok ? descend(tv, I[0], I[1], I[2]) : 0u;
    if (OPS & kOpLocate) ids[k] = ok ? (int32_t)(e & kIdMask) : -1;
    if (!(OPS & (kOpInterp | kOpSpread))) return;

    T U[3] = {T(0), T(0), T(0)};
    if (ok) {
        Stencil<T> st;
        make_stencil<T>(tv, X, I, e, st);
        T F[3] = {T(0), T(0), T(0)};
        if (OPS & kOpSpread) {
            F[0] = force[3 * k];
            F[1] = force[3 * k + 1];
            F[2] = force[3 * k + 2];
        }
#pragma unroll
        for (int oz = 0; oz < 3; ++oz) {
#pragma unroll
            for (int oy = 0; oy < 3; ++oy) {
                const T wyz = st.w[1][oy] * st.w[2][oz];
#pragma unroll
                for (int ox = 0; ox < 3; ++ox) {
                    const uint32_t need = (1u << ox) | (1u << (3 + oy)) | (1u << (6 + oz));
                    if ((st.valid & need) != need) continue;
                    uint32_t leaf;
                    if (ox == 1 && oy == 1 && oz == 1) leaf = st.host;   // the centre node lies in the host
                    else leaf = descend(tv, st.N[0][ox], st.N[1][oy], st.N[2][oz]) & kIdMask;
                    const T w = st.w[0][ox] * wyz;
                    const int64_t j = 3 * (int64_t)leaf;
                    if (OPS & kOpInterp) {
                        U[0] += w * field[j];
                        U[1] += w * field[j + 1];
                        U[2] += w * field[j + 2];
                    }
                    if (OPS & kOpSpread) {
                        if (MODE == kModeFixed) {
#pragma unroll
                            for (int c = 0; c < 3; ++c) {
                                const T v = w * F[c];
                                const long long q = __double2ll_rn((double)v * fx_scale);
                                atomicAdd(facc + j + c, (unsigned long long)q);
                            }
                        } else {
                            atomic_add(fout + j, w * F[0]);
                            atomic_add(fout + j + 1, w * F[1]);
                            atomic_add(fout + j + 2, w * F[2]);
                        }
                    }
                }
            }
        }
    }
    if (OPS & kOpInterp) {
        vel[3 * k] = U[0];
        vel[3 * k + 1] = U[1];
        vel[3 * k + 2] = U[2];
    }
}

// grad[k,d] = sum_n (vec_k . field[leaf(n)]) 2^l phi'(r_d) prod_{e!=d} phi(r_e)
template <typename T>
__device__ __forceinline__ void grad_point(const TreeView &tv, int64_t k, const T *__restrict__ pos,
                                           const T *__restrict__ field, const T *__restrict__ vec,
                                           T *__restrict__ grad)
{
    const T X[3] = {pos[3 * k], pos[3 * k + 1], pos[3 * k + 2]};
    uint32_t I[3];
    const bool ok = point_cell<T>(tv, X[0], X[1], X[2], I);
    T G[3] = {T(0), T(0), T(0)};
    if (ok) {
        const uint32_t e = descend(tv, I[0], I[1], I[2]);
        Stencil<T> st;
        make_stencil<T>(tv, X, I, e, st);
        T dw[3][3];
        const T sc = (T)(1 << st.level);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const T s = X[d] * sc;
            T wtmp[3];
            delta3_grad<T>(s - floor(s), wtmp, dw[d]);
#pragma unroll
            for (int o = 0; o < 3; ++o) dw[d][o] *= sc;
        }
        const T v0 = vec[3 * k], v1 = vec[3 * k + 1], v2 = vec[3 * k + 2];
#pragma unroll
        for (int oz = 0; oz < 3; ++oz) {
#pragma unroll
            for (int oy = 0; oy < 3; ++oy) {
#pragma unroll
                for (int ox = 0; ox < 3; ++ox) {
                    const uint32_t need = (1u << ox) | (1u << (3 + oy)) | (1u << (6 + oz));
                    if ((st.valid & need) != need) continue;
                    uint32_t leaf;
                    if (ox == 1 && oy == 1 && oz == 1) leaf = st.host;
                    else leaf = descend(tv, st.N[0][ox], st.N[1][oy], st.N[2][oz]) & kIdMask;
                    const int64_t j = 3 * (int64_t)leaf;
                    const T dot = v0 * field[j] + v1 * field[j + 1] + v2 * field[j + 2];
                    G[0] += dot * dw[0][ox] * st.w[1][oy] * st.w[2][oz];
                    G[1] += dot * st.w[0][ox] * dw[1][oy] * st.w[2][oz];
                    G[2] += dot * st.w[0][ox] * st.w[1][oy] * dw[2][oz];
                }
            }
        }
    }
    grad[3 * k] = G[0];
    grad[3 * k + 1] = G[1];
    grad[3 * k + 2] = G[2];
}

template <typename T>
__global__ void k_fill(T *p, int64_t n, T v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__device__ __forceinline__ unsigned long long abs_bits(float v)
{
    return (unsigned long long)(__float_as_uint(v) & 0x7FFFFFFFu);
}
__device__ __forceinline__ unsigned long long abs_bits(double v)
{
    return (unsigned long long)__double_as_longlong(v) & 0x7FFFFFFFFFFFFFFFull;
}

// max |F| over finite components (bit patterns of non-negative IEEE values
// order like the values, so an integer max is exact and order independent).
template <typename T>
__global__ void k_maxabs(const T *__restrict__ f, int64_t m, unsigned long long *__restrict__ out)
{
    unsigned long long best = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const T v = f[i];
        if (isfinite(v)) best = std::max(best, abs_bits(v));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) best = std::max(best, (unsigned long long)__shfl_xor(best, o, 64));
    if ((threadIdx.x & 63) == 0 && best) atomicMax(out, best);
}

template <typename T>
__device__ __forceinline__ double bits_value(unsigned long long b);
template <>
__device__ __forceinline__ double bits_value<float>(unsigned long long b) { return (double)__uint_as_float((unsigned)b); }
template <>
__device__ __forceinline__ double bits_value<double>(unsigned long long b) { return __longlong_as_double((long long)b); }

// s = 62 - E with n max|F| <= 2^E: every leaf sum stays below 2^62 in
// magnitude (weights are >= 0 and one point's weights sum to 1).
template <typename T>
__global__ void k_fx_prepare(FxState *fx, int64_t n)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double mf = bits_value<T>(fx->maxbits);
    int s = 0;
    if (mf > 0.0 && n > 0) {
        int E;
        (void)frexp((double)n * mf, &E);
        s = 62 - E;
    }
    fx->scale = ldexp(1.0, s);
    fx->inv = ldexp(1.0, -s);
}

template <typename T>
__global__ void k_fx_finalize(const unsigned long long *__restrict__ acc, T *__restrict__ out, int64_t n3,
                              const FxState *__restrict__ fx, int accumulate)
{
    const double inv = fx->inv;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n3; i += (int64_t)gridDim.x * blockDim.x) {
        const T v = (T)((double)(long long)acc[i] * inv);
        out[i] = accumulate ? out[i] + v : v;
    }
}

}  // namespace ot
