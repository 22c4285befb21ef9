// Per-point device code of the tracking step, shared by the plain launches
// and the batched persistent kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "ot_common.h"

namespace ot {

enum : int { kOpLocate = OT_OP_LOCATE, kOpInterp = OT_OP_INTERPOLATE, kOpSpread = OT_OP_SPREAD };
// Position gradient grad[k] = sum_n (force[k] . field[leaf(n)]) grad_X w_kn,
// gathered with the same node lookups as the interpolation.
enum : int { kOpGrad = OT_OP_GRAD_POS };
enum : int { kModeAtomic = OT_SPREAD_ATOMIC, kModeFixed = OT_SPREAD_FIXED };

// Fixed-point spreading state: the header of a spreading workspace (the
// caller's, or a batch plan's).
struct FxState {
    unsigned long long maxbits;   // bit pattern of max |F| (IEEE order == value order for >= 0)
    unsigned long long nonfinite; // != 0: some force component is NaN or infinite
    double scale;                 // 2^s
    double inv;                   // 2^-s
};

// A spreading workspace: header and n_leaves x 3 int64 accumulators.
struct FxWs {
    unsigned long long *acc;
    FxState *fx;
};

__device__ __forceinline__ void atomic_add(float *p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }


// Stencil of one point: host entry, 1-D weights, and per axis the three node
// cells' centre coordinates at the finest level (N) and their root-table
// digits already spread for Morton interleaving (R), so that the root index
// of node (ox, oy, oz) is R[0][ox] | R[1][oy] << 1 | R[2][oz] << 2.
template <typename T>
struct Stencil {
    T w[3][3];
    uint32_t N[3][3];
    uint32_t R[3][3];
    uint32_t valid;      // bit (d*3 + o) set when node o of axis d exists
    int level;
    uint32_t host;
};

template <typename T, bool PER>
__device__ __forceinline__ void make_stencil(const TreeView &tv, const T X[3], const uint32_t I[3], uint32_t e,
                                             Stencil<T> &st)
{
    const int l = (int)((e >> kLevelShift) & 31u);
    const int sh = tv.L - l;
    const int rs = tv.L - tv.lev[0];
    const int32_t Ml = 1 << l;
    const uint32_t half = sh > 0 ? (1u << (sh - 1)) : 0u;
    const T sc = (T)Ml;   // 2^l, exact
    st.level = l;
    st.host = e & kIdMask;
    st.valid = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        T t, r;
        cell_offsets<T>(X[d] * sc, t, r);
        delta3<T>(t, r, st.w[d]);
        const int32_t c = (int32_t)(I[d] >> sh);
#pragma unroll
        for (int o = 0; o < 3; ++o) {
            int32_t nn = c + o - 1;
            bool ok = true;
            if (PER) nn &= (Ml - 1);
            else ok = (nn >= 0) && (nn < Ml);
            if (!ok) nn = 0;   // dropped node: keep its coordinates inside the domain
            const uint32_t Nc = ((uint32_t)nn << sh) | half;
            st.N[d][o] = Nc;
            st.R[d][o] = part1by2(Nc >> rs);
            st.valid |= (ok ? 1u : 0u) << (d * 3 + o);
        }
    }
}

// ---------------------------------------------------------------------------
// Spreading sinks: where the contributions w F of one point go.
// ---------------------------------------------------------------------------
// Accumulator of one contribution and of the workgroup tables: int64 fixed
// point, or FP64 in ATOMIC mode for both precisions.  FP32 contributions
// are the exact FP64 products of their FP32 factors and are rounded to FP32
// once per table slot, at the device-memory add (LDS FP32 atomic adds run
// several times slower than 64-bit ones on this target).
template <typename T, int MODE>
struct AccType { using type = double; };
template <typename T>
struct AccType<T, kModeFixed> { using type = unsigned long long; };

// Fixed point: q = rint(w F 2^s), formed by one FP64 fused multiply-add
// fma(w, F 2^s, 1.5 * 2^52): the product is rounded once, together with the
// addition, and since |w F 2^s| <= 2^51 by the choice of s the sum lies in
// [2^52, 2^53), where the spacing is 1, so the rounding is to the nearest
// integer (ties to even), held in two's complement in the low mantissa bits.
// For FP32 inputs the product is exact, so q is exactly rint of the exact
// value w F 2^s.  fs = (double)F * 2^s is exact and formed once per point.
__device__ __forceinline__ unsigned long long fx_round_fma(double w, double fs)
{
    const double magic = 6755399441055744.0;   // 1.5 * 2^52
    return (unsigned long long)(__double_as_longlong(fma(w, fs, magic)) - __double_as_longlong(magic));
}

template <typename T, int MODE>
__device__ __forceinline__ typename AccType<T, MODE>::type to_acc(T w, T f, double scale)
{
    if constexpr (MODE == kModeFixed) return fx_round_fma((double)w, (double)f * scale);
    else return (double)w * (double)f;
}

// Device-memory adds of the sinks, through global-address-space pointers
// (the sinks hold fout/facc in structs, where the compiler would emit flat
// atomics, which also count against the LDS counter).
template <typename T, int MODE>
__device__ __forceinline__ void global_add(T *fout, unsigned long long *facc, int64_t j,
                                           typename AccType<T, MODE>::type v)
{
    if constexpr (MODE == kModeFixed)
        __hip_atomic_fetch_add((__attribute__((address_space(1))) unsigned long long *)(facc + j), v, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    else
        __hip_atomic_fetch_add((__attribute__((address_space(1))) T *)(fout + j), (T)v, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
}

// Straight to device memory with one atomic per component.
template <typename T, int MODE>
struct DirectSink {
    T *fout;
    unsigned long long *facc;
    double scale;
    __device__ __forceinline__ void add(uint32_t leaf, T w, const T F[3])
    {
        const int64_t j = 3 * (int64_t)leaf;
#pragma unroll
        for (int c = 0; c < 3; ++c) global_add<T, MODE>(fout, facc, j + c, to_acc<T, MODE>(w, F[c], scale));
    }

    // All 27 stencil nodes of one point; bit q of live: node q exists.
    __device__ __forceinline__ void add27(const uint32_t (&ent)[27], uint32_t live, const T (&w)[3][3], const T F[3],
                                          const uint32_t (&)[3][3], int)
    {
#pragma unroll
        for (int q = 0; q < 27; ++q)
            if ((live >> q) & 1u) add(ent[q] & kIdMask, w[0][q % 3] * w[1][(q / 3) % 3] * w[2][q / 9], F);
    }
};

// Workgroup-local aggregation: an open-addressing table in LDS keyed by leaf
// id accumulates the contributions of all points the workgroup handles;
// flush() adds each occupied slot to device memory once.  The first probe is
// the primary slot (primary(): a root-level leaf's Morton index mod S, else
// id mod S), so the flush's atomics come in runs of neighbouring addresses;
// on a collision the probe moves by an odd stride hashed from the id (double
// hashing), because a workgroup's ids come in runs of consecutive Morton
// ranks that would otherwise pile up into long occupied clusters.  A
// contribution that finds no slot within kProbe steps goes straight to
// device memory.  In FIXED mode every value is the same rounded integer
// either way, so the result does not depend on the path.
template <typename T, int MODE, int S>
struct LdsSink {
    using Acc = typename AccType<T, MODE>::type;
    static constexpr int kProbe = 8;
    static constexpr int kVals = 3 * S;
    uint32_t *keys;     // S, 0 = empty, else leaf + 1
    Acc *vals;          // kVals
    T *fout;
    unsigned long long *facc;
    double scale;

    __device__ __forceinline__ void clear()
    {
        for (int i = threadIdx.x; i < S; i += blockDim.x) {
            keys[i] = 0u;
            vals[3 * i] = Acc(0);
            vals[3 * i + 1] = Acc(0);
            vals[3 * i + 2] = Acc(0);
        }
    }

    // Primary slot of a node leaf (entry e = level << 26 | id).  A leaf at
    // the root table's level is a root cell, and its Morton index there
    // (root: the index its root lookup used) mod S gives all root cells of a
    // 16 x 16 x 8 box distinct slots; other leaves take id mod S.  Ids are
    // ranks, shifted by every refined cell before them in Morton order, so
    // the ids of one tile's runs of root-level leaves can meet mod S where
    // their Morton indices do not.  Within a run of root-level leaves both
    // give neighbouring leaves neighbouring slots.
    static __device__ __forceinline__ uint32_t primary(uint32_t e, uint32_t root, int lev0)
    {
        return (((e >> kLevelShift) & 31u) == (uint32_t)lev0 ? root : e) & (S - 1);
    }

    // Slots after the primary one (double hashing); device memory when none
    // is free within kProbe steps.
    __device__ __forceinline__ void add_probing(uint32_t leaf, uint32_t slot, Acc a0, Acc a1, Acc a2)
    {
        const uint32_t key = leaf + 1u;
        const uint32_t step = ((leaf * 0x9E3779B1u) >> 16) | 1u;
        bool found = false;
#pragma unroll 1
        for (int p = 1; p < kProbe; ++p) {
            slot = (slot + step) & (S - 1);
            uint32_t cur = keys[slot];
            if (cur == 0u) {
                cur = atomicCAS(&keys[slot], 0u, key);
                if (cur == 0u) cur = key;
            }
            if (cur == key) {
                found = true;
                break;
            }
        }
        if (found) {
            atomicAdd(&vals[3 * slot], a0);
            atomicAdd(&vals[3 * slot + 1], a1);
            atomicAdd(&vals[3 * slot + 2], a2);
        } else {
            const int64_t j = 3 * (int64_t)leaf;
            global_add<T, MODE>(fout, facc, j, a0);
            global_add<T, MODE>(fout, facc, j + 1, a1);
            global_add<T, MODE>(fout, facc, j + 2, a2);
        }
    }

    // All 27 stencil nodes of one point; bit q of live: node q exists; R:
    // the stencil's spread root-level digits, lev0 the root table's level.
    // Every node first claims or finds its primary slot with one
    // compare-and-swap (0 -> key; a slot holding the key is left as it is);
    // the 27 swaps are independent, so they are in flight together instead
    // of a chain of LDS round trips per node.  Keys are only removed by
    // flush(), after a barrier, so a slot that reads as this key stays this
    // key's.  A node whose primary slot holds another key probes further.
    __device__ __forceinline__ void add27(const uint32_t (&ent)[27], uint32_t live, const T (&w)[3][3], const T F[3],
                                          const uint32_t (&R)[3][3], int lev0)
    {
        uint32_t hit = 0u;
#pragma unroll
        for (int q = 0; q < 27; ++q) {
            if ((live >> q) & 1u) {
                const uint32_t leaf = ent[q] & kIdMask;
                const uint32_t slot = primary(ent[q], R[0][q % 3] | (R[1][(q / 3) % 3] << 1) | (R[2][q / 9] << 2), lev0);
                const uint32_t old = atomicCAS(&keys[slot], 0u, leaf + 1u);
                hit |= (uint32_t)(old == 0u || old == leaf + 1u) << q;
            }
        }
#pragma unroll
        for (int q = 0; q < 27; ++q) {
            if (!((live >> q) & 1u)) continue;
            const uint32_t leaf = ent[q] & kIdMask;
            const T wq = w[0][q % 3] * w[1][(q / 3) % 3] * w[2][q / 9];
            const Acc a0 = to_acc<T, MODE>(wq, F[0], scale);
            const Acc a1 = to_acc<T, MODE>(wq, F[1], scale);
            const Acc a2 = to_acc<T, MODE>(wq, F[2], scale);
            const uint32_t slot = primary(ent[q], R[0][q % 3] | (R[1][(q / 3) % 3] << 1) | (R[2][q / 9] << 2), lev0);
            if ((hit >> q) & 1u) {
                atomicAdd(&vals[3 * slot], a0);
                atomicAdd(&vals[3 * slot + 1], a1);
                atomicAdd(&vals[3 * slot + 2], a2);
            } else {
                add_probing(leaf, slot, a0, a1, a2);
            }
        }
    }

    // All threads of the workgroup; leaves the table empty.  Value e of the
    // table (slot e / 3, component e % 3) goes to lane e of the sweep, so the
    // three components of a slot are added by neighbouring lanes of one
    // instruction: a run of neighbouring leaves becomes one contiguous span
    // of device memory per instruction, not three strided ones.  The keys
    // are cleared after a barrier, once every lane has read its slot's key.
    __device__ __forceinline__ void flush()
    {
        __syncthreads();
        for (int e = threadIdx.x; e < kVals; e += blockDim.x) {
            const uint32_t i = (uint32_t)e / 3u;
            const uint32_t key = keys[i];
            if (key) {
                global_add<T, MODE>(fout, facc, 3 * (int64_t)(key - 1u) + (int64_t)(e - 3 * (int)i), vals[e]);
                vals[e] = Acc(0);
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < S; i += blockDim.x) keys[i] = 0u;
        __syncthreads();
    }
};

// Table entry (level << 26 | id) of a host given by its leaf id; ids
// outside [0, n_leaves) give no host.
__device__ __forceinline__ bool host_from_id(const TreeView &tv, int32_t h, uint32_t &e)
{
    const bool ok = h >= 0 && h < tv.nleaf;
    e = ok ? (((uint32_t)tv.levels[h] << kLevelShift) | (uint32_t)h) : 0u;
    return ok;
}

// Point k: position X (loaded by the caller from pos[rs k + 0..2]), force
// force[rs k + 0..2] (rs = 3 for the caller's arrays, the record stride for
// sorted records).  For sorted points, word is the point's sort word (the
// host's leaf entry << 32 | input index): the host comes from the word,
// found by the sort's key pass on the same position, and the per-point
// outputs go to the input index.  Otherwise the host is hid[k] when the
// caller gives host ids (Algorithm 1's host_cell_id; -1 or an id out of
// range: no host), else the table descent finds it.  With kOpGrad, force[k]
// is also the vector the gradient contracts the field with, and the
// gradient goes to grad.
template <typename T, int OPS, bool PER, typename Sink>
__device__ __forceinline__ void track_point_at(const TreeView &tv, int64_t k, bool sorted, uint64_t word,
                                               const T (&X)[3], int rs, const T *__restrict__ field,
                                               const T *__restrict__ force, int32_t *__restrict__ ids,
                                               T *__restrict__ vel, Sink &sink, T *__restrict__ grad,
                                               const int32_t *__restrict__ hid, const T *Fpre = nullptr)
{
    const int64_t kd = sorted ? (int64_t)(uint32_t)word : k;
    const int64_t kp = (int64_t)rs * k;
    uint32_t I[3];
    bool ok = point_cell<T>(tv, X[0], X[1], X[2], I);
    uint32_t e = 0u;
    if (sorted) e = (uint32_t)(word >> 32);
    else if (hid) ok = host_from_id(tv, hid[k], e) && ok;
    else if (ok) e = descend(tv, I[0], I[1], I[2]);
    if (!ok) e = 0u;
    if (OPS & kOpLocate) ids[kd] = ok ? (int32_t)(e & kIdMask) : -1;
    if (!(OPS & (kOpInterp | kOpSpread | kOpGrad))) return;

    T U[3] = {T(0), T(0), T(0)};
    T G[3] = {T(0), T(0), T(0)};
    if (ok) {
        Stencil<T> st;
        make_stencil<T, PER>(tv, X, I, e, st);
        // phase 1: root-table entries of the 27 nodes (independent loads);
        // nodes dropped at a non-periodic wall are not looked up
        // All 26 loads are issued before any result is used (a node dropped
        // at a wall loads entry 0 and is then zeroed): the scheduler had
        // interleaved their uses and waited after every eight.
        uint32_t ent[27];
#pragma unroll
        for (int q = 0; q < 27; ++q) {
            const int ox = q % 3, oy = (q / 3) % 3, oz = q / 9;
            if (q == 13) continue;
            const uint32_t need = (1u << ox) | (1u << (3 + oy)) | (1u << (6 + oz));
            const bool use = PER || (st.valid & need) == need;
            ent[q] = ld_table(tv, use ? (st.R[0][ox] | (st.R[1][oy] << 1) | (st.R[2][oz] << 2)) : 0u);
        }
        __builtin_amdgcn_sched_barrier(0);
        ent[13] = st.host | ((uint32_t)st.level << kLevelShift);
        if (!PER) {
#pragma unroll
            for (int q = 0; q < 27; ++q) {
                const int ox = q % 3, oy = (q / 3) % 3, oz = q / 9;
                const uint32_t need = (1u << ox) | (1u << (3 + oy)) | (1u << (6 + oz));
                if (q != 13 && (st.valid & need) != need) ent[q] = 0u;
            }
        }
        // phase 2: nodes inside split root cells continue the descent, the
        // level-1 step of all of them at once
        uint32_t any = 0u;
#pragma unroll
        for (int q = 0; q < 27; ++q) any |= ent[q];
        if (any & kSplit) {
            uint32_t sub[27];
#pragma unroll
            for (int q = 0; q < 27; ++q) {
                const int ox = q % 3, oy = (q / 3) % 3, oz = q / 9;
                sub[q] = ld_table(tv, step1_index(tv, ent[q], st.N[0][ox], st.N[1][oy], st.N[2][oz]));
            }
            __builtin_amdgcn_sched_barrier(0);
            any = 0u;
#pragma unroll
            for (int q = 0; q < 27; ++q) {
                if (ent[q] & kSplit) ent[q] = sub[q];
                any |= ent[q];
            }
            if (any & kSplit) {   // trees more than 3 levels below the root
#pragma unroll
                for (int q = 0; q < 27; ++q) {
                    if (ent[q] & kSplit) {
                        const int ox = q % 3, oy = (q / 3) % 3, oz = q / 9;
                        ent[q] = descend_from_level2(tv, ent[q], st.N[0][ox], st.N[1][oy], st.N[2][oz]);
                    }
                }
            }
        }
        // phase 3: field gathers (interpolation and/or the gradient)
        if (OPS & (kOpInterp | kOpGrad)) {
            // gradient: dw/dX_d = 2^l phi'(r_d) prod_{e != d} phi(r_e)
            T dw[3][3];
            T v[3] = {T(0), T(0), T(0)};
            if (OPS & kOpGrad) {
                const T sc = (T)(1 << st.level);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    T t, r, wtmp[3];
                    cell_offsets<T>(X[d] * sc, t, r);
                    delta3_grad<T>(t, r, wtmp, dw[d]);
#pragma unroll
                    for (int o = 0; o < 3; ++o) dw[d][o] *= sc;
                    v[d] = Fpre ? Fpre[d] : force[kp + d];
                }
            }
            // the gathers are issued in batches of kB rows (FP32: 14 and 13;
            // FP64, whose rows take twice the registers: three of 9), each
            // loaded before any of its rows is used (the scheduler had kept
            // about six in flight); a node dropped at a wall has entry 0 and
            // loads row 0
            constexpr int kB = sizeof(T) == 4 ? 14 : 9;
#pragma unroll
            for (int b = 0; b < (27 + kB - 1) / kB; ++b) {
                const int q0 = b * kB, nq = 27 - q0 < kB ? 27 - q0 : kB;
                T fr[kB][3];
#pragma unroll
                for (int i = 0; i < kB; ++i) {
                    if (i >= nq) break;
                    const int64_t j = 3 * (int64_t)(ent[q0 + i] & kIdMask);
                    fr[i][0] = field[j];
                    fr[i][1] = field[j + 1];
                    fr[i][2] = field[j + 2];
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int i = 0; i < kB; ++i) {
                    if (i >= nq) break;
                    const int q = q0 + i;
                    const int ox = q % 3, oy = (q / 3) % 3, oz = q / 9;
                    const uint32_t need = (1u << ox) | (1u << (3 + oy)) | (1u << (6 + oz));
                    if (!PER && (st.valid & need) != need) continue;
                    const T f0 = fr[i][0], f1 = fr[i][1], f2 = fr[i][2];
                    if (OPS & kOpInterp) {
                        const T w = st.w[0][ox] * st.w[1][oy] * st.w[2][oz];
                        U[0] = fma(w, f0, U[0]);
                        U[1] = fma(w, f1, U[1]);
                        U[2] = fma(w, f2, U[2]);
                    }
                    if (OPS & kOpGrad) {
                        const T dot = fma(v[0], f0, fma(v[1], f1, v[2] * f2));
                        G[0] = fma(dot * dw[0][ox], st.w[1][oy] * st.w[2][oz], G[0]);
                        G[1] = fma(dot * st.w[0][ox], dw[1][oy] * st.w[2][oz], G[1]);
                        G[2] = fma(dot * st.w[0][ox], st.w[1][oy] * dw[2][oz], G[2]);
                    }
                }
            }
        }
        // phase 4: spreading
        if (OPS & kOpSpread) {
            // finish the gathers first: without the barrier the compiler may
            // sink the interpolation sums below the spreading and keep all
            // 27 gathered values alive through it
            if (OPS & kOpInterp) asm volatile("" : "+v"(U[0]), "+v"(U[1]), "+v"(U[2]));
            if (OPS & kOpGrad) asm volatile("" : "+v"(G[0]), "+v"(G[1]), "+v"(G[2]));
            const T F[3] = {Fpre ? Fpre[0] : force[kp], Fpre ? Fpre[1] : force[kp + 1],
                            Fpre ? Fpre[2] : force[kp + 2]};
            uint32_t live = (1u << 27) - 1u;
            if (!PER) {
#pragma unroll
                for (int q = 0; q < 27; ++q) {
                    const int ox = q % 3, oy = (q / 3) % 3, oz = q / 9;
                    const uint32_t need = (1u << ox) | (1u << (3 + oy)) | (1u << (6 + oz));
                    if ((st.valid & need) != need) live &= ~(1u << q);
                }
            }
            sink.add27(ent, live, st.w, F, st.R, tv.lev[0]);
        }
    }
    if (OPS & kOpInterp) {
        vel[3 * kd] = U[0];
        vel[3 * kd + 1] = U[1];
        vel[3 * kd + 2] = U[2];
    }
    if (OPS & kOpGrad) {
        grad[3 * kd] = G[0];
        grad[3 * kd + 1] = G[1];
        grad[3 * kd + 2] = G[2];
    }
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
// order like the values, so an integer max is exact and order independent)
// into out[0], and out[1] != 0 when some component is not finite.  One
// atomic per workgroup: same-address atomics serialise.
template <typename T>
__global__ __launch_bounds__(256) void k_maxabs(const T *__restrict__ f, int64_t m, unsigned long long *__restrict__ out)
{
    __shared__ unsigned long long wmax[4];
    unsigned long long best = 0;
    bool bad = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const T v = f[i];
        if (isfinite(v)) best = std::max(best, abs_bits(v));
        else bad = true;
    }
    if (bad) atomicOr(out + 1, 1ull);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) best = std::max(best, (unsigned long long)__shfl_xor(best, o, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) best = std::max(best, wmax[w]);
        if (best) atomicMax(out, best);
    }
}

template <typename T>
__device__ __forceinline__ double bits_value(unsigned long long b);
template <>
__device__ __forceinline__ double bits_value<float>(unsigned long long b) { return (double)__uint_as_float((unsigned)b); }
template <>
__device__ __forceinline__ double bits_value<double>(unsigned long long b) { return __longlong_as_double((long long)b); }

// s = min(62 - E, 51 - Ef) with n max|F| <= 2^E and max|F| <= 2^Ef: every
// leaf sum stays below 2^62 in magnitude (weights are >= 0 and one point's
// weights sum to 1) and every single contribution below 2^51.
template <typename T>
__device__ __forceinline__ int fx_shift(unsigned long long maxbits, int64_t n)
{
    const double mf = bits_value<T>(maxbits);
    int s = 0;
    if (mf > 0.0 && n > 0) {
        int E, Ef;
        (void)frexp((double)n * mf, &E);
        (void)frexp(mf, &Ef);
        s = min(62 - E, 51 - Ef);
    }
    return s;
}

template <typename T>
__global__ void k_fx_prepare(FxState *fx, int64_t n)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int s = fx_shift<T>(fx->maxbits, n);
    fx->scale = ldexp(1.0, s);
    fx->inv = ldexp(1.0, -s);
}

// Accumulators to field_out.  A non-finite force cannot be carried by the
// integer sums, so when one was seen every output value becomes NaN.
template <typename T>
__global__ void k_fx_finalize(const unsigned long long *__restrict__ acc, T *__restrict__ out, int64_t n3,
                              const FxState *__restrict__ fx, int accumulate)
{
    const double inv = fx->inv;
    const bool poison = fx->nonfinite != 0ull;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n3; i += (int64_t)gridDim.x * blockDim.x) {
        const T v = poison ? T(NAN) : (T)((double)(long long)acc[i] * inv);
        out[i] = accumulate ? out[i] + v : v;
    }
}

// Point k, loading its sort word (kv non-null) and position first.
template <typename T, int OPS, bool PER, typename Sink>
__device__ __forceinline__ void track_point(const TreeView &tv, int64_t k, const uint64_t *__restrict__ kv, int rs,
                                            const T *__restrict__ pos, const T *__restrict__ field,
                                            const T *__restrict__ force, int32_t *__restrict__ ids,
                                            T *__restrict__ vel, Sink &sink, T *__restrict__ grad = nullptr,
                                            const int32_t *__restrict__ hid = nullptr)
{
    const uint64_t word = kv ? kv[k] : 0ull;
    const int64_t kp = (int64_t)rs * k;
    const T X[3] = {pos[kp], pos[kp + 1], pos[kp + 2]};
    track_point_at<T, OPS, PER, Sink>(tv, k, kv != nullptr, word, X, rs, field, force, ids, vel, sink, grad, hid);
}

// Process points [start, end) of one tile with all threads of the workgroup.
template <typename T, int OPS, bool PER, typename Sink>
__device__ __forceinline__ void track_range(const TreeView &tv, int64_t start, int64_t end,
                                            const uint64_t *__restrict__ kv, int rs, const T *__restrict__ pos,
                                            const T *__restrict__ field, const T *__restrict__ force,
                                            int32_t *__restrict__ ids, T *__restrict__ vel, Sink &sink,
                                            T *__restrict__ grad = nullptr, const int32_t *__restrict__ hid = nullptr)
{
    if (!kv) {
        for (int64_t k = start + threadIdx.x; k < end; k += blockDim.x)
            track_point<T, OPS, PER, Sink>(tv, k, kv, rs, pos, field, force, ids, vel, sink, grad, hid);
        return;
    }
    // sorted records: the next point's word, position and force are loaded
    // before this point's work, so they arrive while it runs
    constexpr bool kF = (OPS & (kOpSpread | kOpGrad)) != 0;
    int64_t k = start + threadIdx.x;
    if (k >= end) return;
    uint64_t w = kv[k];
    T X[3] = {pos[(int64_t)rs * k], pos[(int64_t)rs * k + 1], pos[(int64_t)rs * k + 2]};
    T F[3] = {T(0), T(0), T(0)};
    if (kF) {
        F[0] = force[(int64_t)rs * k];
        F[1] = force[(int64_t)rs * k + 1];
        F[2] = force[(int64_t)rs * k + 2];
    }
    for (;;) {
        const int64_t kn = k + blockDim.x;
        const bool more = kn < end;
        // unconditional loads (the last point reloads itself): a load
        // inside a branch is waited for where the branch joins, which had
        // made the prefetch wait before the current point's work
        const int64_t kc = more ? kn : k;
        const uint64_t wn = kv[kc];
        T Xn[3], Fn[3];
        Xn[0] = pos[(int64_t)rs * kc];
        Xn[1] = pos[(int64_t)rs * kc + 1];
        Xn[2] = pos[(int64_t)rs * kc + 2];
        if (kF) {
            Fn[0] = force[(int64_t)rs * kc];
            Fn[1] = force[(int64_t)rs * kc + 1];
            Fn[2] = force[(int64_t)rs * kc + 2];
        }
        track_point_at<T, OPS, PER, Sink>(tv, k, true, w, X, rs, field, force, ids, vel, sink, grad, nullptr,
                                          kF ? F : nullptr);
        if (!more) break;
        k = kn;
        w = wn;
        X[0] = Xn[0];
        X[1] = Xn[1];
        X[2] = Xn[2];
        if (kF) {
            F[0] = Fn[0];
            F[1] = Fn[1];
            F[2] = Fn[2];
        }
    }
}

// LDS table size of the aggregating sink (every slot holds 3 x 8 bytes).
template <typename T, int MODE>
struct SinkSlots { static constexpr int value = 2048; };

// Tiles of at most kSmallTile points spread through a table of kSmallSlots
// slots (14 KiB instead of 56 KiB of LDS): such launches are many small
// workgroups whose time is latency, and the large table would hold the CU
// to two of them (measured on 11 k points: 76 -> 63 us per fused launch;
// tiles of 128 bubble markers already reach more leaves than 512 slots).
constexpr int64_t kSmallTile = 64;
constexpr int kSmallSlots = 512;

// Host side of spreading (track.hip): clear the target (ATOMIC overwrite) or
// the workspace's accumulators, take the fixed-point scale (max |F| over
// `force` unless the caller already maxed it into ws.fx), and convert the
// accumulators into field_out.
// counters (optional): 32-bit words to zero in the same launch (a batch plan's).
int spread_begin(const ot_tree *t, const FxWs &ws, int dtype, int mode, int accumulate, void *fout, hipStream_t s,
                 unsigned *counters = nullptr, int64_t n_counters = 0);
int spread_scale(const ot_tree *t, const FxWs &ws, int dtype, int mode, const void *force, int64_t n, hipStream_t s);
int spread_epilogue(const ot_tree *t, const FxWs &ws, int dtype, int mode, int accumulate, void *fout, hipStream_t s);
FxWs fx_ws(void *work);

}  // namespace ot
