// Host-major pass over host-sorted points.
//
// The batched step visits the points sorted by host leaf.  Points that share
// a host share all 27 stencil nodes (Sec. 2.2: the stencil is the 3x3x3
// block of host-level cells around the host), so the node lookups, the
// field values and the spreading targets can be taken once per host instead
// of once per point.  A workgroup takes a window of consecutive sorted
// points and:
//   1. ranks the window's points by host id with a counting sort in LDS
//      (the global sort only groups them), giving runs of points with one
//      host ("runs");
//   2. finds every run's 27 node leaves (one descent-table lookup each) and
//      claims a slot per distinct leaf in a window hash table, loading the
//      leaf's field value there (a leaf that finds no free slot is used
//      straight from device memory instead);
//   3. interpolates: every thread sums its own point's 27 weights times the
//      slot values (same order and rounding as the per-point path);
//   4. spreads: 9-lane groups each take a contiguous chunk of the sorted
//      window, lane (oy, oz) holding the nodes (0..2, oy, oz) of the current
//      run in registers; at each run change the lanes add their sums to the
//      run's slots with one LDS atomic per node and component;
//   5. adds every slot to device memory once.
// Fixed-point contributions are the same rounded integers as on the
// per-point path (q = rint(w F 2^s) by one FP64 fma), summed exactly in
// int64, so both paths give the same bits.  A window whose hosts span too
// many ids or that holds too many runs is handed to the per-point pass (its
// index goes to a list).
#pragma once

#include <hip/hip_runtime.h>

#include "ot_common.h"
#include "track_device.h"

namespace ot {

constexpr int kHmThreads = 256;     // threads and points per window
constexpr int kHmProbe = 32;        // probes before a node leaf is used from device memory
constexpr int kHmMaxRuns = 128;     // distinct hosts per window
constexpr int kHmSpan = 512;        // host-id span of a window's counting sort
constexpr int kHmBatch = 7;         // node items per thread whose loads are issued together
constexpr int kHmGroupLanes = 9;    // lanes of a spreading group: (oy, oz)
constexpr int kHmGroupsPerWave = 64 / kHmGroupLanes;
constexpr int kHmGroups = kHmGroupsPerWave * (kHmThreads / 64);
// Node entries of a run: a table slot, a leaf used from device memory
// (kHmDirect | leaf), or a node dropped at a wall (kHmNoSlot).
constexpr uint32_t kHmNoSlot = 0xFFFFFFFFu;
constexpr uint32_t kHmDirect = 0x80000000u;

// Window table slots: a window of 256 sorted points reaches ~380 distinct
// node leaves on average on the 10^7-point workload (measured on the CPU
// over the same sort), so 1024 slots keep probe chains short.
template <typename T>
struct HmSlots { static constexpr int value = 1024; };
template <>
struct HmSlots<double> { static constexpr int value = 512; };

template <typename T, int MODE>
struct HmShared {
    using Acc = typename AccType<T, MODE>::type;
    static constexpr int S = HmSlots<T>::value;
    uint32_t key[S];                   // 0 = empty, else leaf + 1
    T u[S][3];                         // field value of the slot's leaf
    Acc acc[S][3];                     // spreading sums of the slot's leaf
    T w[kHmThreads][9];                // 1-D weights w[d][o] at 3 d + o, by sorted slot
    double fs[kHmThreads][3];          // FIXED: F 2^s; ATOMIC: F (exact in FP64), by sorted slot
    uint16_t run_of[kHmThreads];       // run of each sorted slot
    uint32_t rslot[kHmMaxRuns][27];    // node entries of each run (see kHmNoSlot, kHmDirect)
    uint32_t rent[kHmMaxRuns];         // host entry (level << 26 | id) of each run
    uint32_t rcell[kHmMaxRuns][3];     // host cell index at the host level
    uint32_t hist[kHmSpan];            // counting sort: counts, then packed prefix sums
    uint32_t red[2][kHmThreads / 64];  // block reductions
    unsigned tile;
};

// Exclusive scan of one value per thread over the workgroup (kHmThreads).
__device__ __forceinline__ uint32_t hm_exscan(uint32_t v, uint32_t *sh_w, uint32_t &total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh_w[wid] = x;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kHmThreads / 64; ++w) {
        const uint32_t s = sh_w[w];
        if (w < wid) pre += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return pre + x - v;
}

// Fixed point, summed as raw bit patterns: bits(fma(w, fs, 1.5 2^52)) is
// bits(1.5 2^52) + q for the rounded contribution q (see fx_round_fma), so a
// sum of m of them, taken modulo 2^64, is m bits(1.5 2^52) + sum q exactly.
__device__ __forceinline__ unsigned long long fx_bits(double w, double fs)
{
    return (unsigned long long)__double_as_longlong(fma(w, fs, 6755399441055744.0));
}
constexpr unsigned long long kFxMagicBits = 0x4338000000000000ull;   // bits of 1.5 * 2^52

// One node's sums of a run (cnt contributions per component) to its table
// slot, or to device memory when the node's leaf has no slot.
template <typename T, int MODE, typename Acc>
__device__ __forceinline__ void hm_add(Acc (*acc)[3], uint32_t s, const Acc (&a)[3], unsigned cnt, T *fout,
                                       unsigned long long *facc)
{
    if (s == kHmNoSlot) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Acc v = a[c];
        if constexpr (MODE == kModeFixed) v -= (unsigned long long)cnt * kFxMagicBits;
        if (s & kHmDirect) global_add<T, MODE>(fout, facc, 3 * (int64_t)(s & ~kHmDirect) + c, v);
        else atomicAdd(&acc[s][c], v);
    }
}

// OPS: kOpInterp and/or kOpSpread (host ids were written by the sort's key
// pass).  rec: sorted records, stride rs (position, then force).  Windows
// this pass cannot take go to fb_list[*fb_count].
template <typename T, int MODE, bool PER, int OPS>
__global__ __launch_bounds__(kHmThreads) void k_hm(TreeView tv, int64_t n, int64_t n_win,
                                                   unsigned *__restrict__ counter, const uint64_t *__restrict__ kv,
                                                   int rs, const T *__restrict__ rec, const T *__restrict__ field,
                                                   T *__restrict__ vel, T *__restrict__ fout,
                                                   unsigned long long *__restrict__ facc,
                                                   const FxState *__restrict__ fx, uint32_t *__restrict__ fb_list,
                                                   unsigned *__restrict__ fb_count)
{
    using Acc = typename AccType<T, MODE>::type;
    constexpr int kSlots = HmSlots<T>::value;
    __shared__ HmShared<T, MODE> sh;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    constexpr bool kInterp = (OPS & kOpInterp) != 0;
    constexpr bool kSpread = (OPS & kOpSpread) != 0;
    // the fixed-point state exists only for plans that spread
    const double scale = (kSpread && MODE == kModeFixed) ? fx->scale : 1.0;
    const int rsh = tv.L - tv.lev[0];

    for (int i = tid; i < kSlots; i += kHmThreads) {
        sh.key[i] = 0u;
        sh.acc[i][0] = Acc(0);
        sh.acc[i][1] = Acc(0);
        sh.acc[i][2] = Acc(0);
    }
    // This thread's point of window w (word, position, force).
    auto load_point = [&](int64_t w, uint64_t &wd, T (&Xp)[3], T (&Fp)[3]) {
        const int64_t kk = w * kHmThreads + tid;
        wd = 0ull;
        Xp[0] = Xp[1] = Xp[2] = T(0);
        Fp[0] = Fp[1] = Fp[2] = T(0);
        if (w < n_win && kk < n) {
            wd = kv[kk];
            Xp[0] = rec[(int64_t)rs * kk];
            Xp[1] = rec[(int64_t)rs * kk + 1];
            Xp[2] = rec[(int64_t)rs * kk + 2];
            if (kSpread) {
                Fp[0] = rec[(int64_t)rs * kk + 3];
                Fp[1] = rec[(int64_t)rs * kk + 4];
                Fp[2] = rec[(int64_t)rs * kk + 5];
            }
        }
    };
    // Static schedule: workgroups go round-robin over the 8 XCDs, and the
    // workgroups of XCD x take the windows of the x-th eighth of the sorted
    // points in turn, so neighbouring windows (which share node leaves)
    // meet in one L2.  Windows are equal in size, so no queue is needed.
    // The next window's points are loaded while the current one is
    // processed, so that those loads overlap it.
    const int G = (int)gridDim.x, g = (int)blockIdx.x;
    const int xcd = g & 7, xk = g >> 3;
    const int gx = (G - xcd + 7) >> 3;   // workgroups on this XCD
    const int64_t w_end = (n_win * (xcd + 1)) >> 3;
    int64_t win = ((n_win * xcd) >> 3) + xk;
    uint64_t nword;
    T nX[3], nF[3];
    load_point(win < w_end ? win : n_win, nword, nX, nF);
    for (;;) {
        if (win >= w_end) break;   // uniform
        const uint64_t word = nword;
        const T X[3] = {nX[0], nX[1], nX[2]};
        const T F[3] = {nF[0], nF[1], nF[2]};
        const int64_t nxt = win + gx;
        load_point(nxt < w_end ? nxt : n_win, nword, nX, nF);
        __syncthreads();   // orders the previous window's table clears
        const int64_t k = win * kHmThreads + tid;
        const bool have = k < n;
        do {   // one window; `break` hands it over or ends it

        // ---- 1. the window's points, their hosts and the counting sort
        uint32_t I[3];
        const uint32_t e = (uint32_t)(word >> 32);
        const uint32_t id = e & kIdMask;
        const bool ok = have && point_cell<T>(tv, X[0], X[1], X[2], I) && id < (uint32_t)tv.nleaf;
        uint32_t mn = ok ? id : 0xFFFFFFFFu, mx = ok ? id : 0u;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            mn = min(mn, (uint32_t)__shfl_xor(mn, o, 64));
            mx = max(mx, (uint32_t)__shfl_xor(mx, o, 64));
        }
        if (lane == 0) {
            sh.red[0][wid] = mn;
            sh.red[1][wid] = mx;
        }
        for (int i = tid; i < kHmSpan; i += kHmThreads) sh.hist[i] = 0u;
        __syncthreads();
#pragma unroll
        for (int w = 0; w < kHmThreads / 64; ++w) {
            mn = min(mn, sh.red[0][w]);
            mx = max(mx, sh.red[1][w]);
        }
        const bool any = mn <= mx;
        if (any && mx - mn >= (uint32_t)kHmSpan) {   // uniform: the span is the workgroup's
            if (tid == 0) fb_list[atomicAdd(fb_count, 1u)] = (uint32_t)win;
            break;
        }
        const uint32_t b = ok ? id - mn : 0u;
        const uint32_t rank = ok ? atomicAdd(&sh.hist[b], 1u) : 0u;
        __syncthreads();
        // packed exclusive prefix: low 16 bits = first sorted slot of the
        // host, high 16 bits = its run index
        constexpr int kPer = kHmSpan / kHmThreads;
        uint32_t hv[kPer];
        uint32_t loc = 0u;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            const uint32_t c = sh.hist[tid * kPer + j];
            hv[j] = c | (c ? 0x10000u : 0u);
            loc += hv[j];
        }
        uint32_t tot;
        uint32_t pre = hm_exscan(loc, sh.red[0], tot);
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            sh.hist[tid * kPer + j] = pre;
            pre += hv[j];
        }
        const int nruns = (int)(tot >> 16);
        const int nok = (int)(tot & 0xFFFFu);
        __syncthreads();
        if (nruns > kHmMaxRuns) {
            if (tid == 0) fb_list[atomicAdd(fb_count, 1u)] = (uint32_t)win;
            break;
        }
        const uint32_t pk = ok ? sh.hist[b] : 0u;
        const int slot = (int)(pk & 0xFFFFu) + (int)rank;
        const int run = (int)(pk >> 16);
        const int l = (int)((e >> kLevelShift) & 31u);
        T wt[3][3];
        if (ok) {
            const T sc = (T)(1 << l);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                T t, r;
                cell_offsets<T>(X[d] * sc, t, r);
                delta3<T>(t, r, wt[d]);
#pragma unroll
                for (int o = 0; o < 3; ++o) sh.w[slot][3 * d + o] = wt[d][o];
            }
            if (kSpread) {
#pragma unroll
                for (int c = 0; c < 3; ++c) sh.fs[slot][c] = (double)F[c] * scale;
            }
            sh.run_of[slot] = (uint16_t)run;
            if (rank == 0) {
                sh.rent[run] = e;
#pragma unroll
                for (int d = 0; d < 3; ++d) sh.rcell[run][d] = I[d] >> (tv.L - l);
            }
        }
        __syncthreads();

        // ---- 2. node leaves of every run, one table slot per distinct leaf.
        // A thread's items (run, node) are taken in batches whose table loads
        // are all issued before the first is used, and likewise the field
        // loads, so each batch waits for two memory round trips.
        for (int base = 0; base < nruns * 27; base += kHmThreads * kHmBatch) {
            uint32_t ent[kHmBatch], Nn[kHmBatch][3];
            bool valid[kHmBatch];
#pragma unroll
            for (int bb = 0; bb < kHmBatch; ++bb) {
                const int it = base + bb * kHmThreads + tid;
                valid[bb] = false;
                ent[bb] = 0u;
                Nn[bb][0] = Nn[bb][1] = Nn[bb][2] = 0u;
                if (it < nruns * 27) {
                    const int r = it / 27, q = it - 27 * r;
                    const uint32_t he = sh.rent[r];
                    const int hl = (int)((he >> kLevelShift) & 31u);
                    const int hs = tv.L - hl;
                    const int32_t Ml = 1 << hl;
                    const uint32_t half = hs > 0 ? (1u << (hs - 1)) : 0u;
                    const int od[3] = {q % 3, (q / 3) % 3, q / 9};
                    bool v = true;
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        int32_t nn = (int32_t)sh.rcell[r][d] + od[d] - 1;
                        if (PER) nn &= (Ml - 1);
                        else v = v && nn >= 0 && nn < Ml;
                        Nn[bb][d] = v ? (((uint32_t)nn << hs) | half) : 0u;
                    }
                    valid[bb] = v;
                    if (v) ent[bb] = q == 13 ? he : ld_table(tv, interleave3(Nn[bb][0] >> rsh, Nn[bb][1] >> rsh,
                                                                            Nn[bb][2] >> rsh));
                }
            }
            uint32_t sl[kHmBatch];
            bool fresh[kHmBatch];
#pragma unroll
            for (int bb = 0; bb < kHmBatch; ++bb) {
                sl[bb] = kHmNoSlot;
                fresh[bb] = false;
                if (!valid[bb]) continue;
                if (ent[bb] & kSplit) ent[bb] = descend_below_root(tv, ent[bb], Nn[bb][0], Nn[bb][1], Nn[bb][2]);
                const uint32_t leaf = ent[bb] & kIdMask;
                const uint32_t key = leaf + 1u;
                const uint32_t step = ((leaf * 0x9E3779B1u) >> 16) | 1u;
                uint32_t h = leaf & (kSlots - 1);
                sl[bb] = kHmDirect | leaf;   // unless a slot is found
                for (int p = 0; p < kHmProbe; ++p) {
                    const uint32_t old = atomicCAS(&sh.key[h], 0u, key);
                    if (old == 0u || old == key) {
                        sl[bb] = h;
                        fresh[bb] = old == 0u;
                        break;
                    }
                    h = (h + step) & (kSlots - 1);
                }
            }
            if (kInterp) {
                T uv[kHmBatch][3];
#pragma unroll
                for (int bb = 0; bb < kHmBatch; ++bb) {
                    if (fresh[bb]) {
                        const int64_t j = 3 * (int64_t)(ent[bb] & kIdMask);
                        uv[bb][0] = field[j];
                        uv[bb][1] = field[j + 1];
                        uv[bb][2] = field[j + 2];
                    }
                }
#pragma unroll
                for (int bb = 0; bb < kHmBatch; ++bb) {
                    if (fresh[bb]) {
                        sh.u[sl[bb]][0] = uv[bb][0];
                        sh.u[sl[bb]][1] = uv[bb][1];
                        sh.u[sl[bb]][2] = uv[bb][2];
                    }
                }
            }
#pragma unroll
            for (int bb = 0; bb < kHmBatch; ++bb) {
                const int it = base + bb * kHmThreads + tid;
                if (it < nruns * 27) sh.rslot[it / 27][it % 27] = sl[bb];
            }
        }
        __syncthreads();

        // ---- 3. interpolation of this thread's point
        if (kInterp && have) {
            T U[3] = {T(0), T(0), T(0)};
            if (ok) {
#pragma unroll
                for (int q = 0; q < 27; ++q) {
                    const int ox = q % 3, oy = (q / 3) % 3, oz = q / 9;
                    const uint32_t s = sh.rslot[run][q];
                    if (!PER && s == kHmNoSlot) continue;
                    const T wq = wt[0][ox] * wt[1][oy] * wt[2][oz];
                    T u0, u1, u2;
                    if (s & kHmDirect) {   // no table slot: the leaf's value from device memory
                        const int64_t jj = 3 * (int64_t)(s & ~kHmDirect);
                        u0 = field[jj];
                        u1 = field[jj + 1];
                        u2 = field[jj + 2];
                    } else {
                        u0 = sh.u[s][0];
                        u1 = sh.u[s][1];
                        u2 = sh.u[s][2];
                    }
                    U[0] = fma(wq, u0, U[0]);
                    U[1] = fma(wq, u1, U[1]);
                    U[2] = fma(wq, u2, U[2]);
                }
            }
            const int64_t kd = (int64_t)(uint32_t)word;
            vel[3 * kd] = U[0];
            vel[3 * kd + 1] = U[1];
            vel[3 * kd + 2] = U[2];
        }

        // ---- 4. spreading: group G takes sorted slots [lo, hi)
        if (kSpread) {
            const int g = lane / kHmGroupLanes;
            const int j9 = lane - kHmGroupLanes * g;
            const int oy = j9 % 3, oz = j9 / 3;
            if (g < kHmGroupsPerWave) {
                const int G = wid * kHmGroupsPerWave + g;
                const int lo = (G * nok) / kHmGroups, hi = ((G + 1) * nok) / kHmGroups;
                Acc a[3][3];
#pragma unroll
                for (int o = 0; o < 3; ++o) a[o][0] = a[o][1] = a[o][2] = Acc(0);
                unsigned cnt = 0u;
                int cur = -1;
                for (int j = lo; j < hi; ++j) {
                    const int r = sh.run_of[j];
                    if (r != cur) {
                        if (cur >= 0) {
#pragma unroll
                            for (int ox = 0; ox < 3; ++ox) {
                                hm_add<T, MODE>(sh.acc, sh.rslot[cur][ox + 3 * oy + 9 * oz], a[ox], cnt, fout, facc);
                                a[ox][0] = a[ox][1] = a[ox][2] = Acc(0);
                            }
                        }
                        cur = r;
                        cnt = 0u;
                    }
                    const T wy = sh.w[j][3 + oy], wz = sh.w[j][6 + oz];
                    const double f0 = sh.fs[j][0], f1 = sh.fs[j][1], f2 = sh.fs[j][2];
#pragma unroll
                    for (int ox = 0; ox < 3; ++ox) {
                        const double wd = (double)(sh.w[j][ox] * wy * wz);
                        if constexpr (MODE == kModeFixed) {
                            a[ox][0] += fx_bits(wd, f0);
                            a[ox][1] += fx_bits(wd, f1);
                            a[ox][2] += fx_bits(wd, f2);
                        } else {
                            a[ox][0] = fma(wd, f0, a[ox][0]);
                            a[ox][1] = fma(wd, f1, a[ox][1]);
                            a[ox][2] = fma(wd, f2, a[ox][2]);
                        }
                    }
                    ++cnt;
                }
                if (cur >= 0) {
#pragma unroll
                    for (int ox = 0; ox < 3; ++ox)
                        hm_add<T, MODE>(sh.acc, sh.rslot[cur][ox + 3 * oy + 9 * oz], a[ox], cnt, fout, facc);
                }
            }
        }
        __syncthreads();

        // ---- 5. every occupied slot to device memory once; clear the table
        for (int i = tid; i < kSlots; i += kHmThreads) {
            const uint32_t key = sh.key[i];
            if (key) {
                if (kSpread) {
                    const int64_t j = 3 * (int64_t)(key - 1u);
                    global_add<T, MODE>(fout, facc, j, sh.acc[i][0]);
                    global_add<T, MODE>(fout, facc, j + 1, sh.acc[i][1]);
                    global_add<T, MODE>(fout, facc, j + 2, sh.acc[i][2]);
                    sh.acc[i][0] = Acc(0);
                    sh.acc[i][1] = Acc(0);
                    sh.acc[i][2] = Acc(0);
                }
                sh.key[i] = 0u;
            }
        }
        } while (0);
        win = nxt;
    }
}

}  // namespace ot
