// Sorting a batched run's points by host leaf (point_sort.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdint.h>

#include "ot_common.h"

namespace ot {

// Two sets of buffers the passes alternate between (set 1 after the first
// pass, set 0 after the second), plus the counting workspace.
template <typename T>
struct PointSortBufs {
    uint64_t *kv[2];   // n words: host's leaf entry << 32 | input index
    T *rec[2];         // n records of 6 (position, force) or 3 (position) values
    void *ws;          // point_sort_ws_bytes(n)
};

template <typename T>
struct PointSortResult {
    const uint64_t *kv;   // per sorted position: host's leaf entry << 32 | input index
    const T *rec;         // per sorted position: stride values, position first
    int stride;           // 6 with forces, 3 without
};

int64_t point_sort_ws_bytes(int64_t n);

// Key bits [shift, shift + bits) to sort by for a tree of n_leaves leaves
// (keys run up to n_leaves): groups of at most 64 consecutive leaf ids, and
// all of the id when it has at most 16 bits.  Trees of up to 4 M leaves
// take two 8-bit passes, larger ones three (measured on 17 M and 20 M
// leaves: groups of 512 leaves left a tile's points spread over more leaves
// than the spreading table holds; 64 beat 8 and 2 as well).
inline void point_sort_key_bits(int64_t n_leaves, int &shift, int &bits)
{
    int all = 1;
    while ((int64_t(1) << all) <= n_leaves) ++all;
    shift = std::max(0, std::min(6, all - 16));
    bits = all - shift;
}

// Keys (the host's leaf entry, id in the low 26 bits; points without a
// host get n_leaves), ids when ids != null, then ceil(bits / 8) stable
// passes over id bits [shift, shift + bits); bits >= 1.  force != null: records carry forces
// too, and when maxbits != null the first pass also atomically maxes the
// bit pattern of max |F| (finite components) into maxbits[0] and sets
// maxbits[1] when a component is not finite.
template <typename T>
void point_sort(const TreeView &tv, int64_t n, int64_t n_leaves, int shift, int bits, const T *pos, const T *force,
                int32_t *ids, PointSortBufs<T> &b, unsigned long long *maxbits, hipStream_t s,
                PointSortResult<T> &out);

}  // namespace ot
