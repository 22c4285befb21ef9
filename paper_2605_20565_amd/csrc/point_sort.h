// Sorting a batched run's points by host leaf (point_sort.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ot_common.h"

namespace ot {

// Two sets of buffers the passes alternate between (set 1 after the first
// pass, set 0 after the second), plus the counting workspace.
template <typename T>
struct PointSortBufs {
    uint32_t *key[2];
    int32_t *val[2];
    T *pos[2];
    T *force[2];   // may be null when no forces are carried
    void *ws;      // point_sort_ws_bytes(n)
};

template <typename T>
struct PointSortResult {
    const uint32_t *host;  // host leaf id per sorted position (n_leaves: none)
    const int32_t *perm;   // sorted position -> input index
    const T *pos;          // positions in sorted order
    const T *force;        // forces in sorted order (null if not carried)
};

int64_t point_sort_ws_bytes(int64_t n);

// Keys (host leaf ids; points without a host get n_leaves), ids when
// ids != null, then ceil(bits / 8) stable passes over key bits
// [shift, shift + bits).  bits >= 1.
template <typename T>
void point_sort(const TreeView &tv, int64_t n, int64_t n_leaves, int shift, int bits, const T *pos, const T *force,
                int32_t *ids, PointSortBufs<T> &b, hipStream_t s, PointSortResult<T> &out);

}  // namespace ot
