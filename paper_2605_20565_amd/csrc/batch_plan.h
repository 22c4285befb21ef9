// State of a batched plan (ot_batch_plan), shared by the plan's host code
// (batch.hip) and its kernels' enqueue sequence (batch_kernels.h).
#pragma once

#include <hip/hip_runtime.h>

#include <stdint.h>

#include "ot_common.h"

struct ot_batch_plan {
    const ot_tree *tree;
    int dtype, mode;
    int block, tile, grid;
    int ops_union;
    int64_t n_points, n_tiles;
    int64_t *tile_start;      // device
    uint32_t *tile_info;      // device: count | ops << 24
    unsigned *counter;        // device
    hipStream_t capture_stream;
    bool use_graph;           // OT_TUNE_GRAPH: runs replay a captured graph
    bool have_graph;
    hipGraph_t graph;
    hipGraphExec_t exec;
    const void *key[7];
    bool timing;              // record ev[0]/ev[1] around the persistent kernel
    hipEvent_t ev[2];
    // point sorting (OT_TUNE_SORT_POINTS)
    bool sort_points;
    int sort_bits, sort_shift;
    int ops_all;              // the common ops of every instance
    bool grad_plan;           // instances carry OT_OP_GRAD_POS
    bool small_table;         // tiles of at most kSmallTile points: the small spreading table
    uint64_t *skv[2];         // host's leaf entry << 32 | input index, in sorted order
    void *srec[2];            // position (+ force) records in sorted order
    void *sws;                // counting workspace
    void *fxws;               // fixed-point spreading workspace (FIXED plans that spread)
    // host-major pass (sorted forward plans with OT_TUNE_HOST_MAJOR)
    bool use_hm;
    int hm_grid;
    int64_t n_win;            // windows of kHmThreads sorted points
    uint32_t *fb_list;        // device: windows handed to the per-point pass
};

namespace ot {
constexpr uint32_t kCountMask = 0x00FFFFFFu;   // tile_info: point count in the low 24 bits
}  // namespace ot
