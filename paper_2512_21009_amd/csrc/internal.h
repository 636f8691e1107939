// internal.h -- library-internal hooks between the graph code and the request
// server (not part of the C ABI; hidden symbols).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hgt.h"

#define HGT_HIDDEN __attribute__((visibility("hidden")))

// u64 words of the maintained counts: hyperedge [0, 30), incident-vertex
// [30, 33), temporal [33, 129)
constexpr int HGT_COUNT_WORDS = 129;

// Queues a copy of the graph's counts to dst (host, pinned, HGT_COUNT_WORDS words).
HGT_HIDDEN int hgt_counts_async(hgt_graph* g, uint64_t* dst, hipStream_t s);

// Host mirrors of the graph's size (valid while none of its batches is queued).
struct HgtSizes {
    uint32_t n_vertices, track_mask;
    uint64_t n_live, n_inc;
    int device;
};
HGT_HIDDEN HgtSizes hgt_sizes(hgt_graph* g);
