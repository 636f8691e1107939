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

// Scratch of the triad phases.  A server round that sets its own context on
// its thread (hgt_use_phase_ctx) runs its phases on it, so rounds with
// different contexts can overlap on the device; NULL restores the device's
// shared context.
struct PhaseCtx;
HGT_HIDDEN PhaseCtx* hgt_phase_ctx_create(int device);
HGT_HIDDEN void hgt_phase_ctx_destroy(PhaseCtx* c);
HGT_HIDDEN void hgt_use_phase_ctx(PhaseCtx* c);

// Host mirrors of the graph's size (valid while none of its batches is queued).
struct HgtSizes {
    uint32_t n_vertices, track_mask;
    uint64_t n_live, n_inc;
    int device;
};
HGT_HIDDEN HgtSizes hgt_sizes(hgt_graph* g);
