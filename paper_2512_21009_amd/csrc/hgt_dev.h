// hgt_dev.h -- device-side types and helpers shared by the library's HIP sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/hgt.h"

#define HGT_WG 256
#define HGT_WAVE 64
#define HGT_EMPTY 0xffffffffu

// Sticky per-graph scalars that live in device memory.
struct DevScalars {
    int32_t status;       // HGT_OK or the first error of the batch being applied
    uint32_t pad0;
    uint64_t next_id;     // IDs in use are < next_id
    uint64_t h_bump;      // words of the h2v pool handed out
    uint64_t v_bump;      // words of the v2h pool handed out
    uint64_t next_seq;    // arrival sequence of the next inserted hyperedge
    int64_t last_ts;      // largest timestamp inserted so far
    uint64_t n_live;
    uint64_t n_inc;       // sum of live cardinalities
};

// Summary of a batch's non-mutating planning pass, read back by the host once.
struct BatchSummary {
    int32_t status;
    uint32_t pad0;
    uint64_t del_members;   // sum |h| over deleted hyperedges
    uint64_t del_pairs2;    // sum C(|h|,2) over deleted hyperedges
    uint64_t ins_pairs2;    // sum C(|h|,2) over inserted hyperedges
    uint64_t n_free;        // |F|: free IDs including this batch's deletions
    uint64_t next_id_new;
    uint64_t h2v_need;      // words of new h2v blocks
    uint64_t v2h_need;      // words of new v2h blocks
    uint64_t n_touched;     // vertices whose incidence list changes
    uint64_t stage_words;   // old list words of touched vertices
    uint64_t max_lh_del;    // max over deleted h of sum_{u in h} deg(u) (old graph)
    uint64_t max_lh_ins;    // max over inserted h of sum_{u in h} deg(u) (new graph)
    uint64_t max_ins_card;
    uint64_t sum_lh_del;    // sum over deleted h of sum_{u in h} deg(u)
    uint64_t sum_lh_ins;    // sum over inserted h (new graph)
    uint64_t pad[1];
};

// Read-only view of the store used by the triad kernels.  Incidence lists
// (v2h) are ascending by ID; graphs that track temporal triads keep the
// timestamp of every list entry at the same index of v2h_ts, so a kernel can
// drop the entries outside a time window while it streams a list.
struct GraphView {
    const uint64_t* h_off;
    const uint32_t* h_len;
    const uint32_t* h2v;
    const uint64_t* v_off;
    const uint32_t* v_len;
    const uint32_t* v2h;
    const int64_t* h_ts;
    const uint64_t* h_seq;
    const int64_t* v2h_ts;  // NULL unless temporal is tracked
};

__device__ __forceinline__ void set_status(int32_t* st, int code) { atomicCAS(st, 0, code); }

__device__ __forceinline__ uint32_t hash_slot(uint32_t key, uint32_t log_cap) {
    return log_cap == 0 ? 0u : (uint32_t)((key * 2654435761u) >> (32 - log_cap));
}

__host__ __device__ __forceinline__ uint64_t pow2ceil64(uint64_t x) {
    if (x <= 1) return 1;
    x--;
    x |= x >> 1; x |= x >> 2; x |= x >> 4; x |= x >> 8; x |= x >> 16; x |= x >> 32;
    return x + 1;
}

__host__ __device__ __forceinline__ uint32_t log2u64(uint64_t x) {  // floor, x > 0
    uint32_t r = 0;
    while (x > 1) { x >>= 1; r++; }
    return r;
}

// lower_bound over a sorted u32 array
__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t* a, uint32_t n, uint32_t key) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ bool contains_u32(const uint32_t* a, uint32_t n, uint32_t key) {
    uint32_t p = lower_bound_u32(a, n, key);
    return p < n && a[p] == key;
}

// Whether the incidence list lst[0..n) (ascending IDs) holds hyperedge e.
__device__ __forceinline__ bool v2h_contains(const GraphView& g, const uint32_t* lst, uint32_t n, uint32_t e) {
    (void)g;
    return contains_u32(lst, n, e);
}

// t - d and t + d clamped to the int64 range (d >= 0)
__device__ __forceinline__ int64_t ts_sub(int64_t t, int64_t d) { return t < INT64_MIN + d ? INT64_MIN : t - d; }
__device__ __forceinline__ int64_t ts_add(int64_t t, int64_t d) { return t > INT64_MAX - d ? INT64_MAX : t + d; }

// index k with pre[k] <= pos < pre[k+1] over a non-decreasing array pre[0..n]
template <class T>
__device__ __forceinline__ uint32_t seg_of(const T* pre, uint32_t n, T pos) {
    uint32_t lo = 0, hi = n;  // answer in [0, n)
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= pos) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint64_t choose2(uint64_t n) { return n < 2 ? 0 : n * (n - 1) / 2; }
__device__ __forceinline__ uint64_t choose3(uint64_t n) { return n < 3 ? 0 : n * (n - 1) * (n - 2) / 6; }

// Epoch-tagged batch membership: mark = epoch << 32 | rank.
__device__ __forceinline__ bool lower_ranked_member(uint64_t mark, uint32_t epoch, uint32_t rank) {
    return (uint32_t)(mark >> 32) == epoch && (uint32_t)mark < rank;
}

// ---------------------------------------------------------------------------
// host-side primitive launchers (prims.hip)
// ---------------------------------------------------------------------------
// Exclusive scan of n u64 values (n read from n_dev when non-NULL, else n_max);
// out may alias in.  total (device, may be NULL) receives the sum.
void hgt_scan_u64(const uint64_t* in, uint64_t* out, uint64_t n_max, const uint64_t* n_dev,
                  uint64_t* total, void* tmp, hipStream_t s);
size_t hgt_scan_tmp_bytes(uint64_t n_max);

// Ascending LSD radix sort of u64 keys over bits [0, bits); n from n_dev or n_max.
// Result ends in keys (alt is scratch of the same size).
void hgt_radix_sort_u64(uint64_t* keys, uint64_t* alt, uint64_t n_max, const uint64_t* n_dev,
                        int bits, void* tmp, hipStream_t s);
size_t hgt_radix_tmp_bytes(uint64_t n_max);

void hgt_fill_u64(uint64_t* p, uint64_t v, uint64_t n, hipStream_t s);
void hgt_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);
