// triad.h -- launch interface of the triad-delta kernels.
#pragma once

#include "hgt_dev.h"

// Word offsets of the per-workgroup global tables of the large-centre kernel.
struct BigLayout {
    uint64_t nh_keys, nh_vals, hm, nl_x, nl_meta, warea, warea_words, words_per_wg;
};

// Per-graph inputs of one phase of the hyperedge/temporal kernels.  The
// kernels take an array of these, so one launch serves one graph or many.
struct HeGraph {
    GraphView g;
    const uint32_t* centres;  // changed hyperedge IDs; the index is the batch rank
    uint64_t n_centres;
    const uint64_t* mark;     // epoch-tagged batch rank per ID of this phase
    uint32_t epoch;
    uint32_t pad0;
    int64_t window;
    const int32_t* status;    // the graph's batch status: work is skipped unless 0
    uint64_t* out_he;         // u64[30] phase accumulators
    uint64_t* out_tmp;        // u64[96]
    uint32_t* hpool;          // neighbour histograms, 2 words per h2v word
    uint64_t id_base;         // first slot of this graph's IDs in the shared per-ID arrays
};

// The graphs of one launch: work item q belongs to the graph g with
// base[g] <= q < base[g+1] and is that graph's centre q - base[g].
struct Multi {
    const HeGraph* graphs;
    const uint64_t* base;     // n_graphs + 1 entries
    const uint64_t* id_base;  // n_graphs + 1 entries: graph g owns slots [id_base[g], id_base[g+1])
    uint32_t n_graphs;
    uint32_t pad0;
    uint64_t total;           // base[n_graphs]
    uint64_t total_ids;       // id_base[n_graphs]
};

__device__ __forceinline__ uint32_t multi_graph_of(const Multi& M, uint64_t q) {
    return M.n_graphs == 1 ? 0u : seg_of<uint64_t>(M.base, M.n_graphs, q);
}
__device__ __forceinline__ uint32_t multi_graph_of_id(const Multi& M, uint64_t slot) {
    return M.n_graphs == 1 ? 0u : seg_of<uint64_t>(M.id_base, M.n_graphs, slot);
}

// Deferred work items name their graph: graph << 32 | hyperedge ID.
__device__ __forceinline__ uint64_t item_of(uint32_t g, uint32_t h) { return ((uint64_t)g << 32) | h; }

struct TriadParams {
    Multi M;
    int do_he, do_tmp;
    const uint8_t* he_tab;    // [128] class index of a Venn code (255 = not a triad)
    const uint8_t* tmp_tab;   // [128]
    uint32_t* queue;          // work counters, cleared by the launcher
    uint32_t* big_queue;
    uint32_t* big_count;
    uint64_t* big_list;       // items deferred to the large kernel (capacity: all centres)
    uint32_t* big_rank;
    uint32_t* big_scratch;    // grid_big * big.words_per_wg words
    BigLayout big;
    uint32_t* wave_hash;      // per (workgroup, wave) 2-hop hash in global memory for neighbours
    uint32_t wave_slots;      // whose 2-hop list is too long for LDS: 2 * wave_slots words each
    uint64_t* stats;          // optional counters (see TriadStat), NULL = off
    int static_he;            // hyperedge family as a full count (see He2Params::static_mode)
    // Slices of the large kernel's centres (NULL: one per centre): a centre whose
    // members' lists hold many entries is shared by several workgroups, each
    // taking every S-th neighbour.  slice_pre[c] is the first slice of deferred
    // centre c (exclusive prefix); slice_pre[slice_cap] holds the number of
    // deferred centres, slice_pre[slice_cap + 1] the number of slices.
    uint64_t* slice_pre;
    uint64_t slice_cap;
    uint32_t slice_lh;        // member-list entries per slice (0: the default)
    void* slice_scan_tmp;     // hgt_scan_tmp_bytes(slice_cap)
};

// Counters accumulated by the triad kernels when TriadParams.stats is set.
constexpr int HE2_PHASES = 12;  // timed phases of a histogram-kernel stage
enum TriadStat {
    ST_BYTES_SMALL = 0,  // algorithmic bytes gathered by the small-centre kernel
    ST_BYTES_BIG = 1,    // ... by the large-centre kernel
    ST_DEFERRED = 2,     // centres moved to the large-centre kernel
    ST_WITNESS = 3,      // neighbours expanded through the binary-search path
    ST_EXPANDED = 4,     // neighbours expanded
    ST_IV_BYTES = 5,     // algorithmic bytes gathered by the incident-vertex kernel
    ST_DEFER0 = 6,       // centres moved on by histogram-kernel stage 0, 1, 2
    ST_HEB0 = 9,         // algorithmic bytes gathered by histogram-kernel stage 0, 1, 2
    ST_AGG_LONG = 12,    // aggregated pair phase: long runs counted by histogram
    ST_AGG_MULTI = 13,   // ... pairs sharing two or more vertices, corrected
    ST_AGG_ENUM = 14,    // centres whose pairs were enumerated per run instead
    ST_PH0 = 16,         // wall-clock ticks per phase of histogram-kernel stage s: ST_PH0 + HE2_PHASES s + phase
                         // (the last slot of a stage: the longest single centre, a maximum)
    ST_TMP0 = 56,        // the temporal launches' counters: ST_TMP0 + (ST_BYTES_SMALL .. ST_EXPANDED)
    ST_N = 64
};

BigLayout triad_big_layout(uint64_t max_lh, uint64_t max_card);
void triad_he_prepare(TriadParams& P, hipStream_t s);
void triad_he_launch_small(TriadParams& P, unsigned grid, hipStream_t s);
// After the small kernel: the slices of the deferred centres (when P.slice_pre is set).
void triad_he_slices(TriadParams& P, hipStream_t s);
void triad_he_launch_big(TriadParams& P, unsigned grid, hipStream_t s);

// hyperedge family through neighbour histograms (triad_he2.hip)
struct NbrParams {
    Multi M;
    int inserting;               // 1: rebuild the centres' histograms and add them to their neighbours'
    int emit_entries;            // 0: histograms only (build)
    uint64_t* n_entries;         // batch-neighbour entries written (all graphs)
    uint64_t entries_cap;
    uint32_t* ent_x;             // id_base + x
    uint32_t* ent_d;
    uint64_t* ent_pay;           // rank << 32 | k << 1 | [|d| > k]
    uint32_t* queue;             // queue, big_queue, big_count (consecutive)
    uint32_t* big_queue;
    uint32_t* big_count;
    uint64_t* big_list;
    uint32_t* big_rank;
    uint32_t* big_scratch;
    uint64_t big_words;
};

struct He2Params {
    Multi M;
    const uint8_t* he_tab;
    const uint64_t* bl_off;      // per ID slot: batch-neighbour list of x
    const uint64_t* bl_cnt;
    const uint32_t* bl_d;
    const uint64_t* bl_pay;
    uint32_t* queue;             // per stage (3 consecutive counters)
    uint32_t* count;             // items moved on by each stage (3 consecutive)
    uint64_t* list[3];           // list[s]: items stage s could not fit; list[2] feeds
    uint32_t* rank[3];           // the 2-hop kernel (k_delta_big), as do the densest centres
    uint32_t* garena;            // stage-2 tables: garena_words per workgroup
    uint64_t garena_words;
    uint64_t* stats;             // byte and hand-over counters (profiling), NULL = off
    int phase_ticks;             // 1 (with stats): wall-clock ticks per phase, at the cost of a
                                 // clock read and a barrier per phase
    int force_stage;             // test knob: stages below it move every centre on
    int skip_lds148;             // 1: the 148 KB stage moves every centre on to the global stage
    int pair_agg;                // 1: pairs counted per shared vertex by class histograms, pairs
                                 // sharing several vertices found through their vertex pairs
    uint64_t e2_2hop;            // vertex pairs from which a centre goes to the 2-hop kernel (0: default)
    uint32_t w_2hop;             // neighbour-row entries from which it does (0: default)
    int static_mode;             // full count (build): no batch ranks, no open paths through
                                 // neighbours; open triples at their centre, closed ones at the
                                 // smallest-ID centre
};

void he2_nbr_launch(NbrParams& P, unsigned grid_small, unsigned grid_big, hipStream_t s);
// per-ID batch-neighbour lists over all graphs of P.M (M.total_ids slots)
void he2_lists_build(NbrParams& P, uint64_t* bl_cnt, uint64_t* bl_off, uint64_t* bl_cur, uint32_t* bl_d,
                     uint64_t* bl_pay, void* scan_tmp, hipStream_t s);
// after the deletion phase: take the deleted hyperedges out of their neighbours' histograms
void he2_remove_deleted(NbrParams& P, hipStream_t s);
void he2_launch_stage(He2Params& P, int stage, unsigned grid, hipStream_t s);

// incident-vertex family
struct IvParams {
    GraphView g;
    const uint64_t* pairs;       // unique touched vertex pairs owner << 32 | other, ascending (the
                                 // owner is the endpoint of higher degree)
    const uint64_t* n_pairs;     // device count
    const uint64_t* owner_start; // first pair of every distinct u, plus the end
    const uint64_t* n_owners;
    const uint64_t* tab;         // open-addressing hash of the touched pairs (empty = ~0)
    uint64_t tab_mask;
    uint64_t* out;               // u64[2]: sum_p m_p * w_p, sum over triangles with a touched pair of m m m
    const int32_t* status;
    uint32_t* queue;             // per stage (3)
    uint32_t* count;             // owners moved on by stages 0 and 1 (2)
    uint32_t* list;              // owners stage 0 moved on (capacity: all owners)
    uint32_t* list2;             // owners stage 1 moved on (capacity: all owners)
    uint32_t* garena;            // stage 1: garena_words per workgroup
    uint64_t garena_words;
    uint32_t* garena2;           // stage 2: garena2_words per workgroup (the largest owners)
    uint64_t garena2_words;
    uint64_t* stats;             // optional, ST_IV_BYTES
    int force_direct;            // test knob: every owner evaluated pair by pair without a map
    int force_stage;             // test knob: stages below it move every owner on
};
// hash of the touched pairs (canon: lo << 32 | hi) and the owner segments of own
// (owner << 32 | other, sorted)
void iv_touched_build(const uint64_t* canon, const uint64_t* own, const uint64_t* n_pairs, uint64_t* tab,
                      uint64_t tab_slots, uint64_t* head, uint64_t* owner_start, uint64_t* n_owners, uint64_t pairs_cap,
                      void* scan_tmp, hipStream_t s);
void triad_iv_launch(IvParams& P, unsigned grid_lds, unsigned grid_global, unsigned grid_global2, hipStream_t s);
