// store.h -- host-visible pieces of the incidence store (see store.hip).
#pragma once

#include "hgt_dev.h"

// Device arrays of one graph (owned by the host-side graph object).
struct StoreDev {
    uint32_t n_vertices;
    uint64_t id_cap;        // length of every ID-indexed array
    uint64_t next_id_host;  // next_id as of the last synchronisation
    int hb, vb;             // key bits for IDs and vertices in the pair sort
    uint64_t* h_off;
    uint32_t* h_len;
    uint32_t* h_cap;
    int64_t* h_ts;          // NULL unless temporal is tracked
    uint64_t* h_seq;
    uint64_t* free_bm;
    uint32_t* h2v;
    uint64_t h2v_words;
    uint64_t* v_off;
    uint32_t* v_len;
    uint32_t* v_cap;
    uint32_t* v2h;
    int64_t* v2h_ts;        // NULL unless temporal is tracked: timestamp of every v2h entry
    uint64_t v2h_words;
    uint64_t* mark_del;
    uint64_t* mark_ins;
    DevScalars* sc;
};

struct BatchIn {
    const uint32_t* del;
    uint64_t n_del;
    const uint64_t* ins_off;
    const uint32_t* ins_mem;
    uint64_t n_ins_members;
    const int64_t* ins_ts;
    uint64_t n_ins;
    uint32_t epoch_del, epoch_ins;
    int check_order;  // 0 for the build batch and horizontal operations (timestamps not checked)
    const uint32_t* forced_ids;  // device [n_ins] or NULL: insert j takes this ID (horizontal operations,
                                 // where it is the ID deleted at the same rank)
    int keep_seq;     // 1: inserts keep the arrival sequence of their ID (horizontal operations)
};

// Per touched vertex plan (indexed by touched-vertex rank).
struct VPlan {
    uint64_t* dstart;    // first deleted ID of the vertex in D_all
    uint64_t* istart;    // first inserted ID of the vertex in I_all
    uint32_t* nD;
    uint32_t* nI;
    uint64_t* old_len;
    uint32_t* new_len;
    uint64_t* need;      // words of a fresh block, 0 = update in place
    uint64_t* rel;       // exclusive scan of need
    uint64_t* stage_off; // exclusive scan of old_len
};

struct PlanScratch {
    BatchSummary* sum;
    uint64_t* del_bm;
    uint64_t* del_card;
    uint64_t* del_poff;
    uint64_t* ins_rel;
    uint64_t* ins_card;
    uint32_t* canon;
    uint32_t* big_list;
    uint32_t* big_count;
    uint64_t* popc;
    uint64_t* n_words;
    uint64_t* n_free;
    void* scan_tmp;
    uint32_t* assigned;
    uint64_t* h_need;
    uint64_t* h_rel;
    uint64_t* h2v_total;
    uint64_t pairs_cap;
    uint64_t* keys;
    uint64_t* keys_alt;
    void* sort_tmp;
    uint64_t* n_pairs;
    uint64_t* head;
    uint64_t* is_ins;
    uint64_t* n_touched;
    uint64_t* n_ins_pairs;
    uint32_t* tv;
    uint64_t* tseg;
    uint32_t* D_all;
    uint32_t* I_all;
    uint32_t* I_t;
    VPlan vp;
    uint64_t* v2h_total;
    uint64_t* stage_total;
    uint32_t* staging;
    int64_t* staging_ts;    // timestamps of the staged entries (temporal graphs)
    uint64_t* dst;
};

void store_batch_begin(DevScalars* sc, BatchSummary* sum, hipStream_t s);
void store_plan(StoreDev& g, BatchIn& b, PlanScratch& w, hipStream_t s);
void store_commit(StoreDev& g, BatchIn& b, PlanScratch& w, const BatchSummary& sum, uint64_t h_bump,
                  uint64_t v_bump, uint64_t next_seq, hipStream_t s);
void store_max_ts(const int64_t* ts, uint64_t n, DevScalars* sc, hipStream_t s);
void store_counts_update(uint64_t* counts, const uint64_t* plus, const uint64_t* minus, int n,
                         const DevScalars* sc, hipStream_t s);

// Compaction of the pools (every live list into a fresh pool; the blocks of
// free IDs and the blocks left behind by relocations are dropped):
// per-ID / per-vertex block words (0 for free IDs and empty lists) ...
void store_compact_need(const StoreDev& g, uint64_t n_ids, uint64_t* h_need, uint64_t* v_need, hipStream_t s);
// ... and, after the caller's exclusive scans gave new offsets and fresh pools,
// the copies (h2v with its 2-word-per-word histograms, v2h with its
// timestamps, either side array may be NULL) and the new offsets/capacities.
void store_compact_h2v(const StoreDev& g, uint64_t n_ids, const uint64_t* need, const uint64_t* new_off,
                       uint32_t* h2v_new, const uint32_t* hpool, uint32_t* hpool_new, hipStream_t s);
void store_compact_v2h(const StoreDev& g, const uint64_t* need, const uint64_t* new_off, uint32_t* v2h_new,
                       int64_t* v2h_ts_new, hipStream_t s);
void store_compact_scalars(DevScalars* sc, const uint64_t* h_total, const uint64_t* v_total, hipStream_t s);
