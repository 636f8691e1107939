// hops.h -- horizontal operations (see hops.hip).
#pragma once

#include "hgt_dev.h"

struct VopSummary {
    int32_t status;
    uint32_t pad0;
    uint64_t n_mod;       // modified hyperedges
    uint64_t n_members;   // members of their new rows
    uint64_t pad[5];
};

struct VopIn {
    const uint32_t* edge_ids;
    const uint32_t* vertices;
    const uint8_t* insert;
    uint64_t n;
    int hb, vb;              // key bits of IDs (below next_id) and vertices
    uint32_t n_vertices;
    const uint64_t* free_bm;
    const uint64_t* h_off;
    const uint32_t* h_len;
    const uint32_t* h2v;
    const int64_t* h_ts;     // NULL unless temporal is tracked
    DevScalars* sc;
};

struct VopScratch {
    VopSummary* sum;
    uint64_t* keys;
    uint64_t* keys_alt;
    void* sort_tmp;
    void* scan_tmp;
    uint64_t* head;     // segment-head flags, then their exclusive scan
    uint64_t* ins_pre;  // insert flags, then their exclusive scan (n + 1 entries)
    uint64_t* n_mod;    // device count of modified hyperedges
    uint32_t* mod_ids;  // ascending modified IDs
    uint64_t* seg;      // first op of every modified hyperedge, then n (n + 1 entries)
    uint64_t* card;     // new cardinalities
    int64_t* ts;        // their timestamps (temporal graphs)
    uint64_t* new_off;  // new rows (n + 1 entries)
    uint32_t* members;
};

// Validates and groups the ops and sizes the new rows; the summary is read
// after the stream has passed it.  Changes nothing in the graph.
void vops_plan(const VopIn& in, VopScratch& w, hipStream_t s);
// The new member rows of the n_mod modified hyperedges (after vops_plan).
void vops_rows(const VopIn& in, VopScratch& w, uint64_t n_mod, hipStream_t s);
