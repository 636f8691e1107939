// triad.h -- launch interface of the triad-delta kernels.
#pragma once

#include "hgt_dev.h"

// Word offsets of the per-workgroup global tables of the large-centre kernel.
struct BigLayout {
    uint64_t nh_keys, nh_vals, hm, nl_x, nl_meta, warea, warea_words, words_per_wg;
};

struct TriadParams {
    GraphView g;
    const uint32_t* centres;  // changed hyperedge IDs; the index is the batch rank
    uint64_t n_centres;
    const uint64_t* mark;     // epoch-tagged batch rank per ID of this phase
    uint32_t epoch;
    int do_he, do_tmp;
    int64_t window;
    uint64_t* out_he;         // u64[30] phase accumulators
    uint64_t* out_tmp;        // u64[96]
    const uint8_t* he_tab;    // [128] class index of a Venn code (255 = not a triad)
    const uint8_t* tmp_tab;   // [128]
    const int32_t* status;
    uint32_t* queue;          // work counters, cleared by the launcher
    uint32_t* big_queue;
    uint32_t* big_count;
    uint32_t* big_list;       // centres deferred to the large kernel (capacity n_centres)
    uint32_t* big_rank;
    uint32_t* big_scratch;    // grid_big * big.words_per_wg words
    BigLayout big;
    uint64_t* stats;          // optional counters (see TriadStat), NULL = off
};

// Counters accumulated by the triad kernels when TriadParams.stats is set.
enum TriadStat {
    ST_BYTES_SMALL = 0,  // algorithmic bytes gathered by the small-centre kernel
    ST_BYTES_BIG = 1,    // ... by the large-centre kernel
    ST_DEFERRED = 2,     // centres moved to the large-centre kernel
    ST_WITNESS = 3,      // neighbours expanded through the binary-search path
    ST_EXPANDED = 4,     // neighbours expanded
    ST_IV_BYTES = 5,     // algorithmic bytes gathered by the incident-vertex kernel
    ST_N = 8
};

BigLayout triad_big_layout(uint64_t max_lh, uint64_t max_card);
void triad_he_prepare(TriadParams& P, hipStream_t s);
void triad_he_launch_small(TriadParams& P, unsigned grid, hipStream_t s);
void triad_he_launch_big(TriadParams& P, unsigned grid, hipStream_t s);

// incident-vertex family
struct IvParams {
    GraphView g;
    const uint64_t* pairs;    // unique touched vertex pairs u << 32 | v, ascending
    const uint64_t* n_pairs;  // device count
    uint64_t pairs_cap;
    uint64_t* out;            // u64[2]: sum_p m_p * w_p, sum over triangles with a touched pair of m m m
    const int32_t* status;
    uint64_t* stats;          // optional, ST_IV_BYTES
};
void triad_iv_launch(IvParams& P, hipStream_t s);
