// triad_he2.hip -- hyperedge-family triad deltas without 2-hop expansion.
//
// Every live hyperedge x carries a histogram H_x over its line-graph
// neighbours y: H_x[k][f] = #{y : |x & y| = k, [|y| > k] = f} (2|x| u32
// counters, stored beside its h2v block).  A changed hyperedge adds or removes
// one neighbour of each x in N(h), so the histograms are kept exact with one
// atomic per (h, x) pair.
//
// For a centre h and a neighbour x, the triads {h, x, y} with y outside the
// closed neighbourhood of h (open paths h - x - y) have the class
//   h only  = |h| > c_x,  x only = |x| - c_x - |x & y| > 0,  y only = |y| > |x & y|,
//   plus the regions h&x and x&y,
// so they are counted from H_x with one threshold (|x & y| < |x| - c_x), minus
// h itself, minus the batch members that rank below h (read from x's
// batch-neighbour list) and, in the pair phase, minus the other neighbours of h
// that meet x.
// Neighbour pairs {x, y} of h that intersect are found by grouping the member
// vertices of all neighbours of h by vertex in LDS (work sum_{x in N(h)} |x|),
// each pair counted at its smallest common vertex; they get their true class in
// place of the disjoint-pair class that the histogram pass gave them.
#include "triad_common.h"

namespace {

using namespace tri;

constexpr uint32_t ARENA_S = 8192;    // 32 KB of LDS: four workgroups per CU
constexpr uint32_t ARENA_M = 37888;   // 148 KB of LDS: one workgroup per CU
constexpr uint32_t K_MAX = 0xfffffu;  // neighbours with 20 bits
constexpr int KEY_IN = 20;             // entry key: vertex << KEY_V | [vertex in h] << KEY_IN | neighbour
constexpr int KEY_V = 21;
constexpr uint32_t W_MAX = 1u << 21;   // entries of a centre: run starts take 21 bits
constexpr int EMIT_HI = 20;            // vertex-pair key: lo run << EMIT_LO | hi run << EMIT_HI | neighbour
constexpr int EMIT_LO = 41;
// A centre with this many neighbour-row entries or neighbours goes to the 2-hop
// kernel, which shares it among several workgroups: in dense neighbourhoods its
// runs are long (enumerating their pairs is quadratic in one workgroup) and its
// neighbours share many vertices (the vertex pairs of the aggregated phase blow up).
constexpr uint32_t W_2HOP = 65536;
constexpr uint32_t K_2HOP = 0x4000u;
constexpr uint64_t E2_2HOP = 65536;  // ... and so does one whose neighbours hold this many vertex pairs
                                     // (He2Params::e2_2hop overrides it)
// entry key: vertex << 21 | [vertex in h] << 20 | neighbour index (20 bits)

// open-addressing tables of any capacity: slot = multiply-shift hash scaled to cap
__device__ __forceinline__ uint32_t fr_slot(uint32_t key, uint32_t cap) {
    return (uint32_t)(((uint64_t)(key * 2654435761u) * cap) >> 32);
}
__device__ __forceinline__ uint32_t fr_next(uint32_t s, uint32_t cap) { return s + 1 == cap ? 0 : s + 1; }
__device__ __forceinline__ uint32_t hash_cap(uint32_t n) { return n + n / 2 + 32; }  // load <= 2/3

__device__ __forceinline__ void fr_add(uint32_t* keys, uint32_t* vals, uint32_t cap, uint32_t key, uint32_t inc) {
    uint32_t s = fr_slot(key, cap);
    for (uint32_t probe = 0; probe < cap; probe++) {
        uint32_t k = __atomic_load_n(&keys[s], __ATOMIC_RELAXED);
        if (k == HGT_EMPTY) {
            uint32_t prev = atomicCAS(&keys[s], HGT_EMPTY, key);
            if (prev == HGT_EMPTY || prev == key) { atomicAdd(&vals[s], inc); return; }
        } else if (k == key) {
            atomicAdd(&vals[s], inc);
            return;
        }
        s = fr_next(s, cap);
    }
}

// One compare-exchange of the bitonic network between lanes: the lane whose
// index has a zero at hb (the highest bit of the mask m) keeps the smaller key.
__device__ __forceinline__ uint64_t cx_lanes(uint64_t x, uint32_t i, uint32_t m, uint32_t hb) {
    const uint64_t y = __shfl_xor(x, (int)m, 64);
    return (i & hb) ? (x > y ? x : y) : (x < y ? x : y);
}

// The steps of the network whose masks are below 64, in registers: all levels
// up to 64 (first) or the strides 32 .. 1 of a larger level.  Keys past n enter
// as +infinity and are not stored.
__device__ __forceinline__ void sort_lane_steps(uint64_t* k, uint32_t n, bool first) {
    for (uint32_t b = 0; b < n; b += HGT_WG) {
        const uint32_t i = b + threadIdx.x;
        uint64_t x = i < n ? k[i] : ~0ull;
        if (first) {
            for (uint32_t size = 2; size <= 64; size <<= 1) {
                x = cx_lanes(x, i, size - 1, size >> 1);
                for (uint32_t st = size >> 2; st > 0; st >>= 1) x = cx_lanes(x, i, st, st);
            }
        } else {
            for (uint32_t st = 32; st > 0; st >>= 1) x = cx_lanes(x, i, st, st);
        }
        if (i < n) k[i] = x;
    }
    __syncthreads();
}

// Ascending bitonic sort of n keys in place by the whole workgroup.  Each level
// of the network compares i with its mirror in the block (mask size - 1), then
// with i ^ stride for stride = size/4 .. 1, the smaller key going first; absent
// keys past n behave as +infinity, so no padding to a power of two is stored.
// Masks of 64 and more go through memory, one pass each; the smaller ones stay
// inside a wavefront's 64 consecutive keys and run in registers.
__device__ __forceinline__ void sort_keys(uint64_t* k, uint32_t n) {
    if (n < 2) return;
    const uint32_t N = (uint32_t)pow2ceil64(n);
    sort_lane_steps(k, n, true);
    for (uint32_t size = 128; size <= N; size <<= 1) {
        for (uint32_t i = threadIdx.x; i < n; i += HGT_WG) {
            uint32_t p = i ^ (size - 1);
            if (p > i && p < n) {
                uint64_t a = k[i], b = k[p];
                if (b < a) { k[i] = b; k[p] = a; }
            }
        }
        __syncthreads();
        for (uint32_t stride = size >> 2; stride >= 64; stride >>= 1) {
            for (uint32_t i = threadIdx.x; i < n; i += HGT_WG) {
                uint32_t p = i ^ stride;
                if (p > i && p < n) {
                    uint64_t a = k[i], b = k[p];
                    if (b < a) { k[i] = b; k[p] = a; }
                }
            }
            __syncthreads();
        }
        sort_lane_steps(k, n, false);
    }
}

// The same sort for keys in global memory, staged through an LDS tile of TILE_K
// keys: every tile is first sorted in LDS (all levels up to TILE_K), and in each
// larger level only the strides of TILE_K and more go through global memory; the
// strides below run in the tile.  Absent keys past n are +infinity as above.
constexpr uint32_t TILE_K = 4096;  // 32 KB of LDS

// one compare-exchange step in the tile: i against i ^ mask, the smaller key first
__device__ __forceinline__ void tile_cx(uint64_t* t, uint32_t mask) {
    for (uint32_t i = threadIdx.x; i < TILE_K; i += HGT_WG) {
        const uint32_t p = i ^ mask;
        if (p > i) {
            const uint64_t a = t[i], b = t[p];
            if (b < a) { t[i] = b; t[p] = a; }
        }
    }
    __syncthreads();
}

// strides stride .. 1 of a level inside the tile (strides below 64 in registers)
__device__ __forceinline__ void tile_strides(uint64_t* t, uint32_t stride) {
    for (; stride >= 64; stride >>= 1) tile_cx(t, stride);
    sort_lane_steps(t, TILE_K, false);
}

__device__ void sort_keys_tiled(uint64_t* k, uint32_t n, uint64_t* tile) {
    if (n < 2) return;
    const uint32_t N = (uint32_t)pow2ceil64(n);
    // every tile sorted on its own: all levels up to TILE_K
    for (uint32_t t0 = 0; t0 < n; t0 += TILE_K) {
        const uint32_t m = n - t0 < TILE_K ? n - t0 : TILE_K;
        for (uint32_t i = threadIdx.x; i < TILE_K; i += HGT_WG) tile[i] = i < m ? k[t0 + i] : ~0ull;
        __syncthreads();
        sort_lane_steps(tile, TILE_K, true);
        for (uint32_t size = 128; size <= TILE_K; size <<= 1) {
            tile_cx(tile, size - 1);
            tile_strides(tile, size >> 2);
        }
        for (uint32_t i = threadIdx.x; i < m; i += HGT_WG) k[t0 + i] = tile[i];
        __syncthreads();
    }
    for (uint32_t size = 2 * TILE_K; size <= N; size <<= 1) {
        for (uint32_t i = threadIdx.x; i < n; i += HGT_WG) {  // the mirror step, in global memory
            uint32_t p = i ^ (size - 1);
            if (p > i && p < n) {
                uint64_t a = k[i], b = k[p];
                if (b < a) { k[i] = b; k[p] = a; }
            }
        }
        __syncthreads();
        for (uint32_t stride = size >> 2; stride >= TILE_K; stride >>= 1) {
            for (uint32_t i = threadIdx.x; i < n; i += HGT_WG) {
                uint32_t p = i ^ stride;
                if (p > i && p < n) {
                    uint64_t a = k[i], b = k[p];
                    if (b < a) { k[i] = b; k[p] = a; }
                }
            }
            __syncthreads();
        }
        for (uint32_t t0 = 0; t0 < n; t0 += TILE_K) {  // strides below TILE_K, per tile
            const uint32_t m = n - t0 < TILE_K ? n - t0 : TILE_K;
            for (uint32_t i = threadIdx.x; i < TILE_K; i += HGT_WG) tile[i] = i < m ? k[t0 + i] : ~0ull;
            __syncthreads();
            tile_strides(tile, TILE_K >> 1);
            for (uint32_t i = threadIdx.x; i < m; i += HGT_WG) k[t0 + i] = tile[i];
            __syncthreads();
        }
    }
}

struct Sh2 {
    uint32_t h, rank, hlen, lh, K, W, defer, stop;
    uint32_t gi, cur_g, skip;
    uint64_t hoff;
    uint32_t ncap;
    uint32_t o_nh, o_ent;  // arena word offsets
    uint32_t agg, nbig, nb1;   // aggregated pair phase: taken, long runs, long-run members of length > 1
    uint32_t fits_g;           // ... its tables fit the global stage's arena
    uint32_t to2;              // too many vertex pairs: the centre goes to the 2-hop kernel
    uint64_t acc2[NWAVE * HGT_N_HE_CLASSES];  // the centre's changes, doubled (ordered pairs once)
    uint32_t ws[NWAVE];
    uint64_t g[8];
};

__device__ __forceinline__ void acc_sub(uint64_t* acc, int cls) { acc_add(acc, cls, ~0ull); }
__device__ __forceinline__ void acc32_add(uint32_t* acc, int cls, uint32_t v) {
    if (cls < 255) atomicAdd(&acc[cls], v);
}


// ---- per-centre neighbourhood (shared by the neighbour pass and the delta kernel)
// Builds N(h) -> c_x in the hash at keys/vals (already cleared), reading the
// incidence lists of h's members through pre/voff.
__device__ __forceinline__ void build_nh(const GraphView& G, uint32_t h, uint32_t hlen, uint32_t lh, const uint32_t* pre,
                                         const uint64_t* voff, uint32_t* keys, uint32_t* vals, uint32_t cap) {
    for (uint32_t p = threadIdx.x; p < lh; p += HGT_WG) {
        uint32_t k = seg_of<uint32_t>(pre, hlen, p);
        uint32_t x = G.v2h[voff[k] + (p - pre[k])];
        if (x != h) fr_add(keys, vals, cap, x, 1u);
    }
}

// prefix of member degrees and their list offsets; returns lh (all threads)
__device__ __forceinline__ uint32_t member_prefix(const GraphView& G, uint64_t hoff, uint32_t hlen, uint32_t* pre,
                                                  uint64_t* voff, uint32_t* ws) {
    uint32_t carry = 0;
    for (uint32_t b = 0; b < hlen; b += HGT_WG) {
        uint32_t i = b + threadIdx.x, d = 0;
        if (i < hlen) {
            uint32_t m = G.h2v[hoff + i];
            d = G.v_len[m];
            voff[i] = G.v_off[m];
        }
        uint32_t tot;
        uint32_t ex = wg_scan_u32(d, ws, &tot);
        if (i < hlen) pre[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) pre[hlen] = carry;
    __syncthreads();
    return carry;
}

// ===========================================================================
// neighbour pass: batch-neighbour entries (x, d, k = |x & d|, [|d| > k]) and,
// for inserted hyperedges, the histogram updates
// ===========================================================================
template <bool BIG>
__device__ void nbr_pass_body(const NbrParams& P, uint32_t* arena, uint64_t arena_words) {
    __shared__ Sh2 sh;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) {
            uint64_t n = BIG ? (uint64_t)*P.big_count : P.M.total;
            uint32_t c = atomicAdd(BIG ? P.big_queue : P.queue, 1u);
            sh.stop = c >= n;
            if (!sh.stop) {
                uint32_t gi, h, rank;
                if (BIG) {
                    uint64_t it = P.big_list[c];
                    gi = (uint32_t)(it >> 32);
                    h = (uint32_t)it;
                    rank = P.big_rank[c];
                } else {
                    gi = multi_graph_of(P.M, c);
                    rank = (uint32_t)(c - P.M.base[gi]);
                    h = P.M.graphs[gi].centres[rank];
                }
                const HeGraph& Gq = P.M.graphs[gi];
                sh.gi = gi;
                sh.h = h;
                sh.rank = rank;
                sh.skip = *((volatile const int32_t*)Gq.status) != 0;
                sh.hlen = Gq.g.h_len[h];
                sh.hoff = Gq.g.h_off[h];
                // prefix + offsets must fit at the arena end
                sh.defer = (!BIG && 3ull * sh.hlen + 4 > arena_words / 2) ? 1u : 0u;
            }
        }
        __syncthreads();
        if (sh.stop) break;
        if (sh.skip) {
            __syncthreads();
            continue;
        }
        const HeGraph& G = P.M.graphs[sh.gi];
        if (!sh.defer) {
            const uint32_t hlen = sh.hlen;
            uint32_t* pre = arena + arena_words - (3 * hlen + 4);
            uint64_t* voff = (uint64_t*)(pre + ((hlen + 2) & ~1u));
            if (((uintptr_t)voff & 7) != 0) voff = (uint64_t*)((uint32_t*)voff + 1);
            uint32_t lh = member_prefix(G.g, sh.hoff, hlen, pre, voff, sh.ws);
            uint32_t cap = hash_cap(lh);
            if (tid == 0) {
                sh.lh = lh;
                sh.ncap = cap;
                sh.defer = (!BIG && 2ull * cap + 3ull * hlen + 4 > arena_words) ? 1u : 0u;
            }
            __syncthreads();
        }
        if (sh.defer) {
            if (tid == 0) {
                uint32_t q = atomicAdd(P.big_count, 1u);
                P.big_list[q] = item_of(sh.gi, sh.h);
                P.big_rank[q] = sh.rank;
            }
            __syncthreads();
            continue;
        }
        const uint32_t h = sh.h, hlen = sh.hlen, lh = sh.lh, cap = sh.ncap;
        uint32_t* keys = arena;
        uint32_t* vals = arena + cap;
        uint32_t* pre = arena + arena_words - (3 * hlen + 4);
        uint64_t* voff = (uint64_t*)(pre + ((hlen + 2) & ~1u));
        if (((uintptr_t)voff & 7) != 0) voff = (uint64_t*)((uint32_t*)voff + 1);
        for (uint32_t s = tid; s < cap; s += HGT_WG) { keys[s] = HGT_EMPTY; vals[s] = 0; }
        __syncthreads();
        build_nh(G.g, h, hlen, lh, pre, voff, keys, vals, cap);
        __syncthreads();
        uint32_t* hd = G.hpool + 2 * sh.hoff;
        for (uint32_t s = tid; s < cap; s += HGT_WG) {
            uint32_t x = keys[s];
            if (x == HGT_EMPTY) continue;
            uint32_t c = vals[s];
            uint32_t fd = hlen > c ? 1u : 0u;
            if (P.emit_entries) {
                uint64_t q = atomicAdd((unsigned long long*)P.n_entries, 1ull);
                if (q < P.entries_cap) {
                    P.ent_x[q] = (uint32_t)(G.id_base + x);
                    P.ent_d[q] = h;
                    P.ent_pay[q] = ((uint64_t)sh.rank << 32) | ((uint64_t)c << 1) | fd;
                }
            }
            if (P.inserting) {
                uint32_t lx = G.g.h_len[x];
                atomicAdd(&hd[2 * (c - 1) + (lx > c ? 1u : 0u)], 1u);
                // an inserted neighbour builds its own histogram, this one included
                if ((uint32_t)(G.mark[x] >> 32) != G.epoch)
                    atomicAdd(&G.hpool[2 * G.g.h_off[x] + 2 * (c - 1) + fd], 1u);
            }
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(HGT_WG) k_nbr_small(NbrParams P) {
    __shared__ __attribute__((aligned(16))) uint32_t arena[ARENA_S];
    nbr_pass_body<false>(P, arena, ARENA_S);
}

__global__ void __launch_bounds__(HGT_WG) k_nbr_big(NbrParams P) {
    nbr_pass_body<true>(P, P.big_scratch + (uint64_t)blockIdx.x * P.big_words, P.big_words);
}

// clear the histograms of the inserted hyperedges (their blocks may be reused); a wave per centre
__global__ void k_h_clear(Multi M) {
    const int lane = threadIdx.x & 63;
    uint64_t q = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (q >= M.total) return;
    uint32_t gi = multi_graph_of(M, q);
    const HeGraph& G = M.graphs[gi];
    if (*G.status) return;
    uint32_t id = G.centres[q - M.base[gi]];
    uint32_t* hb = G.hpool + 2 * G.g.h_off[id];
    uint32_t w = 2 * G.g.h_len[id];
    for (uint32_t i = lane; i < w; i += 64) hb[i] = 0;
}

// remove the deleted hyperedges from their surviving neighbours' histograms
__global__ void k_h_remove(Multi M, const uint64_t* n_entries_p, uint64_t cap, const uint32_t* __restrict__ ent_x,
                           const uint64_t* __restrict__ ent_pay) {
    uint64_t n = *n_entries_p;
    if (n > cap) n = cap;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t slot = ent_x[i];
        const HeGraph& G = M.graphs[multi_graph_of_id(M, slot)];
        if (*G.status) continue;
        uint32_t x = (uint32_t)(slot - G.id_base);
        if ((uint32_t)(G.mark[x] >> 32) == G.epoch) continue;  // x is deleted too
        uint64_t p = ent_pay[i];
        uint32_t k = (uint32_t)(p >> 1) & 0x7fffffffu, f = (uint32_t)p & 1u;
        atomicSub(&G.hpool[2 * G.g.h_off[x] + 2 * (k - 1) + f], 1u);
    }
}

// counting sort of the entries by ID slot: per-slot counts, then scatter
__global__ void k_bl_count(const uint64_t* n_entries_p, uint64_t cap, const uint32_t* __restrict__ ent_x,
                           uint64_t* bl_cnt) {
    uint64_t n = *n_entries_p;
    if (n > cap) n = cap;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        atomicAdd((unsigned long long*)&bl_cnt[ent_x[i]], 1ull);
}

__global__ void k_bl_scatter(const uint64_t* n_entries_p, uint64_t cap, const uint32_t* __restrict__ ent_x,
                             const uint32_t* __restrict__ ent_d, const uint64_t* __restrict__ ent_pay,
                             uint64_t* bl_cur, uint32_t* out_d, uint64_t* out_pay) {
    uint64_t n = *n_entries_p;
    if (n > cap) n = cap;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t pos = atomicAdd((unsigned long long*)&bl_cur[ent_x[i]], 1ull);
        out_d[pos] = ent_d[i];
        out_pay[pos] = ent_pay[i];
    }
}

// the entry buffer is sized for the worst case; overflow is an internal error of every graph
__global__ void k_entries_check(Multi M, const uint64_t* n_entries_p, uint64_t cap) {
    if (*n_entries_p <= cap) return;
    for (uint32_t g = threadIdx.x; g < M.n_graphs; g += blockDim.x)
        atomicCAS(const_cast<int32_t*>(M.graphs[g].status), 0, HGT_EDEVICE);
}

// ===========================================================================
// the delta kernel
// ===========================================================================
// Stage s takes its centres from the batch (s = 0) or from list s-1 and moves
// the centres whose tables do not fit its arena to list s; list 2 feeds the
// 2-hop kernel.  Stages 0 and 1 keep the arena in LDS (32 KB, 148 KB), stage 2
// in a 1 MB slice of global memory per workgroup.
// |x & y|, |x & y & h| and the smallest common vertex of two sorted rows
__device__ __forceinline__ void row_meet(const uint32_t* X, uint32_t xl, const uint32_t* Y, uint32_t yl,
                                         const uint32_t* hm, uint32_t hlen, uint32_t& s, uint32_t& shh,
                                         uint32_t& first) {
    uint32_t a = 0, b = 0;
    s = 0;
    shh = 0;
    first = HGT_EMPTY;
    while (a < xl && b < yl) {
        uint32_t va = X[a], vb = Y[b];
        if (va < vb) a++;
        else if (va > vb) b++;
        else {
            if (s == 0) first = va;
            s++;
            shh += contains_u32(hm, hlen, va) ? 1u : 0u;
            a++;
            b++;
        }
    }
}

// The class adjustments of one intersecting neighbour pair {x, y} of centre h
// (|x & y| = s, |h & x & y| = shh): in a full count the closed triad at the
// smallest-ID centre, in a delta the open-path and disjoint-pair corrections.
__device__ __forceinline__ void pair_class(const He2Params& P, const Tables& T, uint32_t h, uint32_t hlen,
                                           const uint32_t* nl_x, const uint32_t* nl_meta, uint32_t xi, uint32_t yi,
                                           uint32_t s, uint32_t shh, uint32_t* myacc32) {
    const uint32_t mx = nl_meta[xi], my = nl_meta[yi];
    const uint32_t xl = meta_len(mx), yl = meta_len(my), cx = meta_c(mx), cy = meta_c(my);
    if (P.static_mode) {
        // closed triple: counted at its smallest-ID centre only
        acc32_add(myacc32, T.he[venn_code((int)hlen, (int)xl, (int)yl, (int)cx, 0, (int)cy, 0)], ~0u);
        if (h < nl_x[xi] && h < nl_x[yi])
            acc32_add(myacc32, T.he[venn_code((int)hlen, (int)xl, (int)yl, (int)cx, (int)s, (int)cy, (int)shh)], 1u);
        return;
    }
    // a lower-ranked batch member was already taken off its partner's open paths
    if (meta_elig(mx) && meta_elig(my)) {
        uint32_t base = (hlen > cx ? 1u : 0u) | 24u;
        acc32_add(myacc32, T.he[base | (xl - cx > s ? 2u : 0u) | (yl > s ? 4u : 0u)], ~0u);
        base = (hlen > cy ? 1u : 0u) | 24u;
        acc32_add(myacc32, T.he[base | (yl - cy > s ? 2u : 0u) | (xl > s ? 4u : 0u)], ~0u);
        int ct = T.he[venn_code((int)hlen, (int)xl, (int)yl, (int)cx, (int)s, (int)cy, (int)shh)];
        int cf = T.he[venn_code((int)hlen, (int)xl, (int)yl, (int)cx, 0, (int)cy, 0)];
        if (ct != cf) {
            acc32_add(myacc32, ct, 1u);
            acc32_add(myacc32, cf, ~0u);
        }
    }
}

// ---- single-vertex pairs, aggregated.  Take neighbours x, y of h that meet
// in exactly one vertex v (vin: v in h).  The class changes of the pair depend
// on y only through two bits gy and through how c_y = |y & h| compares with
// |h| - c_x (rng 0: less, 1: equal, 2: greater), so along a long run of
// neighbours at v they are counted from a histogram over (gy, c_y).
constexpr uint32_t RUN_DIRECT = 64;  // runs up to this length enumerate their pairs
static_assert(RUN_DIRECT <= 64, "short-run partners are counted in 6-bit fields");

__device__ __forceinline__ uint32_t single_gy(uint32_t vin, uint32_t yl, uint32_t cy) {
    return vin ? ((yl > cy ? 1u : 0u) | (cy > 1 ? 2u : 0u)) : ((yl > cy ? 1u : 0u) | (yl - cy > 1 ? 2u : 0u));
}

// Venn codes of the closed triad {h, x, y} (ct) and of the same x, y taken as
// disjoint (cf), for a pair meeting in one vertex (the regions of venn_code
// with |x & y| = 1 and |h & x & y| = vin).
__device__ __forceinline__ void single_codes(uint32_t vin, uint32_t xl, uint32_t cx, uint32_t gy, uint32_t rng, int& ct,
                                             int& cf) {
    cf = (rng == 0 ? 1 : 0) | (xl > cx ? 2 : 0) | ((gy & 1u) ? 4 : 0) | 8 | 32;
    if (vin)
        ct = (rng <= 1 ? 1 : 0) | (xl > cx ? 2 : 0) | ((gy & 1u) ? 4 : 0) | (cx > 1 ? 8 : 0) | ((gy & 2u) ? 32 : 0) | 64;
    else
        ct = (rng == 0 ? 1 : 0) | (xl - cx > 1 ? 2 : 0) | ((gy & 2u) ? 4 : 0) | 8 | 16 | 32;
}

// pair_class of a delta (not a full count) with every change weighted by w
__device__ __forceinline__ void pair_class_w(const Tables& T, uint32_t hlen, uint32_t mx, uint32_t my, uint32_t s,
                                             uint32_t shh, uint32_t w, uint32_t* myacc32) {
    const uint32_t xl = meta_len(mx), yl = meta_len(my), cx = meta_c(mx), cy = meta_c(my);
    const uint32_t nw = 0u - w;
    if (meta_elig(mx) && meta_elig(my)) {
        uint32_t base = (hlen > cx ? 1u : 0u) | 24u;
        acc32_add(myacc32, T.he[base | (xl - cx > s ? 2u : 0u) | (yl > s ? 4u : 0u)], nw);
        base = (hlen > cy ? 1u : 0u) | 24u;
        acc32_add(myacc32, T.he[base | (yl - cy > s ? 2u : 0u) | (xl > s ? 4u : 0u)], nw);
        int ct = T.he[venn_code((int)hlen, (int)xl, (int)yl, (int)cx, (int)s, (int)cy, (int)shh)];
        int cf = T.he[venn_code((int)hlen, (int)xl, (int)yl, (int)cx, 0, (int)cy, 0)];
        if (ct != cf) {
            acc32_add(myacc32, ct, w);
            acc32_add(myacc32, cf, nw);
        }
    }
}

// |x & y|, |x & y & h| and the two smallest common vertices of two sorted rows
__device__ __forceinline__ void row_meet2(const uint32_t* X, uint32_t xl, const uint32_t* Y, uint32_t yl,
                                          const uint32_t* hm, uint32_t hlen, uint32_t& s, uint32_t& shh,
                                          uint32_t& f1, uint32_t& f2) {
    uint32_t a = 0, b = 0;
    s = 0;
    shh = 0;
    f1 = f2 = HGT_EMPTY;
    while (a < xl && b < yl) {
        uint32_t va = X[a], vb = Y[b];
        if (va < vb) a++;
        else if (va > vb) b++;
        else {
            if (s == 0) f1 = va;
            else if (s == 1) f2 = va;
            s++;
            shh += contains_u32(hm, hlen, va) ? 1u : 0u;
            a++;
            b++;
        }
    }
}

__device__ __forceinline__ uint32_t lower_bound_u64(const uint64_t* a, uint32_t n, uint64_t key) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Pair number q of a run of R (pairs (a, b), a < b, ordered by a then b): the
// largest a with a R - a (a + 1) / 2 <= q, from the quadratic's root, then
// corrected by one step either way against rounding.
__device__ __forceinline__ void tri_decode(uint32_t R, uint32_t q, uint32_t& a, uint32_t& b) {
    const double r2 = 2.0 * (double)R - 1.0;
    const double d = r2 * r2 - 8.0 * (double)q;
    int64_t aa = (int64_t)((r2 - sqrt(d > 0.0 ? d : 0.0)) * 0.5);
    if (aa < 0) aa = 0;
    if (aa > (int64_t)R - 2) aa = (int64_t)R - 2;
    auto before = [R](uint64_t x) { return x * (2ull * R - x - 1) / 2; };
    while (aa > 0 && before((uint64_t)aa) > q) aa--;
    while (aa + 1 <= (int64_t)R - 2 && before((uint64_t)aa + 1) <= q) aa++;
    a = (uint32_t)aa;
    b = a + 1 + (uint32_t)(q - before((uint64_t)aa));
}

// Neighbours x, y (vertex-pair entries ex, ey of one (u, w) run) that share u
// and w: when u and w are their two smallest common vertices, their s single
// changes give way to the pair's own.
__device__ __forceinline__ void multi_pair(const GraphView& g, const Tables& T, uint32_t hlen, const uint32_t* hm,
                                           const uint64_t* keys, const uint32_t* nl_x, const uint32_t* nl_meta,
                                           uint64_t ex, uint64_t ey, uint64_t* stats, uint32_t* myacc32) {
    const uint32_t xi = (uint32_t)ex & K_MAX, yi = (uint32_t)ey & K_MAX;
    const uint32_t vu = (uint32_t)(keys[(uint32_t)(ex >> EMIT_LO)] >> KEY_V);
    const uint32_t vw = (uint32_t)(keys[(uint32_t)(ex >> EMIT_HI) & (W_MAX - 1)] >> KEY_V);
    const uint32_t mx = nl_meta[xi], my = nl_meta[yi];
    uint32_t s, shh, f1, f2;
    row_meet2(g.h2v + g.h_off[nl_x[xi]], meta_len(mx), g.h2v + g.h_off[nl_x[yi]], meta_len(my), hm, hlen, s, shh, f1, f2);
    // the run order of u and w need not be the vertex order
    if (!((f1 == vu && f2 == vw) || (f1 == vw && f2 == vu))) return;
    if (stats) atomicAdd((unsigned long long*)&stats[ST_AGG_MULTI], 1ull);
    pair_class_w(T, hlen, mx, my, s, shh, 1u, myacc32);
    if (shh) pair_class_w(T, hlen, mx, my, 1, 1, 0u - shh, myacc32);
    if (s > shh) pair_class_w(T, hlen, mx, my, 1, 0, 0u - (s - shh), myacc32);
}

// Adds the per-wave counts to graph g's phase accumulators and clears them.
__device__ void he2_flush_graph(const He2Params& P, uint32_t g, uint64_t* acc_all) {
    __syncthreads();
    if (g != 0xffffffffu) {
        const HeGraph& G = P.M.graphs[g];
        for (int i = threadIdx.x; i < HGT_N_HE_CLASSES; i += HGT_WG) {
            uint64_t s = 0;
            for (int w = 0; w < NWAVE; w++) s += acc_all[w * HGT_N_HE_CLASSES + i];
            if (s) atomicAdd((unsigned long long*)&G.out_he[i], (unsigned long long)s);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < NWAVE * HGT_N_HE_CLASSES; i += HGT_WG) acc_all[i] = 0;
    __syncthreads();
}

template <int STAGE>
__device__ void he2_body(const He2Params& P, uint32_t* arena, const uint32_t ARENA_WORDS, Sh2& sh, const Tables& T,
                         uint64_t* acc_all, uint32_t* acc32_all, uint64_t* st, uint64_t* ph, uint64_t* tile) {
    // keys in a global arena are sorted through the LDS tile; in an LDS arena in place
    auto sort_any = [tile](uint64_t* k, uint32_t n) {
        if (tile && n > TILE_K / 2) sort_keys_tiled(k, n, tile);
        else sort_keys(k, n);
    };
    const int tid = threadIdx.x;
    uint64_t t_mark = 0;    // thread 0: wall clock at the last phase mark (profiling)
    uint64_t t_centre = 0;  // ... at the start of the current centre
#define HE2_MARK(i)                                     \
    do {                                                \
        if (P.phase_ticks && tid == 0) {                \
            uint64_t t_ = wall_clock64();               \
            ph[i] += t_ - t_mark;                       \
            t_mark = t_;                                \
        }                                               \
    } while (0)
    // this centre's changes, doubled (halved when the centre ends): a centre handed on
    // to the next stage midway leaves nothing behind
    uint64_t* cacc = sh.acc2 + (tid >> 6) * HGT_N_HE_CLASSES;
    uint32_t* myacc32 = acc32_all + (tid >> 6) * HGT_N_HE_CLASSES;
    for (;;) {
        if (tid == 0) {
            uint32_t c = atomicAdd(&P.queue[STAGE], 1u);
            sh.stop = c >= (STAGE == 0 ? P.M.total : (uint64_t)P.count[STAGE - 1]);
            if (!sh.stop) {
                uint32_t gi, h, rank;
                if (STAGE == 0) {
                    gi = multi_graph_of(P.M, c);
                    rank = (uint32_t)(c - P.M.base[gi]);
                    h = P.M.graphs[gi].centres[rank];
                } else {
                    uint64_t it = P.list[STAGE - 1][c];
                    gi = (uint32_t)(it >> 32);
                    h = (uint32_t)it;
                    rank = P.rank[STAGE - 1][c];
                }
                const HeGraph& Gq = P.M.graphs[gi];
                sh.gi = gi;
                sh.h = h;
                sh.rank = rank;
                sh.skip = *((volatile const int32_t*)Gq.status) != 0;
                sh.hlen = Gq.g.h_len[h];
                sh.hoff = Gq.g.h_off[h];
                sh.defer = (3ull * sh.hlen + 4 > ARENA_WORDS / 2 || STAGE < P.force_stage || (STAGE == 1 && P.skip_lds148))
                               ? 1u : 0u;
            }
        }
        __syncthreads();
        if (sh.stop) break;
        if (P.phase_ticks && tid == 0) t_mark = t_centre = wall_clock64();
        if (sh.gi != sh.cur_g) {  // the counts so far belong to the previous graph
            he2_flush_graph(P, sh.cur_g, acc_all);
            if (tid == 0) sh.cur_g = sh.gi;
            __syncthreads();
        }
        if (sh.skip) {
            __syncthreads();
            continue;
        }
        const HeGraph& G = P.M.graphs[sh.gi];
        const uint32_t h = sh.h, hlen = sh.hlen;
        // --- members of h: degree prefix and list offsets at the arena end
        uint32_t* pre = arena + ARENA_WORDS - (3 * hlen + 4);
        uint64_t* voff = (uint64_t*)(pre + ((hlen + 2) & ~1u));
        if (((uintptr_t)voff & 7) != 0) voff = (uint64_t*)((uint32_t*)voff + 1);
        if (!sh.defer) {
            uint32_t lh = member_prefix(G.g, sh.hoff, hlen, pre, voff, sh.ws);
            uint32_t cap = hash_cap(lh);
            if (tid == 0) {
                sh.lh = lh;
                sh.ncap = cap;
                sh.o_nh = 0;
                uint64_t a = 2ull * cap + 3ull * hlen + 4, b = 2ull * cap + 4ull * lh + 1 + hlen + 2;
                sh.defer = ((a > b ? a : b) > ARENA_WORDS) ? 1u : 0u;
            }
            __syncthreads();
        }
        if (sh.defer) {
            if (tid == 0) {
                uint32_t q = atomicAdd(&P.count[STAGE], 1u);
                P.list[STAGE][q] = item_of(sh.gi, h);
                P.rank[STAGE][q] = sh.rank;
                atomicAdd((unsigned long long*)&st[0], 1ull);
            }
            HE2_MARK(7);
            __syncthreads();
            continue;
        }
        HE2_MARK(0);
        const uint32_t lh = sh.lh, ncap = sh.ncap;
        uint32_t* nkeys = arena;
        uint32_t* nvals = arena + ncap;
        for (uint32_t s = tid; s < ncap; s += HGT_WG) { nkeys[s] = HGT_EMPTY; nvals[s] = 0; }
        if (tid == 0) sh.K = 0;
        __syncthreads();
        build_nh(G.g, h, hlen, lh, pre, voff, nkeys, nvals, ncap);
        __syncthreads();
        HE2_MARK(1);
        // --- compact N(h): x, meta (c | len | eligible), member offsets later
        uint32_t* nl_x = arena + 2 * ncap;
        uint32_t* nl_meta = nl_x + lh;
        uint32_t* nl_mo = nl_meta + lh;  // lh + 1 words
        uint32_t* nl_msh = nl_mo + lh + 1;  // members shared with another neighbour
        for (uint32_t s = tid; s < ncap; s += HGT_WG) {
            uint32_t x = nkeys[s];
            if (x == HGT_EMPTY) continue;
            uint32_t c = nvals[s];
            uint32_t len = G.g.h_len[x];
            bool elig = P.static_mode || !lower_ranked_member(G.mark[x], G.epoch, sh.rank);
            uint32_t meta = c | (len << 14) | ((uint32_t)elig << 28);
            nvals[s] = meta;
            uint32_t q = atomicAdd(&sh.K, 1u);
            nl_x[q] = x;
            nl_meta[q] = meta;
        }
        __syncthreads();
        const uint32_t K = sh.K;
        // member offsets of the neighbours in the entry array
        uint32_t* hm = nl_msh + lh;  // members of h
        {
            uint32_t carry = 0;
            for (uint32_t b = 0; b < K; b += HGT_WG) {
                uint32_t i = b + tid;
                uint32_t v = i < K ? meta_len(nl_meta[i]) : 0;
                uint32_t tot;
                uint32_t ex = wg_scan_u32(v, sh.ws, &tot);
                if (i < K) nl_mo[i] = carry + ex;
                carry += tot;
            }
            if (tid == 0) {
                nl_mo[K] = carry;
                sh.W = carry;
                // h's row and its members' incidence lists, each neighbour's row and metadata
                if (P.stats)
                    atomicAdd((unsigned long long*)&st[1],
                              (unsigned long long)(4ull * (hlen + lh) + 20ull * K + 4ull * carry));
                uint64_t o_ent = (uint64_t)(hm + hlen - arena);
                o_ent = (o_ent + 1) & ~1ull;
                uint64_t need = 2ull * carry > 2ull * hlen + 2 ? 2ull * carry : 2ull * hlen + 2;
                sh.o_ent = (uint32_t)o_ent;
                // too large for this arena: the next stage; too dense for any: the 2-hop kernel
                sh.defer = (o_ent + need > ARENA_WORDS) ? 1u : 0u;
                if (K >= K_2HOP || carry >= (P.w_2hop ? P.w_2hop : W_2HOP)) sh.defer = 2u;
            }
            __syncthreads();
        }
        if (sh.defer) {
            if (tid == 0) {
                const int to = sh.defer == 2u ? 2 : STAGE;
                uint32_t q = atomicAdd(&P.count[to], 1u);
                P.list[to][q] = item_of(sh.gi, h);
                P.rank[to][q] = sh.rank;
                atomicAdd((unsigned long long*)&st[0], 1ull);
            }
            HE2_MARK(7);
            __syncthreads();
            continue;
        }
        HE2_MARK(2);
        const uint32_t W = sh.W;
        uint64_t* keys = (uint64_t*)(arena + sh.o_ent);
        for (uint32_t i = tid; i < hlen; i += HGT_WG) hm[i] = G.g.h2v[sh.hoff + i];
        // --- disjoint-pair classes of all eligible neighbour pairs (histogram over c)
        {
            uint32_t* cnt = (uint32_t*)keys;  // 2 (hlen + 1) words, free until the entries are written
            const uint32_t Wc = hlen + 1;
            for (uint32_t i = tid; i < 2 * Wc; i += HGT_WG) cnt[i] = 0;
            if (tid < 8) sh.g[tid] = 0;
            __syncthreads();
            for (uint32_t i = tid; i < K; i += HGT_WG) {
                uint32_t m = nl_meta[i];
                if (!meta_elig(m)) continue;
                uint32_t c = meta_c(m);
                atomicAdd(&cnt[(meta_len(m) > c ? Wc : 0) + c], 1u);
            }
            __syncthreads();
            for (uint32_t f = 0; f < 2; f++) {
                uint32_t carry2 = 0;
                for (uint32_t b = 0; b < Wc; b += HGT_WG) {
                    uint32_t i = b + tid;
                    uint32_t v = i < Wc ? cnt[f * Wc + i] : 0;
                    uint32_t tot;
                    uint32_t ex = wg_scan_u32(v, sh.ws, &tot);
                    if (i < Wc) cnt[f * Wc + i] = carry2 + ex;
                    carry2 += tot;
                }
                if (tid == 0) sh.g[6 + f] = carry2;
                __syncthreads();
            }
            const uint64_t N0 = sh.g[6], N1 = sh.g[7];
            uint64_t g00 = 0, g01 = 0, g11 = 0, d0 = 0, d1 = 0;
            for (uint32_t c = 1 + tid; c <= hlen; c += HGT_WG) {
                uint64_t n0 = (uint64_t)((c + 1 < Wc ? cnt[c + 1] : (uint32_t)N0) - cnt[c]);
                uint64_t n1 = (uint64_t)((c + 1 < Wc ? cnt[Wc + c + 1] : (uint32_t)N1) - cnt[Wc + c]);
                uint32_t k = hlen - c;
                uint64_t s0 = N0 - cnt[k], s1 = N1 - cnt[Wc + k];
                g00 += n0 * s0;
                g01 += n0 * s1;
                g11 += n1 * s1;
                if (2 * c >= hlen) { d0 += n0; d1 += n1; }
            }
            atomicAdd((unsigned long long*)&sh.g[0], (unsigned long long)g00);
            atomicAdd((unsigned long long*)&sh.g[1], (unsigned long long)g01);
            atomicAdd((unsigned long long*)&sh.g[2], (unsigned long long)g11);
            atomicAdd((unsigned long long*)&sh.g[3], (unsigned long long)d0);
            atomicAdd((unsigned long long*)&sh.g[4], (unsigned long long)d1);
            __syncthreads();
            if (tid == 0) {
                uint64_t G00 = (sh.g[0] - sh.g[3]) / 2, G11 = (sh.g[2] - sh.g[4]) / 2, G01 = sh.g[1];
                uint64_t T00 = N0 * (N0 - (N0 ? 1 : 0)) / 2, T11 = N1 * (N1 - (N1 ? 1 : 0)) / 2, T01 = N0 * N1;
                acc_add(cacc, T.he[40 | 1], 2 * (T00 - G00));
                acc_add(cacc, T.he[40], 2 * (G00));
                acc_add(cacc, T.he[40 | 4 | 1], 2 * (T01 - G01));
                acc_add(cacc, T.he[40 | 4], 2 * (G01));
                acc_add(cacc, T.he[40 | 6 | 1], 2 * (T11 - G11));
                acc_add(cacc, T.he[40 | 6], 2 * (G11));
            }
            __syncthreads();
        }
        HE2_MARK(3);
        // --- entries: (vertex, v in h, neighbour) for every member of every neighbour,
        // sorted by vertex so that the neighbours meeting at a vertex are contiguous
        for (uint32_t i = tid; i < K; i += HGT_WG) nl_msh[i] = 0;
        {
            // with a global arena, the neighbours' row offsets and entry prefix and h's
            // members are staged in the LDS tile (free until the sort) when they fit
            const uint32_t* mo_p = nl_mo;
            const uint32_t* hm_p = hm;
            const uint64_t* xo_p = nullptr;
            if (tile && 3ull * K + 3 + hlen <= 2ull * TILE_K) {
                uint64_t* xo = tile;
                uint32_t* t32 = (uint32_t*)(tile + K);
                for (uint32_t i = tid; i < K; i += HGT_WG) xo[i] = G.g.h_off[nl_x[i]];
                for (uint32_t i = tid; i <= K; i += HGT_WG) t32[i] = nl_mo[i];
                for (uint32_t i = tid; i < hlen; i += HGT_WG) t32[K + 1 + i] = hm[i];
                __syncthreads();
                xo_p = xo;
                mo_p = t32;
                hm_p = t32 + K + 1;
            }
            for (uint32_t p = tid; p < W; p += HGT_WG) {
                uint32_t xi = seg_of<uint32_t>(mo_p, K, p);
                const uint64_t xoff = xo_p ? xo_p[xi] : G.g.h_off[nl_x[xi]];
                uint32_t v = G.g.h2v[xoff + (p - mo_p[xi])];
                uint64_t inh = contains_u32(hm_p, hlen, v) ? 1ull : 0ull;
                keys[p] = ((uint64_t)v << KEY_V) | (inh << KEY_IN) | xi;
            }
            __syncthreads();
        }
        sort_any(keys, W);
        // vertices met by two or more neighbours; per neighbour, how many it has
        for (uint32_t i = tid; i < W; i += HGT_WG) {
            uint64_t v = keys[i] >> KEY_V;
            bool shared = (i > 0 && (keys[i - 1] >> KEY_V) == v) || (i + 1 < W && (keys[i + 1] >> KEY_V) == v);
            if (shared) atomicAdd(&nl_msh[keys[i] & K_MAX], 1u);
        }
        __syncthreads();
        HE2_MARK(4);
        // --- open paths h - x - y through the histograms, per eligible neighbour
        for (uint32_t i = P.static_mode ? K : tid; i < K; i += HGT_WG) {
            uint32_t m = nl_meta[i];
            if (!meta_elig(m)) continue;
            uint32_t x = nl_x[i];
            uint32_t c = meta_c(m), lx = meta_len(m);
            uint32_t thr = lx - c;  // k < thr  <=>  x has a vertex outside h and y
            uint32_t base = (hlen > c ? 1u : 0u) | 24u;
            const uint32_t* H = G.hpool + 2 * G.g.h_off[x];
            const uint64_t xs = G.id_base + x;
            if (P.stats)  // x's histogram, list bounds and batch-neighbour entries
                atomicAdd((unsigned long long*)&st[1], (unsigned long long)(8ull * lx + 16 + 8ull * P.bl_cnt[xs]));
            // a_f: neighbours y with |x & y| < thr (x keeps a private vertex), b_f: the rest
            uint64_t a0 = 0, a1 = 0, b0 = 0, b1 = 0;
            for (uint32_t k = 1; k <= lx; k++) {
                uint32_t h0 = H[2 * (k - 1)], h1 = H[2 * (k - 1) + 1];
                if (k < thr) { a0 += h0; a1 += h1; }
                else { b0 += h0; b1 += h1; }
            }
            // the histogram holds h itself: k = c, y only = |h| > c
            if (c < thr) { if (hlen > c) a1--; else a0--; }
            else { if (hlen > c) b1--; else b0--; }
            // every lower-ranked batch member adjacent to x (the pair phase leaves out
            // the ones that meet h)
            uint64_t bo = P.bl_off[xs], bn = P.bl_cnt[xs];
            for (uint64_t e = 0; e < bn; e++) {
                uint64_t pay = P.bl_pay[bo + e];
                if ((uint32_t)(pay >> 32) >= sh.rank) continue;
                uint32_t k = (uint32_t)(pay >> 1) & 0x7fffffffu, f = (uint32_t)pay & 1u;
                if (k < thr) { if (f) a1--; else a0--; }
                else { if (f) b1--; else b0--; }
            }
            acc_add(cacc, T.he[base | 2], 2 * (a0));
            acc_add(cacc, T.he[base | 2 | 4], 2 * (a1));
            acc_add(cacc, T.he[base], 2 * (b0));
            acc_add(cacc, T.he[base | 4], 2 * (b1));
        }
        if (P.phase_ticks) __syncthreads();
        HE2_MARK(5);
        // --- intersecting neighbour pairs, aggregated.  Every pair of neighbours in the
        // run of a shared vertex v is first taken as meeting only at v: its changes are
        // enumerated along runs of up to RUN_DIRECT entries and counted from a (gy, c_y)
        // histogram along longer runs, the closed-class changes once per ordered pair
        // (twice per pair, halved at the end).  Pairs that share s >= 2 vertices were
        // so counted once at each of them; they are found through the vertex pairs
        // (u, w) that each neighbour holds among its shared vertices (sorted, so the
        // neighbours holding u and w are contiguous), each at its two smallest common
        // vertices, and get their true changes in place of the s single ones.  Layout
        // after the entries: long runs, histogram, per-neighbour offsets of the shared
        // vertices and of the vertex pairs, fill cursors, shared vertices, vertex pairs,
        // the vertex pairs' pair numbering.
        if (tid == 0) {
            sh.agg = 0;
            sh.fits_g = 0;
            sh.to2 = 0;
            sh.nbig = 0;
            sh.g[6] = 0;  // shared entries of neighbours with two or more
            sh.g[7] = 0;  // their vertex pairs
        }
        __syncthreads();
        const uint32_t nb_cap = W / (RUN_DIRECT + 1) + 1, n_hist = 4u * (hlen + 1);
        const uint64_t o_big = (uint64_t)sh.o_ent + 2ull * W, o_hist = o_big + 2ull * nb_cap, o_off = o_hist + n_hist;
        const uint64_t o_eoff = o_off + K + 1, o_cur = o_eoff + K + 1, o_sl = o_cur + K;
        if (!P.static_mode && P.pair_agg && W < W_2HOP) {
            for (uint32_t i = tid; i < K; i += HGT_WG) {
                const uint64_t m = nl_msh[i];
                if (m >= 2) {
                    atomicAdd((unsigned long long*)&sh.g[6], (unsigned long long)m);
                    atomicAdd((unsigned long long*)&sh.g[7], (unsigned long long)(m * (m - 1) / 2));
                }
            }
            __syncthreads();
            if (tid == 0) {
                const uint64_t o_emit = (o_sl + sh.g[6] + 1) & ~1ull;  // then pp: one word per vertex pair
                const uint64_t need = o_emit + 3ull * sh.g[7];
                sh.agg = (o_sl <= ARENA_WORDS && need <= ARENA_WORDS) ? 1u : 0u;
                sh.fits_g = need <= P.garena_words ? 1u : 0u;
                if (sh.g[7] >= (P.e2_2hop ? P.e2_2hop : E2_2HOP)) sh.agg = sh.fits_g = 0, sh.to2 = 1;
            }
            __syncthreads();
        }
        // no room to aggregate here: a centre that the global stage can aggregate moves on
        // (dropping its changes so far); one that no stage can aggregate enumerates here
        const bool hand_on = STAGE < 2 && !sh.agg && sh.fits_g;
        if (hand_on || sh.to2) {
            for (uint32_t i = tid; i < NWAVE * HGT_N_HE_CLASSES; i += HGT_WG) {
                sh.acc2[i] = 0;
                acc32_all[i] = 0;
            }
            if (tid == 0) {
                const int to = sh.to2 ? 2 : STAGE;  // list 2 feeds the 2-hop kernel
                uint32_t q = atomicAdd(&P.count[to], 1u);
                P.list[to][q] = item_of(sh.gi, h);
                P.rank[to][q] = sh.rank;
                atomicAdd((unsigned long long*)&st[0], 1ull);
            }
            HE2_MARK(7);
            __syncthreads();
            continue;
        }
        if (P.stats && tid == 0 && !P.static_mode && !sh.agg) atomicAdd((unsigned long long*)&P.stats[ST_AGG_ENUM], 1ull);
        if (sh.agg) {
            const uint32_t S = (uint32_t)sh.g[6], E2 = (uint32_t)sh.g[7];
            uint32_t* big = arena + o_big;
            uint32_t* hist = arena + o_hist;
            uint32_t* off = arena + o_off;
            uint32_t* eoff = arena + o_eoff;
            uint32_t* cur = arena + o_cur;
            uint32_t* sl = arena + o_sl;
            uint64_t* emit = (uint64_t*)(arena + ((o_sl + S + 1) & ~1ull));
            {
                uint32_t carry_s = 0, carry_e = 0;
                for (uint32_t b = 0; b < K; b += HGT_WG) {
                    const uint32_t i = b + tid;
                    uint32_t m = i < K ? nl_msh[i] : 0;
                    if (m < 2) m = 0;
                    uint32_t tot_s, tot_e;
                    const uint32_t ex_s = wg_scan_u32(m, sh.ws, &tot_s);
                    const uint32_t ex_e = wg_scan_u32(m * (m - 1) / 2, sh.ws, &tot_e);
                    if (i < K) {
                        off[i] = carry_s + ex_s;
                        eoff[i] = carry_e + ex_e;
                        cur[i] = 0;
                    }
                    carry_s += tot_s;
                    carry_e += tot_e;
                }
                if (tid == 0) {
                    off[K] = carry_s;
                    eoff[K] = carry_e;
                }
            }
            __syncthreads();
            // runs: shared vertices per neighbour, long runs listed, short runs enumerated
            for (uint32_t i = tid; i < W; i += HGT_WG) {
                const uint64_t ki = keys[i];
                const uint64_t v = ki >> KEY_V;
                const uint32_t st0 = lower_bound_u64(keys, W, v << KEY_V);
                const uint32_t en = lower_bound_u64(keys, W, (v + 1) << KEY_V);
                const uint32_t R = en - st0;
                if (R < 2) continue;
                const uint32_t xi = (uint32_t)ki & K_MAX;
                if (nl_msh[xi] >= 2) sl[off[xi] + atomicAdd(&cur[xi], 1u)] = st0;
                if (R > RUN_DIRECT) {
                    if (i == st0) {
                        const uint32_t q = atomicAdd(&sh.nbig, 1u);
                        big[2 * q] = st0;
                        big[2 * q + 1] = R;
                    }
                    continue;
                }
                const uint32_t mx = nl_meta[xi];
                if (!meta_elig(mx)) continue;
                const uint32_t vin = (uint32_t)(ki >> KEY_IN) & 1u;
                const uint32_t xl = meta_len(mx), cx = meta_c(mx), dx = hlen - cx;
                const uint32_t ob = (hlen > cx ? 1u : 0u) | 24u | (xl - cx > 1 ? 2u : 0u);
                // partners counted per (gy, rng) cell in 6-bit fields (a run holds at most 63)
                uint32_t n_el = 0, n_big = 0;
                uint64_t c_lo = 0, c_hi = 0;  // cells 0..9, 10..11
                for (uint32_t j = st0; j < en; j++) {
                    if (j == i) continue;
                    const uint32_t my = nl_meta[(uint32_t)keys[j] & K_MAX];
                    if (!meta_elig(my)) continue;
                    const uint32_t yl = meta_len(my), cy = meta_c(my);
                    n_el++;
                    n_big += yl > 1 ? 1u : 0u;
                    const uint32_t cell = single_gy(vin, yl, cy) * 3u + (cy < dx ? 0u : (cy == dx ? 1u : 2u));
                    if (cell < 10) c_lo += 1ull << (6 * cell);
                    else c_hi += 1ull << (6 * (cell - 10));
                }
                if (n_big) acc32_add(myacc32, T.he[ob | 4u], 0u - n_big);
                if (n_el > n_big) acc32_add(myacc32, T.he[ob], 0u - (n_el - n_big));
                for (uint32_t cell = 0; cell < 12; cell++) {
                    const uint32_t n = (uint32_t)((cell < 10 ? c_lo >> (6 * cell) : c_hi >> (6 * (cell - 10))) & 63u);
                    if (!n) continue;
                    int ct, cf;
                    single_codes(vin, xl, cx, cell / 3u, cell % 3u, ct, cf);
                    const int c1 = T.he[ct], c2 = T.he[cf];
                    if (c1 != c2) {
                        if (c1 < 255) atomicAdd((unsigned long long*)&cacc[c1], (unsigned long long)n);
                        if (c2 < 255) atomicAdd((unsigned long long*)&cacc[c2], 0ull - (unsigned long long)n);
                    }
                }
            }
            __syncthreads();
            HE2_MARK(8);
            // vertex pairs (u, w), u < w, of each neighbour's shared vertices, as run starts
            for (uint32_t a = tid; a < S; a += HGT_WG) {
                const uint32_t x = seg_of<uint32_t>(off, K, a);
                const uint32_t o = off[x], m = off[x + 1] - o, j = a - o;
                uint32_t pos = eoff[x] + j * (m - 1) - j * (j - 1) / 2;
                const uint32_t u = sl[a];
                for (uint32_t q = j + 1; q < m; q++) {
                    const uint32_t w = sl[o + q];
                    const uint32_t lo = u < w ? u : w, hi = u < w ? w : u;
                    emit[pos++] = ((uint64_t)lo << EMIT_LO) | ((uint64_t)hi << EMIT_HI) | x;
                }
            }
            __syncthreads();
            sort_any(emit, E2);
            HE2_MARK(9);
            // long runs, one at a time: histogram over (gy, c_y) of the eligible members
            const uint32_t nbig = sh.nbig;
            if (P.stats && tid == 0 && nbig) atomicAdd((unsigned long long*)&P.stats[ST_AGG_LONG], (unsigned long long)nbig);
            for (uint32_t r = 0; r < nbig; r++) {
                const uint32_t st0 = big[2 * r], R = big[2 * r + 1];
                const uint32_t vin = (uint32_t)(keys[st0] >> KEY_IN) & 1u;
                for (uint32_t c = tid; c < n_hist; c += HGT_WG) hist[c] = 0;
                if (tid == 0) sh.nb1 = 0;
                __syncthreads();
                for (uint32_t i = st0 + tid; i < st0 + R; i += HGT_WG) {
                    const uint32_t my = nl_meta[(uint32_t)keys[i] & K_MAX];
                    if (!meta_elig(my)) continue;
                    const uint32_t yl = meta_len(my), cy = meta_c(my);
                    if (yl > 1) atomicAdd(&sh.nb1, 1u);
                    atomicAdd(&hist[single_gy(vin, yl, cy) * (hlen + 1) + cy], 1u);
                }
                __syncthreads();
                {  // inclusive prefix over the rows laid end to end
                    uint32_t carry = 0;
                    for (uint32_t b = 0; b < n_hist; b += HGT_WG) {
                        const uint32_t i = b + tid;
                        const uint32_t v = i < n_hist ? hist[i] : 0;
                        uint32_t tot;
                        const uint32_t ex = wg_scan_u32(v, sh.ws, &tot);
                        if (i < n_hist) hist[i] = carry + ex + v;
                        carry += tot;
                    }
                }
                __syncthreads();
                const uint32_t nb1 = sh.nb1, ne = hist[n_hist - 1];  // eligible members: of length > 1, all
                for (uint32_t i = st0 + tid; i < st0 + R; i += HGT_WG) {
                    const uint32_t mx = nl_meta[(uint32_t)keys[i] & K_MAX];
                    if (!meta_elig(mx)) continue;
                    const uint32_t xl = meta_len(mx), cx = meta_c(mx), dx = hlen - cx;
                    const uint32_t ob = (hlen > cx ? 1u : 0u) | 24u | (xl - cx > 1 ? 2u : 0u);
                    const uint64_t n_big = nb1 - (xl > 1 ? 1u : 0u), n_small = (uint64_t)(ne - 1) - n_big;
                    if (n_big) acc_add(cacc, T.he[ob | 4u], 2 * (0ull - n_big));
                    if (n_small) acc_add(cacc, T.he[ob], 2 * (0ull - n_small));
                    const uint32_t gx = single_gy(vin, xl, cx);
                    for (uint32_t g = 0; g < 4; g++) {
                        const uint32_t row = g * (hlen + 1);
                        const uint32_t before = hist[row];  // the rows before (nothing at c_y = 0)
                        const uint32_t tot = hist[row + hlen] - before;
                        uint32_t n3[3];
                        n3[0] = dx >= 2 ? hist[row + dx - 1] - before : 0u;
                        n3[1] = dx >= 1 ? hist[row + dx] - hist[row + dx - 1] : 0u;
                        n3[2] = tot - n3[0] - n3[1];
                        if (g == gx) n3[cx < dx ? 0 : (cx == dx ? 1 : 2)]--;  // x itself
                        for (uint32_t rng = 0; rng < 3; rng++) {
                            if (!n3[rng]) continue;
                            int ct, cf;
                            single_codes(vin, xl, cx, g, rng, ct, cf);
                            const int c1 = T.he[ct], c2 = T.he[cf];
                            if (c1 != c2) {
                                if (c1 < 255) atomicAdd((unsigned long long*)&cacc[c1], (unsigned long long)n3[rng]);
                                if (c2 < 255) atomicAdd((unsigned long long*)&cacc[c2], 0ull - (unsigned long long)n3[rng]);
                            }
                        }
                    }
                }
                __syncthreads();
            }
            HE2_MARK(10);
            // pairs sharing two or more vertices, at their two smallest common ones.  The
            // pairs within every run of equal (u, w) are numbered in one index space
            // (pp: exclusive prefix of the run heads' pair counts), so that a long run
            // spreads over the whole workgroup.
            uint32_t* pp = (uint32_t*)(emit + E2);
            if (tid == 0) sh.g[5] = 0;
            __syncthreads();
            {
                uint32_t carry = 0;
                for (uint32_t b = 0; b < E2; b += HGT_WG) {
                    const uint32_t i = b + tid;
                    uint32_t c = 0;
                    if (i < E2) {
                        const uint64_t uw = emit[i] >> EMIT_HI;
                        if (i == 0 || (emit[i - 1] >> EMIT_HI) != uw) {
                            const uint64_t R = lower_bound_u64(emit, E2, (uw + 1) << EMIT_HI) - i;
                            const uint64_t c64 = R * (R - 1) / 2;
                            atomicAdd((unsigned long long*)&sh.g[5], (unsigned long long)c64);
                            c = (uint32_t)c64;  // used only when the total fits 31 bits
                        }
                    }
                    uint32_t tot;
                    const uint32_t ex = wg_scan_u32(c, sh.ws, &tot);
                    if (i < E2) pp[i] = carry + ex;
                    carry += tot;
                }
            }
            __syncthreads();
            const uint64_t T2 = sh.g[5];
            if (T2 < 0x80000000ull) {
                for (uint32_t p = tid; p < (uint32_t)T2; p += HGT_WG) {
                    const uint32_t i = seg_of<uint32_t>(pp, E2, p);  // the run's head
                    const uint64_t uw = emit[i] >> EMIT_HI;
                    const uint32_t R = lower_bound_u64(emit, E2, (uw + 1) << EMIT_HI) - i;
                    uint32_t a, b;
                    tri_decode(R, p - pp[i], a, b);
                    multi_pair(G.g, T, hlen, hm, keys, nl_x, nl_meta, emit[i + a], emit[i + b], P.stats, myacc32);
                }
            } else {
                for (uint32_t i = tid; i < E2; i += HGT_WG) {
                    const uint64_t uw = emit[i] >> EMIT_HI;
                    for (uint32_t j = i + 1; j < E2 && (emit[j] >> EMIT_HI) == uw; j++)
                        multi_pair(G.g, T, hlen, hm, keys, nl_x, nl_meta, emit[i], emit[j], P.stats, myacc32);
                }
            }
        } else {
        // --- intersecting neighbour pairs, enumerated: the neighbours that meet at a vertex v
        // form a run of the sorted keys and every pair of a run meets at v; a pair whose
        // sides share several vertices is counted at its smallest common vertex (found by
        // merging the two rows).
            for (uint32_t i = tid; i + 1 < W; i += HGT_WG) {
                const uint64_t ki = keys[i];
                const uint64_t v = ki >> KEY_V;
                if ((keys[i + 1] >> KEY_V) != v) continue;
                const uint32_t xi = (uint32_t)ki & K_MAX;
                const uint32_t vin = (uint32_t)(ki >> KEY_IN) & 1u;
                const uint32_t xsh = nl_msh[xi];
                for (uint32_t j = i + 1; j < W; j++) {
                    const uint64_t kj = keys[j];
                    if ((kj >> KEY_V) != v) break;
                    const uint32_t yi = (uint32_t)kj & K_MAX;
                    uint32_t sc = 1, shh = vin;
                    if (xsh > 1 && nl_msh[yi] > 1) {
                        uint32_t first;
                        row_meet(G.g.h2v + G.g.h_off[nl_x[xi]], meta_len(nl_meta[xi]), G.g.h2v + G.g.h_off[nl_x[yi]],
                                 meta_len(nl_meta[yi]), hm, hlen, sc, shh, first);
                        if ((uint64_t)first != v) continue;
                    }
                    pair_class(P, T, h, hlen, nl_x, nl_meta, xi, yi, sc, shh, myacc32);
                }
            }
        }  // aggregated or enumerated pairs
        __syncthreads();
        // fold the per-centre 32-bit pair counters (signed) into the 64-bit ones
        for (uint32_t i = tid; i < NWAVE * HGT_N_HE_CLASSES; i += HGT_WG) {
            int32_t v = (int32_t)acc32_all[i];
            if (v) {
                atomicAdd((unsigned long long*)&acc_all[i], (unsigned long long)(int64_t)v);
                acc32_all[i] = 0;
            }
        }
        {  // the doubled changes: over all waves, halved
            for (uint32_t c = tid; c < HGT_N_HE_CLASSES; c += HGT_WG) {
                int64_t s2 = 0;
                for (int w = 0; w < NWAVE; w++) {
                    s2 += (int64_t)sh.acc2[w * HGT_N_HE_CLASSES + c];
                    sh.acc2[w * HGT_N_HE_CLASSES + c] = 0;
                }
                if (s2) atomicAdd((unsigned long long*)&acc_all[c], (unsigned long long)(s2 / 2));
            }
        }
        __syncthreads();
        HE2_MARK(6);
        // the longest centre this workgroup finished (slot HE2_PHASES - 1 holds a maximum)
        if (P.phase_ticks && tid == 0 && t_mark - t_centre > ph[HE2_PHASES - 1]) ph[HE2_PHASES - 1] = t_mark - t_centre;
    }
#undef HE2_MARK
}

template <int STAGE>
__device__ void he2_flush_stats(const He2Params& P, const uint64_t* st, const uint64_t* ph) {
    if (P.phase_ticks && threadIdx.x < HE2_PHASES - 1 && ph[threadIdx.x])
        atomicAdd((unsigned long long*)&P.stats[ST_PH0 + HE2_PHASES * STAGE + threadIdx.x],
                  (unsigned long long)ph[threadIdx.x]);
    if (P.phase_ticks && threadIdx.x == HE2_PHASES - 1 && ph[threadIdx.x])
        atomicMax((unsigned long long*)&P.stats[ST_PH0 + HE2_PHASES * STAGE + threadIdx.x],
                  (unsigned long long)ph[threadIdx.x]);
    if (P.stats && threadIdx.x == 0 && st[0])
        atomicAdd((unsigned long long*)&P.stats[ST_DEFER0 + STAGE], (unsigned long long)st[0]);
    if (P.stats && threadIdx.x == 0 && st[1])
        atomicAdd((unsigned long long*)&P.stats[ST_HEB0 + STAGE], (unsigned long long)st[1]);
}

#define HE2_PROLOGUE                                                                   \
    __shared__ Sh2 sh;                                                                 \
    __shared__ Tables T;                                                               \
    __shared__ uint64_t acc[NWAVE][HGT_N_HE_CLASSES];                                  \
    __shared__ uint32_t acc32[NWAVE][HGT_N_HE_CLASSES];                                \
    __shared__ uint64_t st[2];                                                         \
    __shared__ uint64_t ph[HE2_PHASES];                                                \
    if (threadIdx.x < HE2_PHASES) ph[threadIdx.x] = 0;                                 \
    if (threadIdx.x == 0) sh.cur_g = 0xffffffffu;                                      \
    for (int i = threadIdx.x; i < 128; i += HGT_WG) T.he[i] = P.he_tab[i];             \
    for (int i = threadIdx.x; i < NWAVE * HGT_N_HE_CLASSES; i += HGT_WG) {             \
        (&acc[0][0])[i] = 0;                                                           \
        (&acc32[0][0])[i] = 0;                                                         \
    }                                                                                  \
    if (threadIdx.x < 2) st[threadIdx.x] = 0;                                          \
    for (int i = threadIdx.x; i < NWAVE * HGT_N_HE_CLASSES; i += HGT_WG) sh.acc2[i] = 0; \
    __syncthreads();

__global__ void __launch_bounds__(HGT_WG) k_he2_s0(He2Params P) {
    __shared__ __attribute__((aligned(16))) uint32_t arena[ARENA_S];
    HE2_PROLOGUE
    he2_body<0>(P, arena, ARENA_S, sh, T, &acc[0][0], &acc32[0][0], st, ph, nullptr);
    he2_flush_graph(P, sh.cur_g, &acc[0][0]);
    he2_flush_stats<0>(P, st, ph);
}

__global__ void __launch_bounds__(HGT_WG) k_he2_s1(He2Params P) {
    __shared__ __attribute__((aligned(16))) uint32_t arena[ARENA_M];
    HE2_PROLOGUE
    he2_body<1>(P, arena, ARENA_M, sh, T, &acc[0][0], &acc32[0][0], st, ph, nullptr);
    he2_flush_graph(P, sh.cur_g, &acc[0][0]);
    he2_flush_stats<1>(P, st, ph);
}

__global__ void __launch_bounds__(HGT_WG) k_he2_s2(He2Params P) {
    __shared__ uint64_t tile[TILE_K];
    HE2_PROLOGUE
    he2_body<2>(P, P.garena + (uint64_t)blockIdx.x * P.garena_words, (uint32_t)P.garena_words, sh, T, &acc[0][0],
                &acc32[0][0], st, ph, tile);
    he2_flush_graph(P, sh.cur_g, &acc[0][0]);
    he2_flush_stats<2>(P, st, ph);
}

}  // namespace

void he2_nbr_launch(NbrParams& P, unsigned grid_small, unsigned grid_big, hipStream_t s) {
    hgt_fill_u32(P.queue, 0, 3, s);
    hgt_fill_u64(P.n_entries, 0, 1, s);
    if (P.M.total == 0) return;
    if (P.inserting) k_h_clear<<<(unsigned)((P.M.total * 64 + 255) / 256), 256, 0, s>>>(P.M);
    k_nbr_small<<<grid_small, HGT_WG, 0, s>>>(P);
    k_nbr_big<<<grid_big, HGT_WG, 0, s>>>(P);
    k_entries_check<<<1, 256, 0, s>>>(P.M, P.n_entries, P.entries_cap);
}

void he2_lists_build(NbrParams& P, uint64_t* bl_cnt, uint64_t* bl_off, uint64_t* bl_cur, uint32_t* bl_d,
                     uint64_t* bl_pay, void* scan_tmp, hipStream_t s) {
    const uint64_t n_ids = P.M.total_ids;
    hgt_fill_u64(bl_cnt, 0, n_ids, s);
    unsigned g = 2048;
    k_bl_count<<<g, 256, 0, s>>>(P.n_entries, P.entries_cap, P.ent_x, bl_cnt);
    hgt_scan_u64(bl_cnt, bl_off, n_ids, nullptr, nullptr, scan_tmp, s);
    (void)hipMemcpyAsync(bl_cur, bl_off, n_ids * 8, hipMemcpyDeviceToDevice, s);
    k_bl_scatter<<<g, 256, 0, s>>>(P.n_entries, P.entries_cap, P.ent_x, P.ent_d, P.ent_pay, bl_cur, bl_d, bl_pay);
}

void he2_remove_deleted(NbrParams& P, hipStream_t s) {
    if (P.M.total == 0) return;
    k_h_remove<<<2048, 256, 0, s>>>(P.M, P.n_entries, P.entries_cap, P.ent_x, P.ent_pay);
}

void he2_launch_stage(He2Params& P, int stage, unsigned grid, hipStream_t s) {
    if (!P.M.total) return;
    if (stage == 0) k_he2_s0<<<grid, HGT_WG, 0, s>>>(P);
    else if (stage == 1) k_he2_s1<<<grid, HGT_WG, 0, s>>>(P);
    else k_he2_s2<<<grid, HGT_WG, 0, s>>>(P);
}
