// triad_he.hip -- hyperedge-based and temporal triad deltas (Alg. 3, steps 2 and 5).
//
// For a set of changed hyperedges C (the deleted ones on the old graph, or the
// inserted ones on the new graph) the kernels count, per class, every triad
// that contains at least one member of C, each exactly once: a triad is
// counted at its member of C with the smallest batch rank.  This is the exact
// form of Alg. 3's affected-region count; count_new - count_old over these
// triads is the change of the full count.
//
// The triads that contain a centre h are {h,x,y} with
//   (i)  x, y both line-graph neighbours of h, and
//   (ii) x a neighbour of h, y a neighbour of x that is neither h nor meets h.
// Work per centre h (one 256-thread workgroup):
//   1. N(h) with c_x = |h & x| is built in an open-addressing hash from the
//      incidence lists of h's members (coalesced segment reads).
//   2. Pairs of type (i) are first all classified as if x and y were disjoint;
//      for the hyperedge family this depends only on (c_x, |x| > c_x) of each
//      side and on c_x + c_y < |h|, so a histogram over c gives every class
//      count in O(|N(h)| + |h|).  The temporal family (window-limited, few
//      pairs) enumerates these pairs directly.
//   3. Each wave takes neighbours x and gathers the incidence lists of x's
//      members into a wave-private LDS hash (y -> |x & y|, |h & x & y|).
//      Every y found there is an intersecting pair: if y is in N(h) the pair's
//      class from step 2 is replaced by its true class; otherwise {h,x,y} is a
//      type (ii) path.
// Class counts are accumulated in LDS (u64, modular) and flushed once per
// workgroup.  Centres whose neighbourhood does not fit the LDS tables are
// deferred to a second kernel that keeps the same tables in global scratch.
#include "triad_common.h"

namespace {

using namespace tri;
// small-centre (LDS) configuration
constexpr uint32_t S_LH = 1024;        // max sum of member degrees
constexpr uint32_t S_NH = 2048;        // N(h) hash slots
constexpr uint32_t S_WAREA = 4096;     // u32 words shared area (per-wave hashes alias it)
constexpr uint32_t WH_SLOTS = 512;     // per-wave 2-hop hash slots
constexpr uint32_t WH_MAX_L = WH_SLOTS / 2;
constexpr uint32_t CHUNK = 64;

// Per-wave member info of the neighbour x being expanded.
struct WaveMem {
    uint32_t pre[CHUNK + 1];
    uint64_t voff[CHUNK];
    uint32_t inh[CHUNK];
};

// Storage of one workgroup (LDS for the small kernel, global for the big one).
struct WgStore {
    uint32_t* nh_keys;
    uint32_t* nh_vals;
    uint32_t* hm;      // members of h
    uint32_t* nl_x;    // compacted N(h)
    uint32_t* nl_meta;
    uint32_t* warea;   // shared area
    uint64_t warea_words;
    uint32_t* wh;      // per-wave 2-hop hashes (NWAVE * 2 * WH_SLOTS words)
};

struct Shared {
    uint32_t h, rank, hlen, lh, K, Kt, defer, stop;
    uint32_t slice, nslice;  // this workgroup's share of the centre: neighbours slice, slice + nslice, ...
    uint32_t gi, cur_g, skip;
    uint64_t hoff;
    int64_t th;
    uint64_t sh;
    uint32_t ws[NWAVE];
    uint64_t g[8];
};

// The slice of a sliced centre that owns neighbour x (a property of x alone, so
// every slice, whatever order its lists come in, agrees on it).
__device__ __forceinline__ uint32_t slice_of(uint32_t x, uint32_t nslice) {
    return (uint32_t)(((uint64_t)(x * 2654435761u) * nslice) >> 32);
}

// classify the intersecting pair (x, y) found in x's 2-hop lists
__device__ __forceinline__ void classify(const TriadParams& P, const HeGraph& G, const Tables& T, const WgStore& S,
                                         const Shared& sh,
                                         uint32_t nh_log, uint32_t x, uint32_t meta_x, int64_t tx, uint64_t sx,
                                         uint32_t y, uint32_t cxy, uint32_t chxy, uint64_t* acc_he, uint64_t* acc_tmp) {
    const int nh = (int)sh.hlen;
    const int nx = (int)meta_len(meta_x), hx = (int)meta_c(meta_x);
    uint32_t slot = hash_find(S.nh_keys, nh_log, y);
    if (slot != HGT_EMPTY) {
        // (i) both neighbours of h and intersecting: replace the disjoint-pair class
        if (x > y) return;
        uint32_t my = __atomic_load_n(&S.nh_vals[slot], __ATOMIC_RELAXED);
        if (!meta_elig(my)) return;
        const int ny = (int)meta_len(my), hy = (int)meta_c(my);
        if (P.do_he && P.static_he) {
            // full count: a closed triple only at its smallest-ID centre
            acc_add(acc_he, T.he[venn_code(nh, nx, ny, hx, 0, hy, 0)], ~0ull);
            if (sh.h < x && sh.h < y) acc_add(acc_he, T.he[venn_code(nh, nx, ny, hx, (int)cxy, hy, (int)chxy)], 1);
        } else if (P.do_he) {
            int ct = T.he[venn_code(nh, nx, ny, hx, (int)cxy, hy, (int)chxy)];
            int cf = T.he[venn_code(nh, nx, ny, hx, 0, hy, 0)];
            if (ct != cf) {
                acc_add(acc_he, ct, 1);
                acc_add(acc_he, cf, ~0ull);
            }
        }
        if (P.do_tmp && meta_win(meta_x) && meta_win(my)) {
            int64_t ty = G.g.h_ts[y];
            if (within(sh.th, tx, ty, G.window)) {
                const uint64_t sy = (ty == sh.th || ty == tx) ? G.g.h_seq[y] : 0;  // only ties need it
                int ct = T.tmp[time_code(sh.th, sh.sh, tx, sx, ty, sy, nh, nx, ny, hx, (int)cxy, hy, (int)chxy)];
                int cf = T.tmp[time_code(sh.th, sh.sh, tx, sx, ty, sy, nh, nx, ny, hx, 0, hy, 0)];
                if (ct != cf) {
                    acc_add(acc_tmp, ct, 1);
                    acc_add(acc_tmp, cf, ~0ull);
                }
            }
        }
        return;
    }
    // (ii) path h - x - y with y outside the closed neighbourhood of h (its centre is x)
    if (P.static_he) return;
    if (lower_ranked_member(G.mark[y], G.epoch, sh.rank)) return;
    int64_t ty = 0;
    if (P.do_tmp) {
        ty = G.g.h_ts[y];
        if (!P.do_he && !within(sh.th, tx, ty, G.window)) return;
    }
    const int ny = (int)G.g.h_len[y];
    if (P.do_he) acc_add(acc_he, T.he[venn_code(nh, nx, ny, hx, (int)cxy, 0, 0)], 1);
    if (P.do_tmp && meta_win(meta_x) && within(sh.th, tx, ty, G.window)) {
        const uint64_t sy = (ty == sh.th || ty == tx) ? G.g.h_seq[y] : 0;  // only ties need it
        acc_add(acc_tmp, T.tmp[time_code(sh.th, sh.sh, tx, sx, ty, sy, nh, nx, ny, hx, (int)cxy, 0, 0)], 1);
    }
}

// Member lists of x's members in chunks of CHUNK: per lane member its list
// offset, whether it lies in h, and the prefix of the list lengths in wm.pre.
__device__ __forceinline__ uint32_t chunk_lists(const HeGraph& G, const WgStore& S, const Shared& sh, WaveMem& wm,
                                                uint64_t xoff, uint32_t b, uint32_t cnt, bool with_inh) {
    const int lane = threadIdx.x & 63;
    uint32_t d = 0;
    if ((uint32_t)lane < cnt) {
        uint32_t m = G.g.h2v[xoff + b + lane];
        wm.voff[lane] = G.g.v_off[m];
        d = G.g.v_len[m];
        if (with_inh) wm.inh[lane] = contains_u32(S.hm, sh.hlen, m) ? 1u : 0u;
    }
    uint32_t inc = d;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    if ((uint32_t)lane < cnt) wm.pre[lane + 1] = inc;
    if (lane == 0) wm.pre[0] = 0;
    wave_sync();
    return wm.pre[cnt];
}

// Expand neighbour x of the current centre (one wave): every y sharing a vertex
// with x, with |x & y| and |x & y & h|, from the member lists of x.  For the
// temporal family only y within the window of both h and x can complete a
// triad (then the span of {h, x, y} is within the window too), so the other
// list entries are dropped by their timestamp before hashing.
__device__ void expand_x(const TriadParams& P, const HeGraph& G, const Tables& T, const WgStore& S, const Shared& sh,
                         uint32_t nh_log,
                         WaveMem& wm, uint32_t* wkeys, uint32_t* wvals, uint32_t x, uint32_t meta_x, uint64_t* acc_he,
                         uint64_t* acc_tmp, uint64_t* acc_st) {
    const int lane = threadIdx.x & 63;
    const uint32_t nx = meta_len(meta_x);
    const uint64_t xoff = G.g.h_off[x];
    int64_t tx = 0;
    uint64_t sx = 0;
    if (P.do_tmp) {
        tx = G.g.h_ts[x];
        sx = G.g.h_seq[x];
    }
    const bool win = P.do_tmp && G.g.v2h_ts;
    const int64_t w_lo = ts_sub(sh.th > tx ? sh.th : tx, G.window), w_hi = ts_add(sh.th < tx ? sh.th : tx, G.window);
    auto in_win = [&](uint64_t at) {
        const int64_t t = G.g.v2h_ts[at];
        return t >= w_lo && t <= w_hi;
    };
    // total length of the member lists, then (temporal) the entries within the window
    uint32_t lx_all = 0;
    for (uint32_t b = 0; b < nx; b += CHUNK) {
        uint32_t d = 0;
        if (b + lane < nx) d = G.g.v_len[G.g.h2v[xoff + b + lane]];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o, 64);
        lx_all += d;
    }
    uint32_t lx = lx_all;
    if (win && lx_all > WH_MAX_L) {
        lx = 0;
        for (uint32_t b = 0; b < nx; b += CHUNK) {
            const uint32_t cnt = nx - b < CHUNK ? nx - b : CHUNK;
            const uint32_t len = chunk_lists(G, S, sh, wm, xoff, b, cnt, false);
            uint32_t c = 0;
            for (uint32_t p = lane; p < len; p += 64) {
                uint32_t k = seg_of<uint32_t>(wm.pre, cnt, p);
                c += in_win(wm.voff[k] + (p - wm.pre[k])) ? 1u : 0u;
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
            lx += c;
            wave_sync();
        }
    }
    if (lane == 0 && P.stats) {
        // x's row, its members' lists (and their timestamps when filtered)
        atomicAdd((unsigned long long*)&acc_st[0], (unsigned long long)(4ull * nx + (win ? 12ull : 4ull) * lx_all));
        atomicAdd((unsigned long long*)&acc_st[3], 1ull);
    }
    // The hash lives in LDS for short lists.  Longer ones use the wave's slice of
    // global memory, filled in passes: pass (m, r) takes the y whose part hash is
    // r modulo m, so each y, with all its occurrences, falls in exactly one pass.
    // A pass whose table overflows is dropped before anything is classified and
    // split in two (modulus doubled), so no y is counted twice.
    const bool lds = lx <= WH_MAX_L || !P.wave_hash;
    uint32_t* hk = wkeys;
    uint32_t* hv = wvals;
    uint32_t cap, mod = 1;
    if (lds) {
        cap = (uint32_t)pow2ceil64(2 * (uint64_t)lx < 64 ? 64 : 2 * (uint64_t)lx);
        if (cap > WH_SLOTS) cap = WH_SLOTS;  // only without a global slice (then passes split the y)
    } else {
        const int wave = threadIdx.x >> 6;
        hk = P.wave_hash + ((uint64_t)blockIdx.x * NWAVE + wave) * 2ull * P.wave_slots;
        hv = hk + P.wave_slots;
        cap = (uint32_t)pow2ceil64(2 * (uint64_t)lx);
        if (cap > P.wave_slots) cap = P.wave_slots;
    }
    // parts of at most half the table each: one pass whenever the table holds 2 lx slots
    while ((uint64_t)mod * (cap / 2) < lx) mod <<= 1;
    if (mod > 1 && lane == 0 && P.stats) atomicAdd((unsigned long long*)&acc_st[2], 1ull);
    const uint32_t log_cap = log2u64(cap);
    constexpr int kStack = 48;
    uint32_t st_m[kStack], st_r[kStack];
    for (uint32_t r0 = 0; r0 < mod; r0++) {
        int sp = 0;
        st_m[sp] = mod;
        st_r[sp++] = r0;
        while (sp > 0) {
            --sp;
            const uint32_t m = st_m[sp], r = st_r[sp];
            for (uint32_t s = lane; s < cap; s += 64) { hk[s] = HGT_EMPTY; hv[s] = 0; }
            wave_sync();
            bool fail = false;
            for (uint32_t b = 0; b < nx; b += CHUNK) {
                const uint32_t cnt = nx - b < CHUNK ? nx - b : CHUNK;
                const uint32_t len = chunk_lists(G, S, sh, wm, xoff, b, cnt, true);
                for (uint32_t p = lane; p < len; p += 64) {
                    uint32_t k = seg_of<uint32_t>(wm.pre, cnt, p);
                    const uint64_t at = wm.voff[k] + (p - wm.pre[k]);
                    if (win && !in_win(at)) continue;
                    uint32_t y = G.g.v2h[at];
                    if (y == x || y == sh.h) continue;
                    if (m > 1 && (part_hash(y) & (m - 1)) != r) continue;
                    if (!hash_add_ok(hk, hv, log_cap, y, 1u + (wm.inh[k] << 16))) fail = true;
                }
                wave_sync();
            }
            if (__any(fail)) {
                if (sp + 2 > kStack) {  // cannot happen for tables of at least 64 slots
                    if (lane == 0) set_status(const_cast<int32_t*>(G.status), HGT_EDEVICE);
                    return;
                }
                st_m[sp] = 2 * m;
                st_r[sp++] = r + m;
                st_m[sp] = 2 * m;
                st_r[sp++] = r;
                continue;
            }
            for (uint32_t s = lane; s < cap; s += 64) {
                uint32_t y = __atomic_load_n(&hk[s], __ATOMIC_RELAXED);
                if (y != HGT_EMPTY) {
                    uint32_t v = __atomic_load_n(&hv[s], __ATOMIC_RELAXED);
                    classify(P, G, T, S, sh, nh_log, x, meta_x, tx, sx, y, v & 0xffffu, v >> 16, acc_he, acc_tmp);
                }
            }
            wave_sync();
        }
    }
}

// Adds the workgroup's counts to graph g's phase accumulators and clears them.
__device__ void flush_counts(const TriadParams& P, uint32_t g, uint64_t* acc_he, uint64_t* acc_tmp) {
    __syncthreads();
    if (g != 0xffffffffu) {
        const HeGraph& G = P.M.graphs[g];
        for (int i = threadIdx.x; i < HGT_N_HE_CLASSES; i += HGT_WG)
            if (acc_he[i]) atomicAdd((unsigned long long*)&G.out_he[i], (unsigned long long)acc_he[i]);
        for (int i = threadIdx.x; i < HGT_N_TEMPORAL_CLASSES; i += HGT_WG)
            if (acc_tmp[i]) atomicAdd((unsigned long long*)&G.out_tmp[i], (unsigned long long)acc_tmp[i]);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < HGT_N_HE_CLASSES; i += HGT_WG) acc_he[i] = 0;
    for (int i = threadIdx.x; i < HGT_N_TEMPORAL_CLASSES; i += HGT_WG) acc_tmp[i] = 0;
    __syncthreads();
}

// The whole per-centre computation; BIG selects global tables and no deferral.
template <bool BIG>
__device__ void run_centres(const TriadParams& P, const Tables& T, const WgStore& S, Shared& sh, WaveMem* wmem,
                            uint64_t* acc_he, uint64_t* acc_tmp, uint64_t* acc_st, uint32_t lh_limit, uint32_t hm_cap) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (;;) {
        if (tid == 0) {
            const bool sliced = BIG && P.slice_pre;
            uint64_t n = sliced ? P.slice_pre[P.slice_cap + 1] : BIG ? (uint64_t)*P.big_count : P.M.total;
            uint32_t c = atomicAdd(BIG ? P.big_queue : P.queue, 1u);
            sh.stop = c >= n;
            sh.slice = 0;
            sh.nslice = 1;
            if (!sh.stop && sliced) {  // slice c of the deferred centres' slices
                const uint64_t nc = P.slice_pre[P.slice_cap];
                const uint32_t ci = seg_of<uint64_t>(P.slice_pre, (uint32_t)nc, c);
                const uint64_t first = P.slice_pre[ci];
                const uint64_t next = ci + 1 < nc ? P.slice_pre[ci + 1] : n;
                sh.slice = (uint32_t)(c - first);
                sh.nslice = (uint32_t)(next - first);
                c = ci;
            }
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
                if (P.do_tmp) {
                    sh.th = Gq.g.h_ts[h];
                    sh.sh = Gq.g.h_seq[h];
                }
                sh.defer = (!BIG && sh.hlen > hm_cap) ? 1u : 0u;
            }
        }
        __syncthreads();
        if (sh.stop) break;
        if (sh.gi != sh.cur_g) {  // results so far belong to the previous graph
            flush_counts(P, sh.cur_g, acc_he, acc_tmp);
            if (tid == 0) sh.cur_g = sh.gi;
            __syncthreads();
        }
        if (sh.skip) {
            __syncthreads();
            continue;
        }
        const HeGraph& G = P.M.graphs[sh.gi];
        if (sh.defer) {
            if (tid == 0) {
                uint32_t q = atomicAdd(P.big_count, 1u);
                P.big_list[q] = item_of(sh.gi, sh.h);
                P.big_rank[q] = sh.rank;
                if (P.stats) atomicAdd((unsigned long long*)&acc_st[1], 1ull);
            }
            __syncthreads();
            continue;
        }
        const uint32_t hlen = sh.hlen, h = sh.h;
        // members of h, their degrees and list offsets (prefix in warea)
        uint32_t* pre = S.warea;                                  // hlen + 1 words
        uint64_t* voff = (uint64_t*)(S.warea + ((hlen + 2) & ~1u));  // hlen u64, 8-byte aligned
        uint32_t carry = 0;
        for (uint32_t b = 0; b < hlen; b += HGT_WG) {
            uint32_t i = b + tid, d = 0;
            if (i < hlen) {
                uint32_t m = G.g.h2v[sh.hoff + i];
                S.hm[i] = m;
                voff[i] = G.g.v_off[m];
                d = G.g.v_len[m];
            }
            uint32_t tot;
            uint32_t ex = wg_scan_u32(d, sh.ws, &tot);
            if (i < hlen) pre[i] = carry + ex;
            carry += tot;
        }
        if (tid == 0) {
            pre[hlen] = carry;
            sh.lh = carry;
            sh.defer = (!BIG && carry > lh_limit) ? 1u : 0u;
        }
        __syncthreads();
        if (sh.defer) {
            if (tid == 0) {
                uint32_t q = atomicAdd(P.big_count, 1u);
                P.big_list[q] = item_of(sh.gi, h);
                P.big_rank[q] = sh.rank;
                if (P.stats) atomicAdd((unsigned long long*)&acc_st[1], 1ull);
            }
            __syncthreads();
            continue;
        }
        const uint32_t lh = sh.lh;
        // temporal family: only neighbours within the window of h can share a triad
        // with it; the others are dropped by their timestamp in the lists
        const bool win = P.do_tmp && G.g.v2h_ts;
        const int64_t w_lo = ts_sub(sh.th, G.window), w_hi = ts_add(sh.th, G.window);
        if (tid == 0 && P.stats)
            atomicAdd((unsigned long long*)&acc_st[0], (unsigned long long)(4ull * hlen + (win ? 12ull : 4ull) * lh));
        uint32_t nh_log = log2u64(pow2ceil64(2 * (uint64_t)lh < 64 ? 64 : 2 * (uint64_t)lh));
        uint32_t nh_cap = 1u << nh_log;
        for (uint32_t s = tid; s < nh_cap; s += HGT_WG) { S.nh_keys[s] = HGT_EMPTY; S.nh_vals[s] = 0; }
        if (tid == 0) { sh.K = 0; sh.Kt = 0; }
        __syncthreads();
        // 1. N(h) with c_x
        for (uint32_t p = tid; p < lh; p += HGT_WG) {
            uint32_t k = seg_of<uint32_t>(pre, hlen, p);
            const uint64_t at = voff[k] + (p - pre[k]);
            if (win) {
                const int64_t t = G.g.v2h_ts[at];
                if (t < w_lo || t > w_hi) continue;
            }
            uint32_t x = G.g.v2h[at];
            if (x != h) hash_add(S.nh_keys, S.nh_vals, nh_log, x, 1u);
        }
        __syncthreads();
        // compact, attaching |x|, eligibility and window flags
        for (uint32_t s = tid; s < nh_cap; s += HGT_WG) {
            uint32_t x = __atomic_load_n(&S.nh_keys[s], __ATOMIC_RELAXED);
            if (x == HGT_EMPTY) continue;
            uint32_t c = __atomic_load_n(&S.nh_vals[s], __ATOMIC_RELAXED);
            uint32_t len = G.g.h_len[x];
            bool elig = P.static_he || !lower_ranked_member(G.mark[x], G.epoch, sh.rank);
            bool in_w = true;  // the window filter above already dropped the others
            if (P.do_tmp && !win) {
                int64_t t = G.g.h_ts[x];
                in_w = t >= w_lo && t <= w_hi;
            }
            uint32_t meta = c | (len << 14) | ((uint32_t)elig << 28) | ((uint32_t)in_w << 29);
            S.nh_vals[s] = meta;
            uint32_t q = atomicAdd(&sh.K, 1u);
            S.nl_x[q] = x;
            S.nl_meta[q] = meta;
        }
        __syncthreads();
        const uint32_t K = sh.K;
        const uint32_t slice = sh.slice, nslice = sh.nslice;
        // 2a. hyperedge family: every eligible pair of neighbours classified as disjoint
        // (by the centre's first slice)
        if (P.do_he && slice == 0) {
            uint32_t* cnt = S.warea;  // cnt[f * (hlen + 1) + c]
            const uint32_t W = hlen + 1;
            for (uint32_t i = tid; i < 2 * W; i += HGT_WG) cnt[i] = 0;
            if (tid < 8) sh.g[tid] = 0;
            __syncthreads();
            for (uint32_t i = tid; i < K; i += HGT_WG) {
                uint32_t m = S.nl_meta[i];
                if (!meta_elig(m)) continue;
                uint32_t c = meta_c(m);
                uint32_t f = meta_len(m) > c ? 1u : 0u;
                atomicAdd(&cnt[f * W + c], 1u);
            }
            __syncthreads();
            // exclusive prefix over c for each f (in place) -> number of x with c_x < k
            for (uint32_t f = 0; f < 2; f++) {
                uint32_t carry2 = 0;
                for (uint32_t b = 0; b < W; b += HGT_WG) {
                    uint32_t i = b + tid;
                    uint32_t v = i < W ? cnt[f * W + i] : 0;
                    uint32_t tot;
                    uint32_t ex = wg_scan_u32(v, sh.ws, &tot);
                    if (i < W) cnt[f * W + i] = carry2 + ex;
                    carry2 += tot;
                }
                if (tid == 0) sh.g[6 + f] = carry2;  // N_f
                __syncthreads();
            }
            const uint64_t N0 = sh.g[6], N1 = sh.g[7];
            // S_f(k) = #{x in f : c_x >= k} = N_f - pre_f(k)
            // G(f1,f2) = sum_c n_f1(c) * S_f2(hlen - c)
            uint64_t g00 = 0, g01 = 0, g11 = 0, d0 = 0, d1 = 0;
            for (uint32_t c = 1 + tid; c <= hlen; c += HGT_WG) {
                uint64_t n0 = (uint64_t)((c + 1 < W ? cnt[c + 1] : (uint32_t)N0) - cnt[c]);
                uint64_t n1 = (uint64_t)((c + 1 < W ? cnt[W + c + 1] : (uint32_t)N1) - cnt[W + c]);
                uint32_t k = hlen - c;
                uint64_t s0 = N0 - cnt[k], s1 = N1 - cnt[W + k];
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
                // code bits: 1 h only, 2 x only, 4 y only, 8 h&x only, 32 h&y only
                acc_add(acc_he, T.he[40 | 1], T00 - G00);
                acc_add(acc_he, T.he[40], G00);
                acc_add(acc_he, T.he[40 | 4 | 1], T01 - G01);
                acc_add(acc_he, T.he[40 | 4], G01);
                acc_add(acc_he, T.he[40 | 6 | 1], T11 - G11);
                acc_add(acc_he, T.he[40 | 6], G11);
            }
            __syncthreads();
        }
        // 2b. temporal family: eligible in-window neighbour pairs enumerated directly
        if (P.do_tmp) {
            uint32_t* tl = S.warea;  // 4 words per entry: x, meta, t lo, t hi
            // A sliced centre lists the neighbours that its slice owns first (rows
            // 0 .. Ko-1), the others after them; unsliced, every entry is a row.
            if (nslice > 1) {
                if (tid == 0) sh.g[0] = 0;
                __syncthreads();
                for (uint32_t i = tid; i < K; i += HGT_WG) {
                    const uint32_t m = S.nl_meta[i];
                    if (meta_elig(m) && meta_win(m) && slice_of(S.nl_x[i], nslice) == slice)
                        atomicAdd((unsigned long long*)&sh.g[0], 1ull);
                }
                __syncthreads();
            }
            const uint32_t Ko0 = nslice > 1 ? (uint32_t)sh.g[0] : 0;
            if (tid == 0) sh.g[1] = 0;
            __syncthreads();
            for (uint32_t i = tid; i < K; i += HGT_WG) {
                uint32_t m = S.nl_meta[i];
                if (!meta_elig(m) || !meta_win(m)) continue;
                uint32_t x = S.nl_x[i];
                uint32_t q;
                if (nslice == 1) q = atomicAdd(&sh.Kt, 1u);
                else if (slice_of(x, nslice) == slice) q = (uint32_t)atomicAdd((unsigned long long*)&sh.g[1], 1ull);
                else q = Ko0 + atomicAdd(&sh.Kt, 1u);
                int64_t t = G.g.h_ts[x];
                tl[4 * q] = x;
                tl[4 * q + 1] = m;
                tl[4 * q + 2] = (uint32_t)(uint64_t)t;
                tl[4 * q + 3] = (uint32_t)((uint64_t)t >> 32);
            }
            __syncthreads();
            const uint32_t Kt = sh.Kt + Ko0;
            // Unsliced: pairs (i, j), i < j, over the Kt x Kt square (the lower half is
            // skipped).  Sliced: each unordered pair belongs to the slice that owns its
            // endpoint of smaller ID; rows i < Ko against every j, kept when x_j > x_i.
            const uint64_t rows = nslice == 1 ? Kt : Ko0;
            const uint64_t nsq = rows * Kt;
            for (uint64_t q = tid; q < nsq; q += HGT_WG) {
                uint32_t i, j;
                if (Kt < 65536u) {
                    i = (uint32_t)q / Kt;
                    j = (uint32_t)q - i * Kt;
                } else {
                    i = (uint32_t)(q / Kt);
                    j = (uint32_t)(q - (uint64_t)i * Kt);
                }
                if (nslice == 1 ? j <= i : tl[4 * j] <= tl[4 * i]) continue;
                int64_t ti = (int64_t)((uint64_t)tl[4 * i + 2] | ((uint64_t)tl[4 * i + 3] << 32));
                int64_t tj = (int64_t)((uint64_t)tl[4 * j + 2] | ((uint64_t)tl[4 * j + 3] << 32));
                if (!within(sh.th, ti, tj, G.window)) continue;
                uint32_t mi = tl[4 * i + 1], mj = tl[4 * j + 1];
                // arrival sequences matter only between equal timestamps
                uint64_t si = 0, sj = 0;
                if (ti == tj || ti == sh.th || tj == sh.th) {
                    si = G.g.h_seq[tl[4 * i]];
                    sj = G.g.h_seq[tl[4 * j]];
                }
                int code = time_code(sh.th, sh.sh, ti, si, tj, sj, (int)hlen, (int)meta_len(mi), (int)meta_len(mj),
                                     (int)meta_c(mi), 0, (int)meta_c(mj), 0);
                acc_add(acc_tmp, T.tmp[code], 1);
            }
            __syncthreads();
        }
        // 3. intersecting pairs and paths through each neighbour
        uint32_t* wk = S.wh + (uint64_t)wave * 2 * WH_SLOTS;
        uint32_t* wv = wk + WH_SLOTS;
        for (uint32_t i = wave; i < K; i += NWAVE) {
            uint32_t x = S.nl_x[i];
            uint32_t m = S.nl_meta[i];
            if (!meta_elig(m)) continue;
            if (nslice > 1 && slice_of(x, nslice) != slice) continue;  // another slice's neighbour
            if (!P.do_he && !meta_win(m)) continue;
            expand_x(P, G, T, S, sh, nh_log, wmem[wave], wk, wv, x, m, acc_he, acc_tmp, acc_st);
        }
        __syncthreads();
        (void)lane;
    }
}

__global__ void __launch_bounds__(HGT_WG) k_delta_small(TriadParams P) {
    __shared__ uint32_t nh_keys[S_NH], nh_vals[S_NH];
    __shared__ uint32_t hm[S_LH], nl_x[S_LH], nl_meta[S_LH];
    __shared__ __attribute__((aligned(16))) uint32_t warea[S_WAREA];
    __shared__ WaveMem wmem[NWAVE];
    __shared__ Shared sh;
    __shared__ Tables T;
    __shared__ uint64_t acc_he[HGT_N_HE_CLASSES], acc_tmp[HGT_N_TEMPORAL_CLASSES], acc_st[4];
    for (int i = threadIdx.x; i < 128; i += HGT_WG) { T.he[i] = P.he_tab[i]; T.tmp[i] = P.tmp_tab[i]; }
    if (threadIdx.x == 0) sh.cur_g = 0xffffffffu;
    if (threadIdx.x < 4) acc_st[threadIdx.x] = 0;
    for (int i = threadIdx.x; i < HGT_N_HE_CLASSES; i += HGT_WG) acc_he[i] = 0;
    for (int i = threadIdx.x; i < HGT_N_TEMPORAL_CLASSES; i += HGT_WG) acc_tmp[i] = 0;
    __syncthreads();
    WgStore S{nh_keys, nh_vals, hm, nl_x, nl_meta, warea, S_WAREA, warea};
    run_centres<false>(P, T, S, sh, wmem, acc_he, acc_tmp, acc_st, S_LH, S_LH);
    flush_counts(P, sh.cur_g, acc_he, acc_tmp);
    if (P.stats && threadIdx.x == 0) {
        atomicAdd((unsigned long long*)&P.stats[ST_BYTES_SMALL], (unsigned long long)acc_st[0]);
        atomicAdd((unsigned long long*)&P.stats[ST_DEFERRED], (unsigned long long)acc_st[1]);
        atomicAdd((unsigned long long*)&P.stats[ST_WITNESS], (unsigned long long)acc_st[2]);
        atomicAdd((unsigned long long*)&P.stats[ST_EXPANDED], (unsigned long long)acc_st[3]);
    }
}

__global__ void __launch_bounds__(HGT_WG) k_delta_big(TriadParams P) {
    __shared__ uint32_t wh[NWAVE * 2 * WH_SLOTS];
    __shared__ WaveMem wmem[NWAVE];
    __shared__ Shared sh;
    __shared__ Tables T;
    __shared__ uint64_t acc_he[HGT_N_HE_CLASSES], acc_tmp[HGT_N_TEMPORAL_CLASSES], acc_st[4];
    for (int i = threadIdx.x; i < 128; i += HGT_WG) { T.he[i] = P.he_tab[i]; T.tmp[i] = P.tmp_tab[i]; }
    if (threadIdx.x == 0) sh.cur_g = 0xffffffffu;
    if (threadIdx.x < 4) acc_st[threadIdx.x] = 0;
    for (int i = threadIdx.x; i < HGT_N_HE_CLASSES; i += HGT_WG) acc_he[i] = 0;
    for (int i = threadIdx.x; i < HGT_N_TEMPORAL_CLASSES; i += HGT_WG) acc_tmp[i] = 0;
    __syncthreads();
    const BigLayout& L = P.big;
    uint32_t* base = P.big_scratch + (uint64_t)blockIdx.x * L.words_per_wg;
    WgStore S{base + L.nh_keys, base + L.nh_vals, base + L.hm, base + L.nl_x, base + L.nl_meta, base + L.warea,
              L.warea_words, wh};
    run_centres<true>(P, T, S, sh, wmem, acc_he, acc_tmp, acc_st, 0xffffffffu, 0xffffffffu);
    flush_counts(P, sh.cur_g, acc_he, acc_tmp);
    if (P.stats && threadIdx.x == 0) {
        atomicAdd((unsigned long long*)&P.stats[ST_BYTES_BIG], (unsigned long long)acc_st[0]);
        atomicAdd((unsigned long long*)&P.stats[ST_DEFERRED], (unsigned long long)acc_st[1]);
        atomicAdd((unsigned long long*)&P.stats[ST_WITNESS], (unsigned long long)acc_st[2]);
        atomicAdd((unsigned long long*)&P.stats[ST_EXPANDED], (unsigned long long)acc_st[3]);
    }
}

}  // namespace

BigLayout triad_big_layout(uint64_t max_lh, uint64_t max_card) {
    BigLayout L{};
    uint64_t nh = pow2ceil64(2 * (max_lh < 32 ? 32 : max_lh));
    uint64_t off = 0;
    auto take = [&](uint64_t words) { uint64_t o = off; off += (words + 3) & ~3ull; return o; };
    L.nh_keys = take(nh);
    L.nh_vals = take(nh);
    L.hm = take(max_card);
    L.nl_x = take(max_lh);
    L.nl_meta = take(max_lh);
    // shared area: prefix + offsets of h's members (3 words each + slack), histogram
    // (2 * (card + 1)), temporal list (4 words per neighbour)
    uint64_t wa = 3 * (max_card + 2) + 4;
    if (2 * (max_card + 1) > wa) wa = 2 * (max_card + 1);
    if (4 * max_lh > wa) wa = 4 * max_lh;
    L.warea_words = wa;
    L.warea = take(wa);
    L.words_per_wg = off;
    return L;
}

void triad_he_prepare(TriadParams& P, hipStream_t s) {
    hgt_fill_u32(P.queue, 0, 3, s);  // queue, big_queue, big_count
}

void triad_he_launch_small(TriadParams& P, unsigned grid, hipStream_t s) {
    if (P.M.total) k_delta_small<<<grid, HGT_WG, 0, s>>>(P);
}

namespace {

constexpr uint32_t kSliceLh = 4096;  // member-list entries per slice of a deferred centre (default)
constexpr uint32_t kMaxSlices = 32;

// one wave per deferred centre: its slice count from its members' list lengths
__global__ void k_slice_count(Multi M, const uint64_t* __restrict__ list, const uint32_t* n_p, uint64_t cap,
                              uint32_t per, uint64_t* pre) {
    const int lane = threadIdx.x & 63;
    const uint64_t c = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint32_t n = *n_p;
    if (c == 0 && lane == 0) pre[cap] = n;
    if (c >= n) return;
    const uint64_t it = list[c];
    const GraphView& g = M.graphs[(uint32_t)(it >> 32)].g;
    const uint32_t h = (uint32_t)it;
    const uint32_t* row = g.h2v + g.h_off[h];
    const uint32_t len = g.h_len[h];
    uint64_t lh = 0;
    for (uint32_t i = lane; i < len; i += 64) lh += g.v_len[row[i]];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) lh += __shfl_xor(lh, o, 64);
    if (lane == 0) {
        const uint64_t sl = (lh + per - 1) / per;
        pre[c] = sl < 1 ? 1 : (sl > kMaxSlices ? kMaxSlices : sl);
    }
}

}  // namespace

void triad_he_slices(TriadParams& P, hipStream_t s) {
    if (!P.slice_pre || !P.M.total) return;
    const uint64_t cap = P.slice_cap;
    k_slice_count<<<(unsigned)((cap * 64 + 255) / 256), 256, 0, s>>>(P.M, P.big_list, P.big_count, cap,
                                                                     P.slice_lh ? P.slice_lh : kSliceLh, P.slice_pre);
    // exclusive prefix over the deferred centres; the total after the count
    hgt_scan_u64(P.slice_pre, P.slice_pre, cap, P.slice_pre + cap, P.slice_pre + cap + 1, P.slice_scan_tmp, s);
}

void triad_he_launch_big(TriadParams& P, unsigned grid, hipStream_t s) {
    if (P.M.total) k_delta_big<<<grid, HGT_WG, 0, s>>>(P);
}
