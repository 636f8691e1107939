// store.hip -- the dual incidence store: batch validation, canonicalisation,
// ID assignment, block allocation and the h2v / v2h updates.
//
// Layout in HBM (one graph):
//   h2v pool  : u32 words; hyperedge `id` owns a block [h_off[id], h_off[id]+h_cap[id])
//               whose first h_len[id] words are its sorted member vertices.
//   v2h pool  : u32 words; vertex v owns a block [v_off[v], v_off[v]+v_cap[v]) whose
//               first v_len[v] words are the IDs of its live hyperedges, ascending.
//   v2h_ts    : (graphs that track temporal triads) one int64 per v2h word: the
//               timestamp of the entry at the same index, rewritten with it.
//   free_bm   : one bit per ID below next_id, set when the ID is free.
// Block capacities are powers of two (>= 4 words).  A deleted hyperedge keeps
// its block and the block is reused in place by the next hyperedge that takes
// the same ID, when it fits (the paper's Case 1, Sec. III-B); a hyperedge or a
// vertex list that outgrows its block gets a fresh block from the pool's bump
// region (Cases 2 and 3: block sizes -> prefix sum -> start addresses).
// Every kernel that runs before the host has read the batch summary leaves
// the graph unchanged, so a rejected batch has no effect.
#include <algorithm>

#include "store.h"

namespace {

__device__ __forceinline__ bool status_bad(const int32_t* st) { return *((volatile const int32_t*)st) != 0; }

// ---------------------------------------------------------------------------
// validation and canonicalisation (non-mutating)
// ---------------------------------------------------------------------------
__global__ void k_batch_begin(DevScalars* sc, BatchSummary* sum) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        sc->status = 0;
        BatchSummary z = {};
        *sum = z;
    }
}

// One thread per deleted ID: liveness, duplicates, deletion marks and sizes.
__global__ void k_del_check(const uint32_t* __restrict__ del, uint64_t n_del, DevScalars* sc,
                            const uint64_t* __restrict__ free_bm, uint64_t* del_bm, uint64_t* mark_del,
                            uint32_t epoch, const uint32_t* __restrict__ h_len, const uint64_t* __restrict__ h_off,
                            const uint32_t* __restrict__ h2v, const uint32_t* __restrict__ v_len,
                            uint64_t* del_card, BatchSummary* sum) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_del) return;
    uint32_t id = del[i];
    if ((uint64_t)id >= sc->next_id || ((free_bm[id >> 6] >> (id & 63)) & 1ull)) {
        set_status(&sc->status, HGT_ENOENT);
        del_card[i] = 0;
        return;
    }
    uint64_t bit = 1ull << (id & 63);
    uint64_t old = atomicOr((unsigned long long*)&del_bm[id >> 6], (unsigned long long)bit);
    if (old & bit) {
        set_status(&sc->status, HGT_EDUP);
        del_card[i] = 0;
        return;
    }
    mark_del[id] = ((uint64_t)epoch << 32) | (uint32_t)i;
    uint64_t d = h_len[id];
    del_card[i] = d;
    atomicAdd((unsigned long long*)&sum->del_members, (unsigned long long)d);
    atomicAdd((unsigned long long*)&sum->del_pairs2, (unsigned long long)choose2(d));
    uint64_t lh = 0;
    const uint32_t* m = h2v + h_off[id];
    for (uint64_t k = 0; k < d; k++) lh += v_len[m[k]];
    atomicMax((unsigned long long*)&sum->max_lh_del, (unsigned long long)lh);
    atomicAdd((unsigned long long*)&sum->sum_lh_del, (unsigned long long)lh);
}

// One thread per insert: CSR sanity, cardinality bounds, temporal order.
__global__ void k_ins_check(const uint64_t* __restrict__ off, uint64_t n_ins, uint64_t n_members,
                            const int64_t* __restrict__ ts, int check_order, DevScalars* sc,
                            uint64_t* ins_rel, uint64_t* ins_card, BatchSummary* sum) {
    uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_ins) return;
    uint64_t a = off[j], b = off[j + 1], o0 = off[0];
    uint64_t card = 0;
    if (a < o0 || b < a || b - o0 > n_members) {
        set_status(&sc->status, HGT_EINVAL);
    } else {
        card = b - a;
        if (card < 1 || card > HGT_MAX_CARD) set_status(&sc->status, HGT_EINVAL);
    }
    if (j == n_ins - 1 && off[n_ins] - o0 != n_members) set_status(&sc->status, HGT_EINVAL);
    ins_rel[j] = (a >= o0) ? a - o0 : 0;
    if (j == n_ins - 1) ins_rel[n_ins] = n_members;
    ins_card[j] = card;
    atomicAdd((unsigned long long*)&sum->ins_pairs2, (unsigned long long)choose2(card));
    atomicMax((unsigned long long*)&sum->max_ins_card, (unsigned long long)card);
    if (ts && check_order) {
        if (j > 0 && ts[j] < ts[j - 1]) set_status(&sc->status, HGT_EORDER);
        if (j == 0 && ts[0] < sc->last_ts) set_status(&sc->status, HGT_EORDER);
    }
}

// One wave per insert of cardinality <= 64: bitonic sort across lanes, then
// range and repeat checks.  Larger rows are queued for k_canon_big.
__global__ void __launch_bounds__(HGT_WG) k_canon_small(const uint32_t* __restrict__ mem,
                                                        const uint64_t* __restrict__ ins_rel, uint64_t n_ins,
                                                        uint32_t n_vertices, DevScalars* sc,
                                                        uint32_t* __restrict__ canon, uint32_t* big_list,
                                                        uint32_t* big_count) {
    if (status_bad(&sc->status)) return;
    const int lane = threadIdx.x & 63;
    uint64_t j = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (j >= n_ins) return;
    uint64_t a = ins_rel[j], card = ins_rel[j + 1] - a;
    if (card > 64) {
        if (lane == 0) big_list[atomicAdd(big_count, 1u)] = (uint32_t)j;
        return;
    }
    uint32_t v = (uint64_t)lane < card ? mem[a + lane] : 0xffffffffu;
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int s = k >> 1; s > 0; s >>= 1) {
            uint32_t o = __shfl_xor(v, s, 64);
            bool up = (lane & k) == 0;
            bool lower = (lane & s) == 0;
            uint32_t mn = v < o ? v : o, mx = v < o ? o : v;
            v = (up == lower) ? mn : mx;
        }
    }
    uint32_t nxt = __shfl_down(v, 1, 64);
    if ((uint64_t)lane < card) {
        if (v >= n_vertices) set_status(&sc->status, HGT_EINVAL);
        if ((uint64_t)lane + 1 < card && nxt == v) set_status(&sc->status, HGT_EINVAL);
        canon[a + lane] = v;
    }
}

// One workgroup per queued row (64 < card <= HGT_MAX_CARD): bitonic sort in LDS.
__global__ void __launch_bounds__(HGT_WG) k_canon_big(const uint32_t* __restrict__ mem,
                                                      const uint64_t* __restrict__ ins_rel, uint32_t n_vertices,
                                                      DevScalars* sc, uint32_t* __restrict__ canon,
                                                      const uint32_t* big_list, const uint32_t* big_count) {
    __shared__ uint32_t buf[HGT_MAX_CARD];
    __shared__ uint32_t bad;
    // other workgroups of this launch may set the status meanwhile: one read,
    // shared, so the whole workgroup leaves (or stays) before any barrier
    if (threadIdx.x == 0) bad = status_bad(&sc->status) ? 1u : 0u;
    __syncthreads();
    if (bad) return;
    uint32_t nb = *big_count;
    for (uint32_t q = blockIdx.x; q < nb; q += gridDim.x) {
        uint64_t j = big_list[q];
        uint64_t a = ins_rel[j];
        uint32_t card = (uint32_t)(ins_rel[j + 1] - a);
        uint32_t n = (uint32_t)pow2ceil64(card);
        for (uint32_t i = threadIdx.x; i < n; i += HGT_WG) buf[i] = i < card ? mem[a + i] : 0xffffffffu;
        __syncthreads();
        for (uint32_t k = 2; k <= n; k <<= 1) {
            for (uint32_t s = k >> 1; s > 0; s >>= 1) {
                for (uint32_t i = threadIdx.x; i < n; i += HGT_WG) {
                    uint32_t p = i ^ s;
                    if (p > i) {
                        bool up = (i & k) == 0;
                        uint32_t x = buf[i], y = buf[p];
                        if ((x > y) == up) { buf[i] = y; buf[p] = x; }
                    }
                }
                __syncthreads();
            }
        }
        for (uint32_t i = threadIdx.x; i < card; i += HGT_WG) {
            uint32_t v = buf[i];
            if (v >= n_vertices) set_status(&sc->status, HGT_EINVAL);
            if (i + 1 < card && buf[i + 1] == v) set_status(&sc->status, HGT_EINVAL);
            canon[a + i] = v;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// ID assignment: the j-th insert takes the j-th smallest free ID
// ---------------------------------------------------------------------------
__global__ void k_free_popc(const uint64_t* __restrict__ free_bm, const uint64_t* __restrict__ del_bm,
                            const DevScalars* sc, uint64_t* popc, uint64_t* n_words_out) {
    uint64_t nw = (sc->next_id + 63) >> 6;
    uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w == 0) *n_words_out = nw;
    if (w >= nw) return;
    popc[w] = __popcll(free_bm[w] | del_bm[w]);
}

__global__ void k_assign_free(const uint64_t* __restrict__ free_bm, const uint64_t* __restrict__ del_bm,
                              const uint64_t* __restrict__ pre, const uint64_t* n_words, uint64_t n_ins,
                              uint32_t* assigned) {
    uint64_t w = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= *n_words) return;
    uint64_t r = pre[w];
    if (r >= n_ins) return;
    uint64_t bits = free_bm[w] | del_bm[w];
    while (bits && r < n_ins) {
        int b = __ffsll((unsigned long long)bits) - 1;
        assigned[r++] = (uint32_t)(w * 64 + b);
        bits &= bits - 1;
    }
}

__global__ void k_assign_fresh(uint64_t n_ins, const DevScalars* sc, BatchSummary* sum, uint32_t* assigned,
                               uint64_t* mark_ins, uint32_t epoch) {
    uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t nf = sum->n_free;
    if (j == 0) sum->next_id_new = sc->next_id + (n_ins > nf ? n_ins - nf : 0);
    if (j >= n_ins) return;
    if (j >= nf) assigned[j] = (uint32_t)(sc->next_id + (j - nf));
    mark_ins[assigned[j]] = ((uint64_t)epoch << 32) | (uint32_t)j;
}

// horizontal operations: insert j takes forced[j], the ID deleted at rank j
__global__ void k_assign_forced(uint64_t n_ins, const uint32_t* __restrict__ forced, const DevScalars* sc,
                                BatchSummary* sum, uint32_t* assigned, uint64_t* mark_ins, uint32_t epoch) {
    uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j == 0) {
        sum->next_id_new = sc->next_id;
        sum->n_free = n_ins;
    }
    if (j >= n_ins) return;
    assigned[j] = forced[j];
    mark_ins[forced[j]] = ((uint64_t)epoch << 32) | (uint32_t)j;
}

// words of a fresh h2v block for insert j (0 when the ID's retained block fits)
__global__ void k_h2v_need(const uint32_t* __restrict__ assigned, const uint64_t* __restrict__ ins_card,
                           uint64_t n_ins, const DevScalars* sc, const uint32_t* __restrict__ h_cap,
                           uint64_t* need) {
    uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_ins) return;
    uint32_t id = assigned[j];
    uint64_t cap = (uint64_t)id < sc->next_id ? h_cap[id] : 0;
    uint64_t card = ins_card[j];
    need[j] = card > cap ? pow2ceil64(card < 4 ? 4 : card) : 0;
}

// ---------------------------------------------------------------------------
// (vertex, hyperedge, is_insert) pairs, sorted, and the per-vertex plan
// ---------------------------------------------------------------------------
__global__ void k_pairs_del(const uint32_t* __restrict__ del, uint64_t n_del, const uint64_t* __restrict__ del_poff,
                            const uint64_t* __restrict__ h_off, const uint32_t* __restrict__ h_len,
                            const uint32_t* __restrict__ h2v, int hb, uint64_t* keys, const DevScalars* sc) {
    if (status_bad(&sc->status)) return;
    const int lane = threadIdx.x & 63;
    uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (i >= n_del) return;
    uint32_t id = del[i];
    uint64_t d = h_len[id], o = h_off[id], p = del_poff[i];
    for (uint64_t k = lane; k < d; k += 64) keys[p + k] = ((uint64_t)h2v[o + k] << (hb + 1)) | ((uint64_t)id << 1);
}

__global__ void k_pairs_ins(const uint32_t* __restrict__ canon, const uint64_t* __restrict__ ins_rel, uint64_t n_ins,
                            uint64_t n_members, const uint32_t* __restrict__ assigned, int hb, const BatchSummary* sum,
                            uint64_t* keys, const DevScalars* sc) {
    if (status_bad(&sc->status)) return;
    uint64_t m = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n_members) return;
    uint32_t j = seg_of<uint64_t>(ins_rel, (uint32_t)n_ins, m);
    keys[sum->del_members + m] = ((uint64_t)canon[m] << (hb + 1)) | ((uint64_t)assigned[j] << 1) | 1ull;
}

__global__ void k_pair_count(const BatchSummary* sum, uint64_t n_ins_members, uint64_t* n_pairs) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *n_pairs = sum->del_members + n_ins_members;
}

__global__ void k_heads(const uint64_t* __restrict__ keys, const uint64_t* n_pairs_p, int hb, uint64_t* head,
                        uint64_t* is_ins) {
    uint64_t n = *n_pairs_p;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t k = keys[i];
    head[i] = (i == 0 || (keys[i - 1] >> (hb + 1)) != (k >> (hb + 1))) ? 1 : 0;
    is_ins[i] = k & 1ull;
}

// head[] was scanned in place into tidx[] (exclusive), is_ins into ins_pre[].
// After a failed validation the pair keys were not (all) written: the plan
// kernels that index arrays with decoded keys then stop.
__global__ void k_split(const uint64_t* __restrict__ keys, const uint64_t* n_pairs_p, int hb,
                        const uint64_t* __restrict__ tidx, const uint64_t* __restrict__ ins_pre, uint32_t* tv,
                        uint64_t* tseg, uint32_t* D_all, uint32_t* I_all, uint32_t* I_t, const uint64_t* n_touched_p,
                        const DevScalars* sc) {
    if (status_bad(&sc->status)) return;
    uint64_t n = *n_pairs_p;
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) tseg[*n_touched_p] = n;
    if (i >= n) return;
    uint64_t k = keys[i];
    uint32_t v = (uint32_t)(k >> (hb + 1));
    uint32_t h = (uint32_t)((k >> 1) & ((1ull << hb) - 1));
    bool hd = (i == 0) || ((keys[i - 1] >> (hb + 1)) != (k >> (hb + 1)));
    uint64_t t = tidx[i] + (hd ? 1 : 0) - 1;
    if (hd) {
        tv[t] = v;
        tseg[t] = i;
    }
    uint64_t ip = ins_pre[i];
    if (k & 1ull) {
        I_all[ip] = h;
        I_t[ip] = (uint32_t)t;
    } else {
        D_all[i - ip] = h;
    }
}

__global__ void k_vplan(const uint64_t* n_touched_p, const uint32_t* __restrict__ tv, const uint64_t* __restrict__ tseg,
                        const uint64_t* __restrict__ ins_pre, const uint64_t* n_pairs_p, const uint64_t* ins_total,
                        const uint32_t* __restrict__ v_len, const uint32_t* __restrict__ v_cap, VPlan p,
                        DevScalars* sc) {
    if (status_bad(&sc->status)) return;
    uint64_t nt = *n_touched_p;
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt) return;
    uint64_t s = tseg[t], e = tseg[t + 1], n = *n_pairs_p;
    uint64_t ips = ins_pre[s];
    uint64_t ipe = e < n ? ins_pre[e] : *ins_total;
    uint64_t nI = ipe - ips, nD = (e - s) - nI;
    uint32_t v = tv[t];
    uint64_t old = v_len[v];
    if (nD > old) { set_status(&sc->status, HGT_EDEVICE); nD = old; }
    uint64_t nw = old - nD + nI;
    p.dstart[t] = s - ips;
    p.istart[t] = ips;
    p.nD[t] = (uint32_t)nD;
    p.nI[t] = (uint32_t)nI;
    p.old_len[t] = old;
    p.new_len[t] = (uint32_t)nw;
    p.need[t] = nw > v_cap[v] ? pow2ceil64(nw < 4 ? 4 : nw) : 0;
}

// per insert: sum over its members of their new incidence-list length
__global__ void k_lh_ins(const uint32_t* __restrict__ canon, const uint64_t* __restrict__ ins_rel, uint64_t n_ins,
                         const uint32_t* __restrict__ tv, const uint64_t* n_touched_p,
                         const uint32_t* __restrict__ new_len, BatchSummary* sum, const DevScalars* sc) {
    if (status_bad(&sc->status)) return;
    uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_ins) return;
    uint32_t nt = (uint32_t)*n_touched_p;
    uint64_t lh = 0;
    for (uint64_t m = ins_rel[j]; m < ins_rel[j + 1]; m++) {
        uint32_t t = lower_bound_u32(tv, nt, canon[m]);
        if (t < nt) lh += new_len[t];
    }
    atomicMax((unsigned long long*)&sum->max_lh_ins, (unsigned long long)lh);
    atomicAdd((unsigned long long*)&sum->sum_lh_ins, (unsigned long long)lh);
}

__global__ void k_summary_finish(const DevScalars* sc, BatchSummary* sum, const uint64_t* n_free,
                                 const uint64_t* h2v_need, const uint64_t* v2h_need, const uint64_t* n_touched,
                                 const uint64_t* stage_words) {
    if (threadIdx.x || blockIdx.x) return;
    sum->status = sc->status;
    sum->h2v_need = *h2v_need;
    sum->v2h_need = *v2h_need;
    sum->n_touched = *n_touched;
    sum->stage_words = *stage_words;
    (void)n_free;
}

__global__ void k_set_nfree(BatchSummary* sum, const uint64_t* n_free) {
    if (threadIdx.x == 0 && blockIdx.x == 0) sum->n_free = *n_free;
}

// ---------------------------------------------------------------------------
// mutation (after the host accepted the summary)
// ---------------------------------------------------------------------------
__global__ void k_apply_delete(const uint32_t* __restrict__ del, uint64_t n_del, uint64_t* free_bm, uint32_t* h_len) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_del) return;
    uint32_t id = del[i];
    atomicOr((unsigned long long*)&free_bm[id >> 6], (unsigned long long)(1ull << (id & 63)));
    h_len[id] = 0;
}

__global__ void k_h2v_meta(const uint32_t* __restrict__ assigned, const uint64_t* __restrict__ ins_card, uint64_t n_ins,
                           const uint64_t* __restrict__ need, const uint64_t* __restrict__ rel, uint64_t next_id_old,
                           uint64_t h_bump, const int64_t* __restrict__ ts, uint64_t next_seq, int keep_seq,
                           uint64_t* h_off, uint32_t* h_len, uint32_t* h_cap, int64_t* h_ts, uint64_t* h_seq,
                           uint64_t* free_bm) {
    uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_ins) return;
    uint32_t id = assigned[j];
    if (need[j]) {
        h_off[id] = h_bump + rel[j];
        h_cap[id] = (uint32_t)need[j];
    }
    h_len[id] = (uint32_t)ins_card[j];
    if (h_ts) h_ts[id] = ts ? ts[j] : 0;
    if (!keep_seq) h_seq[id] = next_seq + j;
    if ((uint64_t)id < next_id_old)
        atomicAnd((unsigned long long*)&free_bm[id >> 6], (unsigned long long)~(1ull << (id & 63)));
}

__global__ void k_h2v_copy(const uint32_t* __restrict__ canon, const uint64_t* __restrict__ ins_rel, uint64_t n_ins,
                           uint64_t n_members, const uint32_t* __restrict__ assigned,
                           const uint64_t* __restrict__ h_off, uint32_t* h2v) {
    uint64_t m = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n_members) return;
    uint32_t j = seg_of<uint64_t>(ins_rel, (uint32_t)n_ins, m);
    h2v[h_off[assigned[j]] + (m - ins_rel[j])] = canon[m];
}

__global__ void k_v_stage(const uint64_t* __restrict__ stage_off, const uint32_t* __restrict__ tv, uint64_t n_touched,
                          uint64_t stage_words, const uint64_t* __restrict__ v_off, const uint32_t* __restrict__ v2h,
                          const int64_t* __restrict__ v2h_ts, uint32_t* staging, int64_t* staging_ts) {
    uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= stage_words) return;
    uint32_t t = seg_of<uint64_t>(stage_off, (uint32_t)n_touched, s);
    const uint64_t src = v_off[tv[t]] + (s - stage_off[t]);
    staging[s] = v2h[src];
    if (v2h_ts) staging_ts[s] = v2h_ts[src];
}

__global__ void k_v_dst(uint64_t n_touched, const uint32_t* __restrict__ tv, const uint64_t* __restrict__ need,
                        const uint64_t* __restrict__ rel, uint64_t v_bump, const uint64_t* __restrict__ v_off,
                        uint64_t* dst) {
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_touched) return;
    dst[t] = need[t] ? v_bump + rel[t] : v_off[tv[t]];
}

__global__ void k_v_merge_old(const uint64_t* __restrict__ stage_off, uint64_t n_touched, uint64_t stage_words,
                              const uint32_t* __restrict__ staging, const int64_t* __restrict__ staging_ts, VPlan p,
                              const uint32_t* __restrict__ D_all, const uint32_t* __restrict__ I_all,
                              const uint64_t* __restrict__ dst, uint32_t* v2h, int64_t* v2h_ts) {
    uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= stage_words) return;
    uint32_t t = seg_of<uint64_t>(stage_off, (uint32_t)n_touched, s);
    uint32_t e = staging[s];
    const uint32_t* D = D_all + p.dstart[t];
    uint32_t nD = p.nD[t];
    uint32_t dl = lower_bound_u32(D, nD, e);
    if (dl < nD && D[dl] == e) return;  // deleted
    uint32_t il = lower_bound_u32(I_all + p.istart[t], p.nI[t], e);
    uint64_t pos = (s - stage_off[t]) - dl + il;
    v2h[dst[t] + pos] = e;
    if (v2h_ts) v2h_ts[dst[t] + pos] = staging_ts[s];
}

// h_ts already holds the inserted hyperedges' timestamps (k_h2v_meta runs first)
__global__ void k_v_merge_ins(const uint64_t* n_ins_pairs_p, const uint32_t* __restrict__ I_all,
                              const uint32_t* __restrict__ I_t, const uint64_t* __restrict__ stage_off,
                              const uint32_t* __restrict__ staging, VPlan p, const uint32_t* __restrict__ D_all,
                              const uint64_t* __restrict__ dst, const int64_t* __restrict__ h_ts, uint32_t* v2h,
                              int64_t* v2h_ts) {
    uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= *n_ins_pairs_p) return;
    uint32_t t = I_t[k];
    uint32_t e = I_all[k];
    uint64_t kk = k - p.istart[t];
    uint32_t ol = lower_bound_u32(staging + stage_off[t], (uint32_t)p.old_len[t], e);
    uint32_t dl = lower_bound_u32(D_all + p.dstart[t], p.nD[t], e);
    v2h[dst[t] + kk + ol - dl] = e;
    if (v2h_ts) v2h_ts[dst[t] + kk + ol - dl] = h_ts[e];
}

__global__ void k_v_commit(uint64_t n_touched, const uint32_t* __restrict__ tv, VPlan p,
                           const uint64_t* __restrict__ dst, uint64_t* v_off, uint32_t* v_len, uint32_t* v_cap) {
    uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_touched) return;
    uint32_t v = tv[t];
    v_off[v] = dst[t];
    if (p.need[t]) v_cap[v] = (uint32_t)p.need[t];
    v_len[v] = p.new_len[t];
}

__global__ void k_commit_scalars(DevScalars* sc, const BatchSummary* sum, uint64_t n_del, uint64_t n_ins,
                                 uint64_t n_ins_members, const int64_t* ins_ts, int keep_seq) {
    if (threadIdx.x || blockIdx.x) return;
    sc->next_id = sum->next_id_new;
    sc->h_bump += sum->h2v_need;
    sc->v_bump += sum->v2h_need;
    if (!keep_seq) sc->next_seq += n_ins;
    if (ins_ts && n_ins) {
        int64_t t = ins_ts[n_ins - 1];  // batch timestamps are non-decreasing
        if (t > sc->last_ts) sc->last_ts = t;
    }
    sc->n_live = sc->n_live + n_ins - n_del;
    sc->n_inc = sc->n_inc + n_ins_members - sum->del_members;
}

// last_ts over an arbitrary (unsorted) initial timestamp array
__global__ void k_max_ts(const int64_t* ts, uint64_t n, DevScalars* sc) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        atomicMax((long long*)&sc->last_ts, (long long)ts[i]);
}

__global__ void k_counts_update(uint64_t* counts, const uint64_t* plus, const uint64_t* minus, int n, const DevScalars* sc) {
    if (status_bad(&sc->status)) return;
    int i = threadIdx.x;
    if (i < n) counts[i] += plus[i] - minus[i];
}

// ---------------------------------------------------------------------------
// compaction: every live list moved into a fresh pool, blocks of dead IDs and
// blocks left behind by relocations dropped
// ---------------------------------------------------------------------------
__global__ void k_cmp_hneed(uint64_t n_ids, const uint64_t* __restrict__ free_bm, const uint32_t* __restrict__ h_len,
                            uint64_t* need) {
    for (uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; id < n_ids;
         id += (uint64_t)gridDim.x * blockDim.x) {
        const bool live = !((free_bm[id >> 6] >> (id & 63)) & 1ull);
        const uint64_t len = h_len[id];
        need[id] = live ? pow2ceil64(len < 4 ? 4 : len) : 0;
    }
}

__global__ void k_cmp_vneed(uint64_t n_vertices, const uint32_t* __restrict__ v_len, uint64_t* need) {
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n_vertices;
         v += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t len = v_len[v];
        need[v] = len ? pow2ceil64(len < 4 ? 4 : len) : 0;
    }
}

// one wave per list: `len` words (and `side` words per word of a side array
// that follows the pool: histograms, timestamps) to the list's new offset
template <class S>
__global__ void k_cmp_copy(uint64_t n, const uint64_t* __restrict__ need, const uint64_t* __restrict__ new_off,
                           const uint64_t* __restrict__ old_off, const uint32_t* __restrict__ len,
                           const uint32_t* __restrict__ pool, uint32_t* pool_new, const S* __restrict__ side,
                           S* side_new, int side_per_word) {
    const int lane = threadIdx.x & 63;
    for (uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; i < n;
         i += ((uint64_t)gridDim.x * blockDim.x) >> 6) {
        if (!need[i]) continue;
        const uint64_t o = old_off[i], d = new_off[i], l = len[i];
        for (uint64_t k = lane; k < l; k += 64) pool_new[d + k] = pool[o + k];
        if (side)
            for (uint64_t k = lane; k < l * side_per_word; k += 64)
                side_new[d * side_per_word + k] = side[o * side_per_word + k];
    }
}

__global__ void k_cmp_commit(uint64_t n, const uint64_t* __restrict__ need, const uint64_t* __restrict__ new_off,
                             uint64_t* off, uint32_t* cap) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        off[i] = need[i] ? new_off[i] : 0;
        cap[i] = (uint32_t)need[i];
    }
}

__global__ void k_cmp_scalars(DevScalars* sc, const uint64_t* h_total, const uint64_t* v_total) {
    if (threadIdx.x || blockIdx.x) return;
    sc->h_bump = *h_total;
    sc->v_bump = *v_total;
}

inline unsigned blocks_for(uint64_t n, unsigned per = 256) {
    uint64_t b = (n + per - 1) / per;
    return (unsigned)(b ? b : 1);
}

}  // namespace

void store_compact_need(const StoreDev& g, uint64_t n_ids, uint64_t* h_need, uint64_t* v_need, hipStream_t s) {
    if (n_ids) k_cmp_hneed<<<blocks_for(n_ids > 262144 ? 262144 : n_ids), 256, 0, s>>>(n_ids, g.free_bm, g.h_len, h_need);
    const uint64_t V = g.n_vertices;
    k_cmp_vneed<<<blocks_for(V > 262144 ? 262144 : V), 256, 0, s>>>(V, g.v_len, v_need);
}

void store_compact_h2v(const StoreDev& g, uint64_t n_ids, const uint64_t* need, const uint64_t* new_off,
                       uint32_t* h2v_new, const uint32_t* hpool, uint32_t* hpool_new, hipStream_t s) {
    if (!n_ids) return;
    const unsigned grid = (unsigned)std::min<uint64_t>(65536, (n_ids * 64 + 255) / 256);
    k_cmp_copy<uint32_t><<<grid, 256, 0, s>>>(n_ids, need, new_off, g.h_off, g.h_len, g.h2v, h2v_new, hpool,
                                              hpool_new, 2);
    k_cmp_commit<<<blocks_for(n_ids > 262144 ? 262144 : n_ids), 256, 0, s>>>(n_ids, need, new_off, g.h_off, g.h_cap);
}

void store_compact_v2h(const StoreDev& g, const uint64_t* need, const uint64_t* new_off, uint32_t* v2h_new,
                       int64_t* v2h_ts_new, hipStream_t s) {
    const uint64_t V = g.n_vertices;
    const unsigned grid = (unsigned)std::min<uint64_t>(65536, (V * 64 + 255) / 256);
    k_cmp_copy<int64_t><<<grid, 256, 0, s>>>(V, need, new_off, g.v_off, g.v_len, g.v2h, v2h_new, g.v2h_ts,
                                             v2h_ts_new, 1);
    k_cmp_commit<<<blocks_for(V > 262144 ? 262144 : V), 256, 0, s>>>(V, need, new_off, g.v_off, g.v_cap);
}

void store_compact_scalars(DevScalars* sc, const uint64_t* h_total, const uint64_t* v_total, hipStream_t s) {
    k_cmp_scalars<<<1, 64, 0, s>>>(sc, h_total, v_total);
}

// ===========================================================================
// host launchers
// ===========================================================================
void store_batch_begin(DevScalars* sc, BatchSummary* sum, hipStream_t s) { k_batch_begin<<<1, 64, 0, s>>>(sc, sum); }

void store_plan(StoreDev& g, BatchIn& b, PlanScratch& w, hipStream_t s) {
    const uint64_t n_del = b.n_del, n_ins = b.n_ins, n_mem = b.n_ins_members;
    DevScalars* sc = g.sc;
    hgt_fill_u64(w.del_bm, 0, (g.id_cap + 63) / 64, s);
    if (n_del)
        k_del_check<<<blocks_for(n_del), 256, 0, s>>>(b.del, n_del, sc, g.free_bm, w.del_bm, g.mark_del, b.epoch_del,
                                                      g.h_len, g.h_off, g.h2v, g.v_len, w.del_card, w.sum);
    if (n_ins) {
        k_ins_check<<<blocks_for(n_ins), 256, 0, s>>>(b.ins_off, n_ins, n_mem, b.ins_ts, b.check_order, sc, w.ins_rel,
                                                      w.ins_card, w.sum);
        hgt_fill_u32(w.big_count, 0, 1, s);
        k_canon_small<<<blocks_for(n_ins * 64), 256, 0, s>>>(b.ins_mem, w.ins_rel, n_ins, g.n_vertices, sc, w.canon,
                                                             w.big_list, w.big_count);
        unsigned gb = (unsigned)(n_ins < 1024 ? n_ins : 1024);
        k_canon_big<<<gb, 256, 0, s>>>(b.ins_mem, w.ins_rel, g.n_vertices, sc, w.canon, w.big_list, w.big_count);
    }
    // ID assignment (the free-ID bitmap covers IDs below next_id; host bound words_max)
    if (b.forced_ids) {
        k_assign_forced<<<blocks_for(n_ins), 256, 0, s>>>(n_ins, b.forced_ids, sc, w.sum, w.assigned, g.mark_ins,
                                                          b.epoch_ins);
    } else {
        uint64_t words_max = (g.next_id_host + 63) / 64;
        k_free_popc<<<blocks_for(words_max), 256, 0, s>>>(g.free_bm, w.del_bm, sc, w.popc, w.n_words);
        hgt_scan_u64(w.popc, w.popc, words_max, w.n_words, w.n_free, w.scan_tmp, s);
        k_set_nfree<<<1, 64, 0, s>>>(w.sum, w.n_free);
        if (n_ins) {
            k_assign_free<<<blocks_for(words_max), 256, 0, s>>>(g.free_bm, w.del_bm, w.popc, w.n_words, n_ins,
                                                                w.assigned);
        }
        k_assign_fresh<<<blocks_for(n_ins), 256, 0, s>>>(n_ins, sc, w.sum, w.assigned, g.mark_ins, b.epoch_ins);
    }
    if (n_ins) {
        k_h2v_need<<<blocks_for(n_ins), 256, 0, s>>>(w.assigned, w.ins_card, n_ins, sc, g.h_cap, w.h_need);
        hgt_scan_u64(w.h_need, w.h_rel, n_ins, nullptr, w.h2v_total, w.scan_tmp, s);
    } else {
        hgt_fill_u64(w.h2v_total, 0, 1, s);
    }
    // incidence pairs
    if (n_del) {
        hgt_scan_u64(w.del_card, w.del_poff, n_del, nullptr, nullptr, w.scan_tmp, s);
        k_pairs_del<<<blocks_for(n_del * 64), 256, 0, s>>>(b.del, n_del, w.del_poff, g.h_off, g.h_len, g.h2v, g.hb,
                                                           w.keys, sc);
    }
    if (n_mem)
        k_pairs_ins<<<blocks_for(n_mem), 256, 0, s>>>(w.canon, w.ins_rel, n_ins, n_mem, w.assigned, g.hb, w.sum,
                                                      w.keys, sc);
    k_pair_count<<<1, 64, 0, s>>>(w.sum, n_mem, w.n_pairs);
    uint64_t pmax = w.pairs_cap;
    hgt_radix_sort_u64(w.keys, w.keys_alt, pmax, w.n_pairs, g.hb + 1 + g.vb, w.sort_tmp, s);
    k_heads<<<blocks_for(pmax), 256, 0, s>>>(w.keys, w.n_pairs, g.hb, w.head, w.is_ins);
    hgt_scan_u64(w.head, w.head, pmax, w.n_pairs, w.n_touched, w.scan_tmp, s);
    hgt_scan_u64(w.is_ins, w.is_ins, pmax, w.n_pairs, w.n_ins_pairs, w.scan_tmp, s);
    k_split<<<blocks_for(pmax), 256, 0, s>>>(w.keys, w.n_pairs, g.hb, w.head, w.is_ins, w.tv, w.tseg, w.D_all,
                                             w.I_all, w.I_t, w.n_touched, sc);
    k_vplan<<<blocks_for(pmax), 256, 0, s>>>(w.n_touched, w.tv, w.tseg, w.is_ins, w.n_pairs, w.n_ins_pairs, g.v_len,
                                             g.v_cap, w.vp, sc);
    hgt_scan_u64(w.vp.need, w.vp.rel, pmax, w.n_touched, w.v2h_total, w.scan_tmp, s);
    hgt_scan_u64(w.vp.old_len, w.vp.stage_off, pmax, w.n_touched, w.stage_total, w.scan_tmp, s);
    if (n_ins)
        k_lh_ins<<<blocks_for(n_ins), 256, 0, s>>>(w.canon, w.ins_rel, n_ins, w.tv, w.n_touched, w.vp.new_len, w.sum, sc);
    k_summary_finish<<<1, 64, 0, s>>>(sc, w.sum, w.n_free, w.h2v_total, w.v2h_total, w.n_touched, w.stage_total);
}

void store_commit(StoreDev& g, BatchIn& b, PlanScratch& w, const BatchSummary& sum, uint64_t h_bump,
                  uint64_t v_bump, uint64_t next_seq, hipStream_t s) {
    const uint64_t n_del = b.n_del, n_ins = b.n_ins, n_mem = b.n_ins_members;
    const uint64_t nt = sum.n_touched, sw = sum.stage_words;
    // h2v first: the v2h merge reads the inserted hyperedges' timestamps from h_ts
    // (the v2h steps read only the old lists, which the h2v steps never touch)
    if (n_del) k_apply_delete<<<blocks_for(n_del), 256, 0, s>>>(b.del, n_del, g.free_bm, g.h_len);
    if (n_ins) {
        k_h2v_meta<<<blocks_for(n_ins), 256, 0, s>>>(w.assigned, w.ins_card, n_ins, w.h_need, w.h_rel, g.next_id_host,
                                                     h_bump, b.ins_ts, next_seq, b.keep_seq, g.h_off, g.h_len, g.h_cap,
                                                     g.h_ts, g.h_seq, g.free_bm);
        if (n_mem)
            k_h2v_copy<<<blocks_for(n_mem), 256, 0, s>>>(w.canon, w.ins_rel, n_ins, n_mem, w.assigned, g.h_off, g.h2v);
    }
    if (nt) {
        if (sw)
            k_v_stage<<<blocks_for(sw), 256, 0, s>>>(w.vp.stage_off, w.tv, nt, sw, g.v_off, g.v2h, g.v2h_ts, w.staging,
                                                     w.staging_ts);
        k_v_dst<<<blocks_for(nt), 256, 0, s>>>(nt, w.tv, w.vp.need, w.vp.rel, v_bump, g.v_off, w.dst);
        if (sw)
            k_v_merge_old<<<blocks_for(sw), 256, 0, s>>>(w.vp.stage_off, nt, sw, w.staging, w.staging_ts, w.vp, w.D_all,
                                                         w.I_all, w.dst, g.v2h, g.v2h_ts);
        if (n_mem)
            k_v_merge_ins<<<blocks_for(n_mem), 256, 0, s>>>(w.n_ins_pairs, w.I_all, w.I_t, w.vp.stage_off, w.staging,
                                                            w.vp, w.D_all, w.dst, g.h_ts, g.v2h, g.v2h_ts);
        k_v_commit<<<blocks_for(nt), 256, 0, s>>>(nt, w.tv, w.vp, w.dst, g.v_off, g.v_len, g.v_cap);
    }
    k_commit_scalars<<<1, 64, 0, s>>>(g.sc, w.sum, n_del, n_ins, n_mem, b.check_order ? b.ins_ts : nullptr,
                                      b.keep_seq);
}

void store_max_ts(const int64_t* ts, uint64_t n, DevScalars* sc, hipStream_t s) {
    if (n) k_max_ts<<<blocks_for(n > 262144 ? 262144 : n), 256, 0, s>>>(ts, n, sc);
}

void store_counts_update(uint64_t* counts, const uint64_t* plus, const uint64_t* minus, int n, const DevScalars* sc,
                         hipStream_t s) {
    k_counts_update<<<1, 128, 0, s>>>(counts, plus, minus, n, sc);
}
