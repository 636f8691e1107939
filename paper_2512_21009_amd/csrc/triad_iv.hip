// triad_iv.hip -- incident-vertex triad deltas (types 1-3 with hyperedge multiplicity).
//
// With m_p the number of hyperedges containing the vertex pair p and
// w_p = sum over those hyperedges of (|h| - 2):
//   type 1            = sum_h C(|h|,3)
//   type 1+2+3        = sum over vertex triangles {a,b,c} of m_ab m_bc m_ac
//   type 2            = sum_p m_p w_p - 3 * type 1
// (a type-2 tuple is a vertex triple inside one hyperedge with one of its
// three pairs re-witnessed by a different hyperedge).  Only pairs inside a
// changed hyperedge ("touched" pairs) change m_p, so a batch changes
//   sum_p m_p w_p             by its value over the touched pairs, and
//   the triangle sum          by its value over triangles with a touched pair.
// Both are evaluated on the old graph (before the batch) and on the new graph
// (after it); the difference is the delta.
//
// Every touched pair has an owner, its endpoint of higher degree.  A workgroup
// takes an owner a and builds its weighted clique map M_a : w -> (m_aw, w_aw)
// in LDS from the hyperedges that contain a.  For each touched pair (a, b) it
// owns, m_ab and w_ab are read from the map, and the triangles through (a, b)
// contribute
//   m_ab * sum_{h' containing b} sum_{w in h', w != a, b} M_a[w].m
// (the inner double sum counts w with multiplicity m_bw; b, the endpoint of
// lower degree, is the one scanned).  A triangle with several touched pairs is
// counted at its lexicographically smallest one: with lo < hi the endpoints of
// the pair, the triangle {lo, hi, w} is skipped when {lo, w} is touched and
// w < hi, or {hi, w} is touched and w < lo (a global hash of the touched pairs
// answers).
#include "triad_common.h"

namespace {

using namespace tri;

constexpr uint32_t IV_ARENA = 8192;  // 32 KB of LDS per workgroup: four workgroups per CU

__device__ __forceinline__ uint64_t mix64(uint64_t k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k;
}

__device__ __forceinline__ bool touched(const uint64_t* tab, uint64_t mask, uint32_t x, uint32_t y) {
    uint64_t k = x < y ? ((uint64_t)x << 32 | y) : ((uint64_t)y << 32 | x);
    uint64_t s = mix64(k) & mask;
    for (uint64_t probe = 0; probe <= mask; probe++) {
        uint64_t t = tab[s];
        if (t == k) return true;
        if (t == ~0ull) return false;
        s = (s + 1) & mask;
    }
    return false;
}

__global__ void k_iv_hash_build(const uint64_t* __restrict__ pairs, const uint64_t* n_p, uint64_t* tab, uint64_t mask) {
    uint64_t n = *n_p;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t k = pairs[i];
        uint64_t s = mix64(k) & mask;
        for (uint64_t probe = 0; probe <= mask; probe++) {
            unsigned long long prev = atomicCAS((unsigned long long*)&tab[s], ~0ull, (unsigned long long)k);
            if (prev == ~0ull || prev == k) break;
            s = (s + 1) & mask;
        }
    }
}

// owners: first pair index of every distinct first vertex
__global__ void k_iv_owner_heads(const uint64_t* __restrict__ pairs, const uint64_t* n_p, uint64_t* head) {
    uint64_t n = *n_p;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        head[i] = (i == 0 || (pairs[i] >> 32) != (pairs[i - 1] >> 32)) ? 1 : 0;
}

__global__ void k_iv_owner_list(const uint64_t* __restrict__ pairs, const uint64_t* n_p, const uint64_t* __restrict__ pos,
                                uint64_t* owner_start, const uint64_t* n_owner) {
    uint64_t n = *n_p;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        if (i == 0 || (pairs[i] >> 32) != (pairs[i - 1] >> 32)) owner_start[pos[i]] = i;
    if (blockIdx.x == 0 && threadIdx.x == 0) owner_start[*n_owner] = n;
}

// ---- memory-free fallback for vertices whose map does not fit: per pair,
// m_ab from binary searches and every triangle vertex c from a's hyperedges
// (taken at the first of them that holds c), m_ac and m_bc by list intersection.
// |A & B| for two incidence lists and their first common element in list order
// (both lists are sorted by the same key, so it is the same in either list)
__device__ __forceinline__ uint32_t inter_count_min(const GraphView& g, const uint32_t* A, uint32_t na,
                                                    const uint32_t* B, uint32_t nb, uint32_t* mn) {
    if (na > nb) {
        const uint32_t* t = A; A = B; B = t;
        uint32_t n = na; na = nb; nb = n;
    }
    uint32_t c = 0, first = HGT_EMPTY;
    for (uint32_t i = 0; i < na; i++) {
        uint32_t e = A[i];
        if (v2h_contains(g, B, nb, e)) {
            if (c == 0) first = e;
            c++;
        }
    }
    *mn = first;
    return c;
}

// one wave: returns (lane 0) m_ab * w_ab in *s_out and the attributed triangle sum in *t_out
__device__ void iv_pair_direct(const IvParams& P, uint32_t a, uint32_t b, uint32_t* pre, uint64_t* s_out,
                               uint64_t* t_out) {
    const int lane = threadIdx.x & 63;
    uint32_t la = P.g.v_len[a], lb = P.g.v_len[b];
    if (lb < la) { uint32_t t = a; a = b; b = t; t = la; la = lb; lb = t; }
    const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
    const uint32_t* A = P.g.v2h + P.g.v_off[a];
    const uint32_t* B = P.g.v2h + P.g.v_off[b];
    uint64_t m = 0, w = 0;
    for (uint32_t i = lane; i < la; i += 64) {
        uint32_t h = A[i];
        uint32_t d = P.g.h_len[h];
        if (contains_u32(P.g.h2v + P.g.h_off[h], d, b)) { m++; w += d - 2; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        m += __shfl_xor(m, o, 64);
        w += __shfl_xor(w, o, 64);
    }
    *s_out = m * w;
    uint64_t t_sum = 0;
    if (m) {
        for (uint32_t base = 0; base < la; base += 64) {
            uint32_t cnt = la - base < 64 ? la - base : 64;
            uint32_t d = 0;
            if ((uint32_t)lane < cnt) d = P.g.h_len[A[base + lane]];
            uint32_t inc = d;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                uint32_t t = __shfl_up(inc, o, 64);
                if (lane >= o) inc += t;
            }
            if ((uint32_t)lane < cnt) pre[lane + 1] = inc;
            if (lane == 0) pre[0] = 0;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
            uint32_t tot = pre[cnt];
            for (uint32_t p = lane; p < tot; p += 64) {
                uint32_t k = seg_of<uint32_t>(pre, cnt, p);
                uint32_t hk = A[base + k];
                uint32_t c = P.g.h2v[P.g.h_off[hk] + (p - pre[k])];
                if (c == a || c == b) continue;
                const uint32_t* C = P.g.v2h + P.g.v_off[c];
                uint32_t lc = P.g.v_len[c];
                uint32_t first;
                uint32_t mac = inter_count_min(P.g, A, la, C, lc, &first);
                if (first != hk) continue;
                uint32_t dummy;
                uint32_t mbc = inter_count_min(P.g, B, lb, C, lc, &dummy);
                if (mbc == 0) continue;
                if (c < hi && touched(P.tab, P.tab_mask, lo, c)) continue;
                if (c < lo && touched(P.tab, P.tab_mask, hi, c)) continue;
                t_sum += m * (uint64_t)mac * (uint64_t)mbc;
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) t_sum += __shfl_xor(t_sum, o, 64);
    *t_out = t_sum;
}

struct IvSh {
    uint32_t a, la, L, cap, defer, stop, idx;
    uint64_t off_a, p0, p1;
    uint32_t ws[NWAVE];
};

// The clique map of an owner: open addressing over cap slots, kept as three
// arrays (keys, m, w) so that the probes of a wave read consecutive key words
// rather than every fourth one (fewer LDS bank conflicts); 4 words per slot.
struct IvMap {
    uint32_t* key;
    uint32_t* m;
    uint64_t* w;  // 8-byte aligned
    uint32_t cap;
};

__device__ __forceinline__ IvMap iv_map(uint32_t* arena, uint32_t cap) {
    const uint32_t c2 = (cap + 1) & ~1u;
    return IvMap{arena, arena + c2, (uint64_t*)(arena + 2 * c2), cap};
}

__device__ __forceinline__ uint32_t map_find(const IvMap& mp, uint32_t key) {
    const uint32_t cap = mp.cap;
    uint32_t s = (uint32_t)(((uint64_t)(key * 2654435761u) * cap) >> 32);
    for (uint32_t probe = 0; probe < cap; probe++) {
        uint32_t k = mp.key[s];
        if (k == key) return s;
        if (k == HGT_EMPTY) return HGT_EMPTY;
        s = s + 1 == cap ? 0 : s + 1;
    }
    return HGT_EMPTY;
}

__device__ __forceinline__ void map_add(const IvMap& mp, uint32_t key, uint32_t w) {
    const uint32_t cap = mp.cap;
    uint32_t s = (uint32_t)(((uint64_t)(key * 2654435761u) * cap) >> 32);
    for (uint32_t probe = 0; probe < cap; probe++) {
        uint32_t k = __atomic_load_n(&mp.key[s], __ATOMIC_RELAXED);
        if (k == HGT_EMPTY) {
            uint32_t prev = atomicCAS(&mp.key[s], HGT_EMPTY, key);
            if (prev == HGT_EMPTY || prev == key) break;
        } else if (k == key) {
            break;
        }
        s = s + 1 == cap ? 0 : s + 1;
    }
    atomicAdd(&mp.m[s], 1u);
    atomicAdd((unsigned long long*)&mp.w[s], (unsigned long long)w);
}

template <int STAGE>
__device__ void iv_body(const IvParams& P, uint32_t* arena, uint32_t arena_words, IvSh& sh, uint64_t* acc) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    __shared__ uint32_t wpre[NWAVE][65];
    const uint64_t n_pairs = *P.n_pairs;
    uint64_t s_sum = 0, t_sum = 0, bytes = 0;
    for (;;) {
        if (tid == 0) {
            uint32_t q = atomicAdd(&P.queue[STAGE], 1u);
            uint64_t n = STAGE == 0 ? *P.n_owners : (uint64_t)P.count[STAGE - 1];
            sh.stop = q >= n;
            if (!sh.stop) {
                uint32_t oi = STAGE == 0 ? q : (STAGE == 1 ? P.list[q] : P.list2[q]);
                sh.idx = oi;
                sh.p0 = P.owner_start[oi];
                sh.p1 = P.owner_start[oi + 1];
                uint32_t a = (uint32_t)(P.pairs[sh.p0] >> 32);
                sh.a = a;
                sh.la = P.g.v_len[a];
                sh.off_a = P.g.v_off[a];
            }
        }
        __syncthreads();
        if (sh.stop) break;
        const uint32_t a = sh.a, la = sh.la;
        const uint32_t* A = P.g.v2h + sh.off_a;
        // L = sum of the cardinalities of a's hyperedges
        uint32_t part = 0;
        for (uint32_t i = tid; i < la; i += HGT_WG) part += P.g.h_len[A[i]];
        uint32_t L;
        wg_scan_u32(part, sh.ws, &L);
        if (tid == 0) {
            sh.L = L;
            sh.cap = L + L / 2 + 32;
            sh.defer = (4ull * sh.cap + 2 > arena_words || P.force_direct || STAGE < P.force_stage) ? 1u : 0u;
        }
        __syncthreads();
        if (sh.defer && STAGE < 2) {
            if (tid == 0) {
                if (STAGE == 0) P.list[atomicAdd(&P.count[0], 1u)] = sh.idx;
                else P.list2[atomicAdd(&P.count[1], 1u)] = sh.idx;
            }
            __syncthreads();
            continue;
        }
        if (sh.defer) {
            // too large for any map: pair by pair without one
            for (uint64_t q = sh.p0 + wave; q < sh.p1; q += NWAVE) {
                uint64_t so, to;
                iv_pair_direct(P, a, (uint32_t)P.pairs[q], wpre[wave], &so, &to);
                if (lane == 0) {
                    s_sum += so;
                    t_sum += to;
                }
            }
            __syncthreads();
            continue;
        }
        const uint32_t cap = sh.cap;
        const IvMap mp = iv_map(arena, cap);
        for (uint32_t s = tid; s < cap; s += HGT_WG) {
            mp.key[s] = HGT_EMPTY;
            mp.m[s] = 0;
            mp.w[s] = 0;
        }
        __syncthreads();
        // M_a from a's hyperedges: one wave per hyperedge, lanes over members
        for (uint32_t i = wave; i < la; i += NWAVE) {
            uint32_t h = A[i];
            uint32_t d = P.g.h_len[h];
            const uint32_t* M = P.g.h2v + P.g.h_off[h];
            for (uint32_t k = lane; k < d; k += 64) {
                uint32_t w = M[k];
                if (w != a) map_add(mp, w, d - 2);
            }
        }
        __syncthreads();
        if (lane == 0 && P.stats) bytes += 4ull * (la + L) / NWAVE;
        // touched pairs (a, b), b > a: one wave each
        for (uint64_t q = sh.p0 + wave; q < sh.p1; q += NWAVE) {
            const uint32_t b = (uint32_t)P.pairs[q];
            uint32_t sb = map_find(mp, b);
            uint64_t m_ab = 0, w_ab = 0;
            if (sb != HGT_EMPTY) {
                m_ab = mp.m[sb];
                w_ab = mp.w[sb];
            }
            if (lane == 0) s_sum += m_ab * w_ab;
            if (m_ab == 0) continue;
            const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
            const uint32_t lb = P.g.v_len[b];
            const uint32_t* B = P.g.v2h + P.g.v_off[b];
            uint64_t sum = 0;
            for (uint32_t base = 0; base < lb; base += 64) {
                uint32_t cnt = lb - base < 64 ? lb - base : 64;
                uint32_t d = 0;
                if ((uint32_t)lane < cnt) d = P.g.h_len[B[base + lane]];
                uint32_t inc = d;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    uint32_t t = __shfl_up(inc, o, 64);
                    if (lane >= o) inc += t;
                }
                if ((uint32_t)lane < cnt) wpre[wave][lane + 1] = inc;
                if (lane == 0) wpre[wave][0] = 0;
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
                __builtin_amdgcn_wave_barrier();
                const uint32_t tot = wpre[wave][cnt];
                if (P.stats && lane == 0) bytes += 4ull * (cnt + tot);
                for (uint32_t p = lane; p < tot; p += 64) {
                    uint32_t k = seg_of<uint32_t>(wpre[wave], cnt, p);
                    uint32_t hk = B[base + k];
                    uint32_t w = P.g.h2v[P.g.h_off[hk] + (p - wpre[wave][k])];
                    if (w == a || w == b) continue;
                    uint32_t sw = map_find(mp, w);
                    if (sw == HGT_EMPTY) continue;
                    if (w < hi && touched(P.tab, P.tab_mask, lo, w)) continue;
                    if (w < lo && touched(P.tab, P.tab_mask, hi, w)) continue;
                    sum += mp.m[sw];
                }
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
                __builtin_amdgcn_wave_barrier();
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
            if (lane == 0) t_sum += m_ab * sum;
        }
        __syncthreads();
    }
    if (lane == 0) {
        if (s_sum) atomicAdd((unsigned long long*)&acc[0], (unsigned long long)s_sum);
        if (t_sum) atomicAdd((unsigned long long*)&acc[1], (unsigned long long)t_sum);
        if (bytes && P.stats) atomicAdd((unsigned long long*)&P.stats[ST_IV_BYTES], (unsigned long long)bytes);
    }
}

__global__ void __launch_bounds__(HGT_WG) k_iv_lds(IvParams P) {
    __shared__ __attribute__((aligned(16))) uint32_t arena[IV_ARENA];
    __shared__ IvSh sh;
    __shared__ uint64_t acc[2];
    __shared__ uint32_t bad;
    if (threadIdx.x == 0) bad = *((volatile const int32_t*)P.status) != 0 ? 1u : 0u;
    if (threadIdx.x < 2) acc[threadIdx.x] = 0;
    __syncthreads();
    if (bad) return;  // read once per workgroup: every thread leaves before the body's barriers
    iv_body<0>(P, arena, IV_ARENA, sh, acc);
    __syncthreads();
    if (threadIdx.x < 2 && acc[threadIdx.x]) atomicAdd((unsigned long long*)&P.out[threadIdx.x], (unsigned long long)acc[threadIdx.x]);
}

template <int STAGE>
__global__ void __launch_bounds__(HGT_WG) k_iv_global(IvParams P) {
    __shared__ IvSh sh;
    __shared__ uint64_t acc[2];
    __shared__ uint32_t bad;
    if (threadIdx.x == 0) bad = *((volatile const int32_t*)P.status) != 0 ? 1u : 0u;
    if (threadIdx.x < 2) acc[threadIdx.x] = 0;
    __syncthreads();
    if (bad) return;  // read once per workgroup: every thread leaves before the body's barriers
    uint32_t* arena = STAGE == 1 ? P.garena + (uint64_t)blockIdx.x * P.garena_words
                                 : P.garena2 + (uint64_t)blockIdx.x * P.garena2_words;
    iv_body<STAGE>(P, arena, (uint32_t)(STAGE == 1 ? P.garena_words : P.garena2_words), sh, acc);
    __syncthreads();
    if (threadIdx.x < 2 && acc[threadIdx.x]) atomicAdd((unsigned long long*)&P.out[threadIdx.x], (unsigned long long)acc[threadIdx.x]);
}

}  // namespace

void iv_touched_build(const uint64_t* canon, const uint64_t* own, const uint64_t* n_pairs, uint64_t* tab,
                      uint64_t tab_slots, uint64_t* head, uint64_t* owner_start, uint64_t* n_owners, uint64_t pairs_cap,
                      void* scan_tmp, hipStream_t s) {
    hgt_fill_u64(tab, ~0ull, tab_slots, s);
    k_iv_hash_build<<<2048, 256, 0, s>>>(canon, n_pairs, tab, tab_slots - 1);
    k_iv_owner_heads<<<2048, 256, 0, s>>>(own, n_pairs, head);
    hgt_scan_u64(head, head, pairs_cap, n_pairs, n_owners, scan_tmp, s);
    k_iv_owner_list<<<2048, 256, 0, s>>>(own, n_pairs, head, owner_start, n_owners);
}

void triad_iv_launch(IvParams& P, unsigned grid_lds, unsigned grid_global, unsigned grid_global2, hipStream_t s) {
    hgt_fill_u32(P.queue, 0, 3, s);  // the three stages' queues
    hgt_fill_u32(P.count, 0, 2, s);  // owners moved on by stages 0 and 1
    k_iv_lds<<<grid_lds, HGT_WG, 0, s>>>(P);
    k_iv_global<1><<<grid_global, HGT_WG, 0, s>>>(P);
    k_iv_global<2><<<grid_global2, HGT_WG, 0, s>>>(P);
}
