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
// (after it); the difference is the delta.  A triangle with several touched
// pairs is counted at the smallest one.
//
// One wave per touched pair (a, b): the lanes walk the members w of the
// hyperedges incident to the endpoint with the shorter incidence list; a w is
// taken at the first such hyperedge that contains it (found as the smallest
// common element of the two incidence lists, which also gives m_aw).
#include "triad.h"

namespace {

// |A & B| and the smallest common element of two ascending lists
__device__ __forceinline__ uint32_t inter_count_min(const uint32_t* A, uint32_t na, const uint32_t* B, uint32_t nb,
                                                    uint32_t* mn) {
    if (na > nb) {
        const uint32_t* t = A; A = B; B = t;
        uint32_t n = na; na = nb; nb = n;
    }
    uint32_t c = 0, first = HGT_EMPTY;
    for (uint32_t i = 0; i < na; i++) {
        uint32_t e = A[i];
        if (contains_u32(B, nb, e)) {
            if (c == 0) first = e;
            c++;
        }
    }
    *mn = first;
    return c;
}

__device__ __forceinline__ bool pair_touched_before(const uint64_t* pairs, uint64_t n, uint32_t x, uint32_t y,
                                                    uint64_t key_p) {
    uint64_t k = x < y ? ((uint64_t)x << 32 | y) : ((uint64_t)y << 32 | x);
    if (k >= key_p) return false;
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        uint64_t mid = (lo + hi) >> 1;
        if (pairs[mid] < k) lo = mid + 1; else hi = mid;
    }
    return lo < n && pairs[lo] == k;
}

__global__ void __launch_bounds__(HGT_WG) k_iv_pairs(IvParams P) {
    __shared__ uint64_t acc[2];
    __shared__ uint32_t pre[HGT_WG / 64][65];
    if (*((volatile const int32_t*)P.status) != 0) return;
    if (threadIdx.x < 2) acc[threadIdx.x] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t n = *P.n_pairs;
    uint64_t s_sum = 0, t_sum = 0, bytes = 0;
    for (uint64_t q = (uint64_t)blockIdx.x * (HGT_WG / 64) + wave; q < n; q += (uint64_t)gridDim.x * (HGT_WG / 64)) {
        const uint64_t key = P.pairs[q];
        uint32_t a = (uint32_t)(key >> 32), b = (uint32_t)key;
        uint32_t la = P.g.v_len[a], lb = P.g.v_len[b];
        if (lb < la) { uint32_t t = a; a = b; b = t; t = la; la = lb; lb = t; }
        const uint32_t* A = P.g.v2h + P.g.v_off[a];
        const uint32_t* B = P.g.v2h + P.g.v_off[b];
        // m_ab and w_ab: hyperedges of a that contain b
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
        if (lane == 0) {
            s_sum += m * w;
            bytes += 4ull * la;
        }
        if (m == 0) continue;
        // triangles {a, b, c}: c in a hyperedge of a, taken at its first one
        for (uint32_t base = 0; base < la; base += 64) {
            uint32_t cnt = la - base < 64 ? la - base : 64;
            uint32_t h = 0, d = 0;
            if ((uint32_t)lane < cnt) {
                h = A[base + lane];
                d = P.g.h_len[h];
            }
            uint32_t inc = d;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                uint32_t t = __shfl_up(inc, o, 64);
                if (lane >= o) inc += t;
            }
            if ((uint32_t)lane < cnt) pre[wave][lane + 1] = inc;
            if (lane == 0) pre[wave][0] = 0;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
            uint32_t tot = pre[wave][cnt];
            for (uint32_t p = lane; p < tot; p += 64) {
                uint32_t k = seg_of<uint32_t>(pre[wave], cnt, p);
                uint32_t hk = A[base + k];
                uint32_t c = P.g.h2v[P.g.h_off[hk] + (p - pre[wave][k])];
                if (c == a || c == b) continue;
                const uint32_t* C = P.g.v2h + P.g.v_off[c];
                uint32_t lc = P.g.v_len[c];
                bytes += 4ull * (1 + lc);
                uint32_t first;
                uint32_t mac = inter_count_min(A, la, C, lc, &first);
                if (first != hk) continue;  // c already met in an earlier hyperedge of a
                uint32_t dummy;
                uint32_t mbc = inter_count_min(B, lb, C, lc, &dummy);
                if (mbc == 0) continue;
                if (pair_touched_before(P.pairs, n, a, c, key)) continue;
                if (pair_touched_before(P.pairs, n, b, c, key)) continue;
                t_sum += m * (uint64_t)mac * (uint64_t)mbc;
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (P.stats) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) bytes += __shfl_xor(bytes, o, 64);
        if (lane == 0 && bytes) atomicAdd((unsigned long long*)&P.stats[ST_IV_BYTES], (unsigned long long)bytes);
    }
    if (s_sum) atomicAdd((unsigned long long*)&acc[0], (unsigned long long)s_sum);
    if (t_sum) atomicAdd((unsigned long long*)&acc[1], (unsigned long long)t_sum);
    __syncthreads();
    if (threadIdx.x < 2 && acc[threadIdx.x]) atomicAdd((unsigned long long*)&P.out[threadIdx.x], (unsigned long long)acc[threadIdx.x]);
}

}  // namespace

void triad_iv_launch(IvParams& P, hipStream_t s) {
    uint64_t waves = P.pairs_cap;
    uint64_t blocks = (waves + 3) / 4;
    if (blocks > 8192) blocks = 8192;
    if (blocks == 0) return;
    k_iv_pairs<<<(unsigned)blocks, HGT_WG, 0, s>>>(P);
}
