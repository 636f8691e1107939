// triad_common.h -- device helpers shared by the triad-delta kernels.
#pragma once

#include "triad.h"

namespace tri {

constexpr int NWAVE = HGT_WG / HGT_WAVE;  // 4

// meta word of a neighbour: c (14 bits) | len << 14 | eligible << 28 | in window << 29
__device__ __forceinline__ uint32_t meta_c(uint32_t m) { return m & 0x3fffu; }
__device__ __forceinline__ uint32_t meta_len(uint32_t m) { return (m >> 14) & 0x3fffu; }
__device__ __forceinline__ bool meta_elig(uint32_t m) { return (m >> 28) & 1u; }
__device__ __forceinline__ bool meta_win(uint32_t m) { return (m >> 29) & 1u; }

__device__ __forceinline__ int venn_code(int na, int nb, int nc, int ab, int bc, int ca, int abc) {
    int c = 0;
    c |= (na - ab - ca + abc > 0) ? 1 : 0;
    c |= (nb - ab - bc + abc > 0) ? 2 : 0;
    c |= (nc - bc - ca + abc > 0) ? 4 : 0;
    c |= (ab - abc > 0) ? 8 : 0;
    c |= (bc - abc > 0) ? 16 : 0;
    c |= (ca - abc > 0) ? 32 : 0;
    c |= (abc > 0) ? 64 : 0;
    return c;
}

__device__ __forceinline__ bool key_before(int64_t ta, uint64_t sa, int64_t tb, uint64_t sb) {
    return ta < tb || (ta == tb && sa < sb);
}

// Venn code of the triple (h, x, y) relabelled in arrival order.
__device__ __forceinline__ int time_code(int64_t th, uint64_t sh, int64_t tx, uint64_t sx, int64_t ty, uint64_t sy,
                                         int nh, int nx, int ny, int hx, int xy, int hy, int hxy) {
    // rank of each label in arrival order
    int rh = (int)key_before(tx, sx, th, sh) + (int)key_before(ty, sy, th, sh);
    int rx = (int)key_before(th, sh, tx, sx) + (int)key_before(ty, sy, tx, sx);
    int lab[3];
    lab[rh] = 0;
    lab[rx] = 1;
    lab[3 - rh - rx] = 2;
    int n[3] = {nh, nx, ny};
    // pairwise intersections indexed by label pair
    auto pr = [&](int a, int b) -> int {
        int s = a + b;  // {0,1}->1 hx, {1,2}->3 xy, {0,2}->2 hy
        return s == 1 ? hx : (s == 3 ? xy : hy);
    };
    int a = lab[0], b = lab[1], c = lab[2];
    return venn_code(n[a], n[b], n[c], pr(a, b), pr(b, c), pr(c, a), hxy);
}

__device__ __forceinline__ bool within(int64_t a, int64_t b, int64_t c, int64_t w) {
    int64_t mx = a > b ? a : b, mn = a < b ? a : b;
    mx = mx > c ? mx : c;
    mn = mn < c ? mn : c;
    return mx - mn <= w;
}

// ---- hashing --------------------------------------------------------------
// Adds inc to key's value; false when every slot holds another key (the table
// is too small for the keys offered to it).
__device__ __forceinline__ bool hash_add_ok(uint32_t* keys, uint32_t* vals, uint32_t log_cap, uint32_t key,
                                            uint32_t inc) {
    uint32_t mask = (1u << log_cap) - 1u;
    uint32_t s = hash_slot(key, log_cap);
    for (uint32_t probe = 0; probe <= mask; probe++) {
        uint32_t k = __atomic_load_n(&keys[s], __ATOMIC_RELAXED);
        if (k == HGT_EMPTY) {
            uint32_t prev = atomicCAS(&keys[s], HGT_EMPTY, key);
            if (prev == HGT_EMPTY || prev == key) { atomicAdd(&vals[s], inc); return true; }
        } else if (k == key) {
            atomicAdd(&vals[s], inc);
            return true;
        }
        s = (s + 1) & mask;
    }
    return false;
}

// For tables sized for at least twice the keys offered (cannot fill up).
__device__ __forceinline__ void hash_add(uint32_t* keys, uint32_t* vals, uint32_t log_cap, uint32_t key, uint32_t inc) {
    (void)hash_add_ok(keys, vals, log_cap, key, inc);
}

// A second hash of a key, independent of hash_slot's, that splits keys into parts.
__device__ __forceinline__ uint32_t part_hash(uint32_t key) {
    uint32_t h = key * 0xcc9e2d51u;
    h ^= h >> 15;
    h *= 0x1b873593u;
    h ^= h >> 13;
    return h;
}

// returns slot index or HGT_EMPTY.  The keys are read as atomics: a table in
// global memory was filled by atomics, which bypass the CU's L1 cache.
__device__ __forceinline__ uint32_t hash_find(const uint32_t* keys, uint32_t log_cap, uint32_t key) {
    uint32_t mask = (1u << log_cap) - 1u;
    uint32_t s = hash_slot(key, log_cap);
    for (uint32_t probe = 0; probe <= mask; probe++) {
        uint32_t k = __atomic_load_n(&keys[s], __ATOMIC_RELAXED);
        if (k == key) return s;
        if (k == HGT_EMPTY) return HGT_EMPTY;
        s = (s + 1) & mask;
    }
    return HGT_EMPTY;
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// exclusive workgroup scan of one u32 per thread (all threads participate)
__device__ __forceinline__ uint32_t wg_scan_u32(uint32_t v, uint32_t* ws, uint32_t* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(x, o, 64);
        if (lane >= o) x += t;
    }
    if (lane == 63) ws[wave] = x;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NWAVE; w++) {
        uint32_t s = ws[w];
        if (w < wave) pre += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return pre + x - v;
}


struct Tables {
    uint8_t he[128];
    uint8_t tmp[128];
};

__device__ __forceinline__ void acc_add(uint64_t* acc, int cls, uint64_t v) {
    if (cls < 255) atomicAdd((unsigned long long*)&acc[cls], (unsigned long long)v);
}


}  // namespace tri
