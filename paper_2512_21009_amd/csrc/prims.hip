// prims.hip -- device-wide exclusive scan and LSD radix sort for gfx950.
//
// Both are tile-based with 256-thread workgroups (four wave64s) and 2048
// elements per tile: a reduce pass writes one partial per tile, a single
// workgroup scans the partials, and a down-sweep pass finishes every tile.
// Counts may live in device memory (n_dev) so the host can launch with an
// upper bound and no synchronisation; tiles past the live count exit early.
#include "hgt_dev.h"

namespace {

constexpr int ITEMS = 8;
constexpr int TILE = HGT_WG * ITEMS;  // 2048

__device__ __forceinline__ uint64_t read_n(const uint64_t* n_dev, uint64_t n_max) {
    if (!n_dev) return n_max;
    uint64_t n = *n_dev;
    return n < n_max ? n : n_max;
}

// Exclusive scan of one value per thread across the workgroup.
__device__ __forceinline__ uint64_t wg_exclusive(uint64_t v, uint64_t* wave_sums, uint64_t* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint64_t t = __shfl_up(x, o, 64);
        if (lane >= o) x += t;
    }
    if (lane == 63) wave_sums[wave] = x;
    __syncthreads();
    uint64_t pre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < HGT_WG / 64; w++) {
        uint64_t s = wave_sums[w];
        if (w < wave) pre += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return pre + x - v;
}

__global__ void __launch_bounds__(HGT_WG) k_scan_reduce(const uint64_t* __restrict__ in, uint64_t n_max,
                                                        const uint64_t* n_dev, uint64_t* __restrict__ tile_sums) {
    __shared__ uint64_t ws[HGT_WG / 64];
    const uint64_t n = read_n(n_dev, n_max);
    const uint64_t base = (uint64_t)blockIdx.x * TILE;
    uint64_t s = 0;
    if (base < n) {
        for (int i = 0; i < ITEMS; i++) {
            uint64_t e = base + (uint64_t)i * HGT_WG + threadIdx.x;
            if (e < n) s += in[e];
        }
    }
    uint64_t tot;
    wg_exclusive(s, ws, &tot);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(HGT_WG) k_scan_tiles(uint64_t* tile_sums, uint64_t n_tiles, uint64_t* total) {
    __shared__ uint64_t ws[HGT_WG / 64];
    uint64_t carry = 0;
    for (uint64_t base = 0; base < n_tiles; base += HGT_WG) {
        uint64_t e = base + threadIdx.x;
        uint64_t v = e < n_tiles ? tile_sums[e] : 0;
        uint64_t tot;
        uint64_t ex = wg_exclusive(v, ws, &tot);
        if (e < n_tiles) tile_sums[e] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

__global__ void __launch_bounds__(HGT_WG) k_scan_down(const uint64_t* in, uint64_t* out, uint64_t n_max,
                                                      const uint64_t* n_dev, const uint64_t* __restrict__ tile_sums) {
    __shared__ uint64_t buf[TILE];
    __shared__ uint64_t ws[HGT_WG / 64];
    const uint64_t n = read_n(n_dev, n_max);
    const uint64_t base = (uint64_t)blockIdx.x * TILE;
    if (base >= n) return;
    for (int i = 0; i < ITEMS; i++) {  // striped, coalesced load
        uint64_t e = base + (uint64_t)i * HGT_WG + threadIdx.x;
        buf[i * HGT_WG + threadIdx.x] = e < n ? in[e] : 0;
    }
    __syncthreads();
    uint64_t loc[ITEMS];
    uint64_t s = 0;
    for (int i = 0; i < ITEMS; i++) {  // blocked per thread
        loc[i] = s;
        s += buf[threadIdx.x * ITEMS + i];
    }
    uint64_t tot;
    uint64_t pre = wg_exclusive(s, ws, &tot) + tile_sums[blockIdx.x];
    for (int i = 0; i < ITEMS; i++) buf[threadIdx.x * ITEMS + i] = pre + loc[i];
    __syncthreads();
    for (int i = 0; i < ITEMS; i++) {
        uint64_t e = base + (uint64_t)i * HGT_WG + threadIdx.x;
        if (e < n) out[e] = buf[i * HGT_WG + threadIdx.x];
    }
}

// ---- radix sort --------------------------------------------------------
constexpr int RADIX = 256;

__global__ void __launch_bounds__(HGT_WG) k_rs_hist(const uint64_t* __restrict__ keys, uint64_t n_max,
                                                    const uint64_t* n_dev, int shift, uint64_t n_tiles,
                                                    uint64_t* __restrict__ hist) {
    __shared__ uint32_t h[RADIX];
    const uint64_t n = read_n(n_dev, n_max);
    const uint64_t base = (uint64_t)blockIdx.x * TILE;
    h[threadIdx.x] = 0;
    __syncthreads();
    if (base < n) {
        for (int i = 0; i < ITEMS; i++) {
            uint64_t e = base + (uint64_t)i * HGT_WG + threadIdx.x;
            if (e < n) atomicAdd(&h[(keys[e] >> shift) & (RADIX - 1)], 1u);
        }
    }
    __syncthreads();
    hist[(uint64_t)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

__global__ void __launch_bounds__(HGT_WG) k_rs_scatter(const uint64_t* __restrict__ in, uint64_t* __restrict__ out,
                                                       uint64_t n_max, const uint64_t* n_dev, int shift,
                                                       uint64_t n_tiles, const uint64_t* __restrict__ hist) {
    __shared__ uint64_t base_d[RADIX];
    __shared__ uint32_t running[RADIX];
    __shared__ uint32_t wcnt[HGT_WG / 64][RADIX];
    const uint64_t n = read_n(n_dev, n_max);
    const uint64_t base = (uint64_t)blockIdx.x * TILE;
    if (base >= n) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    base_d[threadIdx.x] = hist[(uint64_t)threadIdx.x * n_tiles + blockIdx.x];
    running[threadIdx.x] = 0;
    const uint64_t lt_mask = (lane == 0) ? 0ull : ((1ull << lane) - 1ull);
    for (int i = 0; i < ITEMS; i++) {
        for (int w = 0; w < HGT_WG / 64; w++) wcnt[w][threadIdx.x] = 0;
        __syncthreads();
        uint64_t e = base + (uint64_t)i * HGT_WG + threadIdx.x;
        bool valid = e < n;
        uint64_t key = valid ? in[e] : 0;
        uint32_t d = (uint32_t)(key >> shift) & (RADIX - 1);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            uint64_t bb = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? bb : ~bb;
        }
        uint32_t lower = __popcll(peers & lt_mask);
        if (valid && lower == 0) wcnt[wave][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t off = running[d] + lower;
            for (int w = 0; w < wave; w++) off += wcnt[w][d];
            out[base_d[d] + off] = key;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < HGT_WG / 64; w++) add += wcnt[w][threadIdx.x];
        running[threadIdx.x] += add;
        __syncthreads();
    }
}

template <class T>
__global__ void k_fill(T* p, T v, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) p[i] = v;
}

inline uint64_t n_tiles_of(uint64_t n) { return (n + TILE - 1) / TILE; }

}  // namespace

size_t hgt_scan_tmp_bytes(uint64_t n_max) { return (n_tiles_of(n_max) + 1) * sizeof(uint64_t); }

void hgt_scan_u64(const uint64_t* in, uint64_t* out, uint64_t n_max, const uint64_t* n_dev, uint64_t* total,
                  void* tmp, hipStream_t s) {
    uint64_t nt = n_tiles_of(n_max);
    uint64_t* ts = (uint64_t*)tmp;
    if (nt == 0) {
        if (total) k_fill<uint64_t><<<1, 64, 0, s>>>(total, 0, 1);
        return;
    }
    k_scan_reduce<<<(unsigned)nt, HGT_WG, 0, s>>>(in, n_max, n_dev, ts);
    k_scan_tiles<<<1, HGT_WG, 0, s>>>(ts, nt, total);
    k_scan_down<<<(unsigned)nt, HGT_WG, 0, s>>>(in, out, n_max, n_dev, ts);
}

size_t hgt_radix_tmp_bytes(uint64_t n_max) {
    uint64_t nt = n_tiles_of(n_max);
    return (uint64_t)RADIX * nt * sizeof(uint64_t) + hgt_scan_tmp_bytes((uint64_t)RADIX * nt);
}

void hgt_radix_sort_u64(uint64_t* keys, uint64_t* alt, uint64_t n_max, const uint64_t* n_dev, int bits, void* tmp,
                        hipStream_t s) {
    uint64_t nt = n_tiles_of(n_max);
    if (nt == 0 || bits <= 0) return;
    uint64_t* hist = (uint64_t*)tmp;
    void* stmp = (void*)(hist + (uint64_t)RADIX * nt);
    int passes = (bits + 7) / 8;
    uint64_t *src = keys, *dst = alt;
    for (int p = 0; p < passes; p++) {
        int shift = 8 * p;
        k_rs_hist<<<(unsigned)nt, HGT_WG, 0, s>>>(src, n_max, n_dev, shift, nt, hist);
        hgt_scan_u64(hist, hist, (uint64_t)RADIX * nt, nullptr, nullptr, stmp, s);
        k_rs_scatter<<<(unsigned)nt, HGT_WG, 0, s>>>(src, dst, n_max, n_dev, shift, nt, hist);
        uint64_t* t = src; src = dst; dst = t;
    }
    if (src != keys) hipMemcpyAsync(keys, src, n_max * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
}

void hgt_fill_u64(uint64_t* p, uint64_t v, uint64_t n, hipStream_t s) {
    if (!n) return;
    uint64_t g = (n + 255) / 256;
    k_fill<uint64_t><<<(unsigned)(g > 4096 ? 4096 : g), 256, 0, s>>>(p, v, n);
}

void hgt_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s) {
    if (!n) return;
    uint64_t g = (n + 255) / 256;
    k_fill<uint32_t><<<(unsigned)(g > 4096 ? 4096 : g), 256, 0, s>>>(p, v, n);
}
