// hops.hip -- horizontal operations: incident-vertex insertions and deletions
// inside live hyperedges (Sec. III-B, "Incident vertex insertion/deletion").
//
// A batch of (hyperedge, vertex, insert?) ops is sorted by (hyperedge, vertex),
// validated (live hyperedge, vertex in range, no pair twice, a deleted vertex
// is a member, an inserted one is not, no hyperedge left empty or above the
// largest cardinality) and grouped per modified hyperedge.  The new member
// row of every modified hyperedge is then merged from its old sorted row and
// its sorted ops.  The library applies the result as one batch that deletes
// the modified hyperedges and inserts their new rows under the same IDs with
// their timestamps and arrival sequences kept, so the triad kernels count the
// change exactly as for any other batch.  Nothing here changes the graph.
#include "hops.h"

namespace {

__device__ __forceinline__ bool bad_status(const int32_t* st) { return *((volatile const int32_t*)st) != 0; }

__global__ void k_vop_reset(DevScalars* sc, VopSummary* sum) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        sc->status = 0;
        VopSummary z = {};
        *sum = z;
    }
}

// key = hyperedge << (vb + 1) | vertex << 1 | insert
__global__ void k_vop_keys(const uint32_t* __restrict__ eid, const uint32_t* __restrict__ vtx,
                           const uint8_t* __restrict__ ins, uint64_t n, int vb, uint32_t n_vertices,
                           const uint64_t* __restrict__ free_bm, DevScalars* sc, uint64_t* keys) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t h = eid[i], v = vtx[i];
    if ((uint64_t)h >= sc->next_id || ((free_bm[h >> 6] >> (h & 63)) & 1ull)) {
        set_status(&sc->status, HGT_ENOENT);
        keys[i] = 0;
        return;
    }
    if (v >= n_vertices) {
        set_status(&sc->status, HGT_EINVAL);
        keys[i] = 0;
        return;
    }
    keys[i] = ((uint64_t)h << (vb + 1)) | ((uint64_t)v << 1) | (ins[i] ? 1ull : 0ull);
}

// per sorted op: repeated pair, membership check, segment heads, insert flags
__global__ void k_vop_check(const uint64_t* __restrict__ keys, uint64_t n, int vb, const uint64_t* __restrict__ h_off,
                            const uint32_t* __restrict__ h_len, const uint32_t* __restrict__ h2v, DevScalars* sc,
                            uint64_t* head, uint64_t* insf) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (bad_status(&sc->status)) return;
    const uint64_t k = keys[i];
    const uint32_t h = (uint32_t)(k >> (vb + 1));
    const uint32_t v = (uint32_t)((k >> 1) & ((1ull << vb) - 1));
    const bool in = k & 1ull;
    if (i > 0 && (keys[i - 1] >> 1) == (k >> 1)) set_status(&sc->status, HGT_EINVAL);
    const bool member = contains_u32(h2v + h_off[h], h_len[h], v);
    if (member == in) set_status(&sc->status, HGT_EINVAL);
    head[i] = (i == 0 || (keys[i - 1] >> (vb + 1)) != h) ? 1ull : 0ull;
    insf[i] = in ? 1ull : 0ull;
}

// head[] scanned (exclusive) into hidx: segment starts and modified IDs
__global__ void k_vop_segments(const uint64_t* __restrict__ keys, uint64_t n, int vb,
                               const uint64_t* __restrict__ hidx, const uint64_t* n_mod_p, DevScalars* sc,
                               uint32_t* mod_ids, uint64_t* seg) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (bad_status(&sc->status)) return;
    const uint64_t k = keys[i];
    const uint32_t h = (uint32_t)(k >> (vb + 1));
    if (i == 0) seg[*n_mod_p] = n;
    if (i == 0 || (keys[i - 1] >> (vb + 1)) != h) {
        mod_ids[hidx[i]] = h;
        seg[hidx[i]] = i;
    }
}

// per modified hyperedge: new cardinality, timestamp; totals in the summary
__global__ void k_vop_cards(const uint32_t* __restrict__ mod_ids, const uint64_t* __restrict__ seg,
                            const uint64_t* n_mod_p, const uint64_t* __restrict__ ins_pre, const uint32_t* __restrict__ h_len,
                            const int64_t* __restrict__ h_ts, DevScalars* sc, uint64_t* card, int64_t* ts,
                            VopSummary* sum) {
    uint64_t m = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t nm = *n_mod_p;
    if (m == 0) sum->n_mod = nm;
    if (m >= nm) return;
    if (bad_status(&sc->status)) return;
    const uint32_t h = mod_ids[m];
    const uint64_t s = seg[m], e = seg[m + 1];
    const uint64_t n_in = ins_pre[e] - ins_pre[s], n_out = (e - s) - n_in;
    const uint64_t c = (uint64_t)h_len[h] + n_in - n_out;
    if (c < 1 || c > HGT_MAX_CARD) set_status(&sc->status, HGT_EINVAL);
    card[m] = c;
    if (ts) ts[m] = h_ts[h];
    atomicAdd((unsigned long long*)&sum->n_members, (unsigned long long)c);
}

__global__ void k_vop_finish(const DevScalars* sc, VopSummary* sum) {
    if (threadIdx.x == 0 && blockIdx.x == 0) sum->status = sc->status;
}

// one wave per modified hyperedge: its old row minus the deleted vertices plus
// the inserted ones, ascending (both inputs are sorted by vertex)
__global__ void k_vop_rows(const uint32_t* __restrict__ mod_ids, uint64_t n_mod, const uint64_t* __restrict__ seg,
                           const uint64_t* __restrict__ keys, int vb, const uint64_t* __restrict__ ins_pre,
                           const uint64_t* __restrict__ h_off, const uint32_t* __restrict__ h_len,
                           const uint32_t* __restrict__ h2v, const uint64_t* __restrict__ new_off, uint32_t* out) {
    const int lane = threadIdx.x & 63;
    const uint64_t m = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (m >= n_mod) return;
    const uint32_t h = mod_ids[m];
    const uint32_t* row = h2v + h_off[h];
    const uint32_t len = h_len[h];
    const uint64_t s = seg[m], n_ops = seg[m + 1] - s;
    const uint64_t vmask = (1ull << vb) - 1;
    uint32_t* dst = out + new_off[m];
    auto op_v = [&](uint64_t j) { return (uint32_t)((keys[s + j] >> 1) & vmask); };
    // ops with vertex below x (binary search over the segment)
    auto ops_below = [&](uint32_t x) {
        uint64_t lo = 0, hi = n_ops;
        while (lo < hi) {
            uint64_t mid = (lo + hi) >> 1;
            if (op_v(mid) < x) lo = mid + 1; else hi = mid;
        }
        return lo;
    };
    for (uint32_t i = lane; i < len; i += 64) {
        const uint32_t u = row[i];
        const uint64_t p = ops_below(u);
        if (p < n_ops && op_v(p) == u) continue;  // deleted (an insert of a member was rejected)
        const uint64_t ins_before = ins_pre[s + p] - ins_pre[s];
        const uint64_t del_before = p - ins_before;
        dst[i - del_before + ins_before] = u;
    }
    for (uint64_t j = lane; j < n_ops; j += 64) {
        if (!(keys[s + j] & 1ull)) continue;
        const uint32_t v = op_v(j);
        const uint64_t ins_before = ins_pre[s + j] - ins_pre[s];
        const uint64_t del_before = j - ins_before;
        dst[lower_bound_u32(row, len, v) - del_before + ins_before] = v;
    }
}

inline unsigned blocks_for(uint64_t n, unsigned per = 256) {
    uint64_t b = (n + per - 1) / per;
    return (unsigned)(b ? b : 1);
}

}  // namespace

void vops_plan(const VopIn& in, VopScratch& w, hipStream_t s) {
    const uint64_t n = in.n;
    k_vop_reset<<<1, 64, 0, s>>>(in.sc, w.sum);
    k_vop_keys<<<blocks_for(n), 256, 0, s>>>(in.edge_ids, in.vertices, in.insert, n, in.vb, in.n_vertices, in.free_bm,
                                             in.sc, w.keys);
    hgt_radix_sort_u64(w.keys, w.keys_alt, n, nullptr, in.hb + in.vb + 1, w.sort_tmp, s);
    k_vop_check<<<blocks_for(n), 256, 0, s>>>(w.keys, n, in.vb, in.h_off, in.h_len, in.h2v, in.sc, w.head, w.ins_pre);
    hgt_scan_u64(w.head, w.head, n, nullptr, w.n_mod, w.scan_tmp, s);
    // inclusive end: ins_pre[n] = total inserts
    hgt_scan_u64(w.ins_pre, w.ins_pre, n, nullptr, w.ins_pre + n, w.scan_tmp, s);
    k_vop_segments<<<blocks_for(n), 256, 0, s>>>(w.keys, n, in.vb, w.head, w.n_mod, in.sc, w.mod_ids, w.seg);
    k_vop_cards<<<blocks_for(n), 256, 0, s>>>(w.mod_ids, w.seg, w.n_mod, w.ins_pre, in.h_len, in.h_ts, in.sc, w.card,
                                              w.ts, w.sum);
    k_vop_finish<<<1, 64, 0, s>>>(in.sc, w.sum);
}

void vops_rows(const VopIn& in, VopScratch& w, uint64_t n_mod, hipStream_t s) {
    if (n_mod == 0) return;
    // exclusive offsets of the new rows (n_mod + 1 entries)
    hgt_scan_u64(w.card, w.new_off, n_mod, nullptr, w.new_off + n_mod, w.scan_tmp, s);
    k_vop_rows<<<blocks_for(n_mod * 64), 256, 0, s>>>(w.mod_ids, n_mod, w.seg, w.keys, in.vb, w.ins_pre, in.h_off,
                                                      in.h_len, in.h2v, w.new_off, w.members);
}
