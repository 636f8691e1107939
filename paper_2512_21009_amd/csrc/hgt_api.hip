// hgt_api.hip -- the C ABI (include/hgt.h): graph objects, batch orchestration,
// device memory management and the class tables.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hops.h"
#include "internal.h"
#include "store.h"
#include "triad.h"

namespace {

// HGT_DEBUG=1 in the environment prints every failing HIP call to stderr.
bool debug_on() {
    static const bool on = [] {
        const char* e = std::getenv("HGT_DEBUG");
        return e && *e && *e != '0';
    }();
    return on;
}

bool hip_failed(hipError_t e, const char* what, int line) {
    if (e == hipSuccess) return false;
    (void)hipGetLastError();
    if (debug_on()) std::fprintf(stderr, "hgt: %s failed at hgt_api.hip:%d: %s\n", what, line, hipGetErrorString(e));
    return true;
}

// inside a do { ... } while (0) block that sets rc
#define HIP_BRK(expr)                                    \
    if (hip_failed((expr), #expr, __LINE__)) {           \
        rc = HGT_EDEVICE;                                \
        break;                                           \
    }

#define HIP_OK(expr)                                       \
    do {                                                   \
        if (hip_failed((expr), #expr, __LINE__)) return HGT_EDEVICE; \
    } while (0)


// ---------------------------------------------------------------------------
// class tables: Venn pattern code -> class index (built from the definitions)
// ---------------------------------------------------------------------------
// label set of each region bit, labels a=bit0, b=bit1, c=bit2
constexpr int kRegionLabels[7] = {1, 2, 4, 3, 6, 5, 7};

bool is_triad_code(int code) {
    int covered = 0, meets = 0;
    for (int r = 0; r < 7; r++)
        if (code & (1 << r)) covered |= kRegionLabels[r];
    if (covered != 7) return false;
    for (int pair : {3, 6, 5}) {
        bool m = false;
        for (int r = 0; r < 7; r++)
            if ((code & (1 << r)) && (kRegionLabels[r] & pair) == pair) m = true;
        meets += m;
    }
    return meets >= 2;
}

int permute_code(int code, const int to[3]) {  // old label l becomes label to[l]
    int out = 0;
    for (int r = 0; r < 7; r++) {
        if (!(code & (1 << r))) continue;
        int labels = 0;
        for (int l = 0; l < 3; l++)
            if (kRegionLabels[r] & (1 << l)) labels |= 1 << to[l];
        for (int q = 0; q < 7; q++)
            if (kRegionLabels[q] == labels) out |= 1 << q;
    }
    return out;
}

struct ClassTables {
    uint8_t he[128], tmp[128];
    std::vector<int32_t> he_codes, tmp_codes;
    ClassTables() {
        const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
        int canon[128];
        for (int c = 0; c < 128; c++) {
            canon[c] = -1;
            if (!is_triad_code(c)) continue;
            canon[c] = c;
            for (auto& p : perms) canon[c] = std::min(canon[c], permute_code(c, p));
            tmp_codes.push_back(c);
        }
        for (int c = 0; c < 128; c++)
            if (canon[c] == c) he_codes.push_back(c);
        for (int c = 0; c < 128; c++) {
            he[c] = tmp[c] = 255;
            if (canon[c] < 0) continue;
            he[c] = (uint8_t)(std::lower_bound(he_codes.begin(), he_codes.end(), canon[c]) - he_codes.begin());
            tmp[c] = (uint8_t)(std::lower_bound(tmp_codes.begin(), tmp_codes.end(), c) - tmp_codes.begin());
        }
    }
};

const ClassTables& tables() {
    static ClassTables t;
    return t;
}

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    template <class T> T* as() const { return (T*)p; }
};

// Scratch of the no-allocation entry point (hgt_apply_batch_noalloc) on the
// calling thread: while it is set, ensure() carves buffers out of the device's
// static scratch array instead of allocating, and every allocation fails.
struct NoAllocArena {
    char* base = nullptr;  // device address of the array on the current device
    uint64_t cap = 0, used = 0;
    struct Undo {
        DevBuf* b;
        DevBuf old;
    };
    Undo undo[160];        // the buffers given arena regions, with their previous contents
    int n_undo = 0;
    char stage[4][512];    // host staging of the per-graph phase descriptors (one graph)
};
thread_local NoAllocArena* t_na = nullptr;
// Set while the post-planning half of a round is captured into a HIP graph:
// nothing may allocate, wait or upload then (all of it was done before).
thread_local int t_capture = 0;

// Launch choices the autotuner picks between (workgroups per CU of the global
// histogram stage, whether centres skip the 148 KB stage, slots of the 2-hop
// kernels' per-wave hashes); t_tune overrides the graph's own for one round.
struct TuneChoice {
    int wg_per_cu, skip_lds148;
    uint32_t wave_slots;
    uint64_t e2_2hop;  // vertex pairs from which a hyperedge centre goes to the 2-hop kernel (0: default)
};
thread_local const TuneChoice* t_tune = nullptr;
thread_local hipEvent_t t_tune_ev[2] = {nullptr, nullptr};  // recorded around an autotuned round's launches

int dev_alloc(DevBuf& b, size_t bytes) {
    if (t_na) {  // the no-allocation entry point allocates nothing
        if (debug_on()) std::fprintf(stderr, "hgt: allocation of %zu bytes refused (no-allocation call)\n", bytes);
        return HGT_ENOMEM;
    }
    if (bytes == 0) bytes = 256;
    void* p = nullptr;
    if (hip_failed(hipMalloc(&p, bytes), "hipMalloc", __LINE__)) return HGT_ENOMEM;
    b.p = p;
    b.bytes = bytes;
    return HGT_OK;
}

void dev_free(DevBuf& b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

// A region of the no-allocation arena for b: a buffer that already got one in
// this call keeps it while it is large enough (its contents then persist, as
// with ensure()); b's previous value is restored when the call ends.
int arena_take(NoAllocArena& a, DevBuf& b, size_t bytes) {
    int rec = -1;
    for (int i = 0; i < a.n_undo; i++)
        if (a.undo[i].b == &b) rec = i;
    if (rec >= 0 && b.bytes >= bytes) return HGT_OK;
    const uint64_t want = ((uint64_t)std::max<size_t>(bytes, 256) + 255) & ~255ull;
    if (a.used + want > a.cap) {
        if (debug_on())
            std::fprintf(stderr, "hgt: no-allocation scratch exhausted (%llu + %llu > %llu bytes)\n",
                         (unsigned long long)a.used, (unsigned long long)want, (unsigned long long)a.cap);
        return HGT_ENOMEM;
    }
    if (rec < 0) {
        if (a.n_undo == (int)(sizeof(a.undo) / sizeof(a.undo[0]))) return HGT_ENOMEM;
        a.undo[a.n_undo++] = {&b, b};
    }
    b.p = a.base + a.used;
    b.bytes = want;
    a.used += want;
    return HGT_OK;
}

// grow-only scratch (contents not preserved)
int ensure(DevBuf& b, size_t bytes) {
    if (t_na) return arena_take(*t_na, b, bytes);
    if (b.p && b.bytes >= bytes) return HGT_OK;
    if (t_capture) return HGT_ENOMEM;  // everything was reserved before the capture
    size_t nb = std::max(bytes, b.bytes + b.bytes / 2);
    nb = (nb + 4095) & ~(size_t)4095;
    dev_free(b);
    return dev_alloc(b, nb);
}

// grow preserving the first `keep` bytes
int grow_keep(DevBuf& b, size_t bytes, size_t keep, hipStream_t s) {
    if (b.p && b.bytes >= bytes) return HGT_OK;
    DevBuf nb;
    int rc = dev_alloc(nb, (bytes + 4095) & ~(size_t)4095);
    if (rc) return rc;
    if (keep && b.p) {
        if (hip_failed(hipMemcpyAsync(nb.p, b.p, std::min(keep, b.bytes), hipMemcpyDeviceToDevice, s),
                       "grow copy", __LINE__) ||
            hip_failed(hipStreamSynchronize(s), "grow sync", __LINE__)) {
            dev_free(nb);
            return HGT_EDEVICE;
        }
    }
    dev_free(b);
    b = nb;
    return HGT_OK;
}

int bits_for(uint64_t max_value) {  // bits to hold values 0..max_value
    int b = 1;
    while (b < 64 && (max_value >> b)) b++;
    return b;
}

constexpr int CNT_HE = 0, CNT_IV = 30, CNT_TMP = 33, CNT_N = 129;
// phase accumulators follow the counts
constexpr int ACC_HE_M = 129, ACC_HE_P = 159, ACC_TMP_M = 189, ACC_TMP_P = 285, ACC_IV_M = 381, ACC_IV_P = 383,
              ACC_T1 = 385, ACC_N = 387;

}  // namespace

// Scratch of the triad phases, one per device, shared by every graph on it:
// work of one call holds the lock while it queues its phases, and each call's
// stream first waits for the previous user's (ordered reuse across streams).
struct PhaseCtx {
    std::mutex mu;
    int device = 0;
    int refs = 0;                 // graphs that use it
    hipEvent_t done = nullptr;    // recorded after the last user's phases
    DevBuf iv_list, iv_list2, iv_garena, iv_garena2;  // incident-vertex stage scratch
    DevBuf t_ctr, t_big_list, t_big_rank, t_big_scratch, t_list1, t_rank1, t_list2, t_rank2, t_garena, t_whash;
    DevBuf t_slices, t_slice_scan;       // slices of the 2-hop kernel's centres
    DevBuf ent_x, ent_d, ent_pay, bl_cnt, bl_off, bl_cur, bl_d, bl_pay, nb_scratch, bl_scan;
    // per-graph phase descriptors: device copies and their pinned staging, one
    // slot per (phase, family) so no upload overwrites one still in flight
    DevBuf desc;
    char* desc_host = nullptr;
    uint64_t desc_cap = 0;       // graphs per slot
    hipEvent_t desc_ev[4] = {nullptr, nullptr, nullptr, nullptr};
    // HIP-graph launches of a round: descriptors uploaded before the capture, and
    // the executable graph of the last round (updated in place when the next
    // round's capture has the same shape)
    Multi pre[4] = {};
    bool pre_ok[4] = {false, false, false, false};
    hipGraphExec_t gexec = nullptr;
    // the null stream cannot be captured: rounds called on it are captured on this
    // stream, ordered after and before the caller's work by the two events
    hipStream_t cap_stream = nullptr;
    hipEvent_t cap_in = nullptr, cap_out = nullptr;
};

struct hgt_graph {
    int device = 0;
    int n_cu = 256;
    hipStream_t last_stream = nullptr;
    uint32_t track_mask = 0;
    int64_t window = 0;
    StoreDev st{};
    DevBuf h_off, h_len, h_cap, h_ts, h_seq, free_bm, mark_del, mark_ins;
    DevBuf h2v, v_off, v_len, v_cap, v2h;
    DevBuf v2h_ts;  // temporal graphs: int64 per v2h word (grown with v2h)
    DevBuf scal, counts, tabs;
    // batch scratch
    DevBuf s_sum, s_del_bm, s_del_card, s_del_poff, s_ins_rel, s_ins_card, s_canon, s_big, s_small, s_popc, s_scan,
        s_assigned, s_h_need, s_h_rel, s_keys, s_keys_alt, s_sort, s_head, s_is_ins, s_tv, s_tseg, s_D, s_I, s_It,
        s_vp, s_staging, s_staging_ts, s_dst;
    // hyperedge-family neighbour histograms (2 words per h2v word)
    DevBuf hpool;
    PhaseCtx* ph = nullptr;  // the device's shared phase scratch
    DevBuf iv_keys, iv_alt, iv_sort, iv_head, iv_uniq, iv_p2, iv_scan, iv_tab, iv_owner, iv_ctr;
    // horizontal operations
    DevBuf vo_sum, vo_keys, vo_alt, vo_sort, vo_scan, vo_head, vo_ins, vo_nmod, vo_mod, vo_seg, vo_card, vo_ts, vo_off,
        vo_mem;
    // host mirrors (valid after each synchronisation)
    uint64_t next_id = 0, h_bump = 0, v_bump = 0, next_seq = 0, n_live = 0, n_inc = 0;
    uint32_t epoch = 0;
    int sticky = HGT_OK;
    bool poisoned = false;          // a batch failed part-way: only hgt_restore / hgt_destroy apply
    uint64_t batches = 0;
    uint64_t compactions = 0;       // pool compactions since build
    uint64_t graph_launches = 0;    // rounds launched as captured HIP graphs (with this graph first)
    int force_stage = 0;            // HGT_FORCE_STAGE (tests): see He2Params
    int pair_agg = 1;               // HGT_PAIR_AGG=0: pairs enumerated per run (see He2Params)
    int global_wg_per_cu = 4;       // HGT_GLOBAL_WG_PER_CU: workgroups per CU of the global stage
    int iv_direct = 0;              // HGT_IV_DIRECT=1 (tests): incident-vertex owners without maps
    int iv_wg_per_cu = 8;           // HGT_IV_WG_PER_CU: workgroups per CU of the incident-vertex global stage
    uint32_t slice_lh = 0;          // HGT_SLICE_LH (tests): list entries per slice of a 2-hop kernel centre
    uint64_t e2_2hop = 0;           // HGT_E2_2HOP: vertex pairs from which a centre goes to the 2-hop kernel
    uint32_t w_2hop = 0;            // HGT_W_2HOP: neighbour-row entries from which it does
    int iv_force_stage = 0;         // HGT_IV_FORCE_STAGE (tests): incident-vertex stages below it pass owners on
    uint32_t wave_slots = 8192;     // HGT_WAVE_SLOTS (tests): slots of the 2-hop kernels' per-wave global hashes
    int skip_lds148 = 1;            // HGT_SKIP_LDS148=0: centres go through the 148 KB stage (one workgroup
                                    // per CU) instead of straight to the global one (four per CU)
    BatchSummary* h_sum = nullptr;  // pinned
    DevScalars* h_sc = nullptr;     // pinned
    // profiling: HIP events around each kernel group, algorithmic-byte counters
    bool prof = false;              // HIP events around kernel groups + algorithmic-byte counters
    bool prof_phases = false;       // also wall-clock ticks per phase of the hyperedge-delta stages
    struct Rec { int kind; hipEvent_t a, b; };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    DevBuf stats;
    uint64_t store_bytes = 0;
};

namespace {

enum ProfKind { PK_PLAN = 0, PK_DELTA_SMALL, PK_DELTA_BIG, PK_IV_PREP, PK_IV_PAIRS, PK_COMMIT, PK_DELTA_MED,
                PK_DELTA_GLOBAL, PK_NBR, PK_TMP, PK_N };
const char* kProfNames[PK_N] = {"store_plan", "he_hist_lds32", "he_2hop", "iv_prepare", "iv_pairs", "store_commit",
                                "he_hist_lds148", "he_hist_global", "he_nbr_pass", "temporal"};

hipEvent_t prof_event(hgt_graph* g) {
    if (g->ev_used == g->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        g->ev_pool.push_back(e);
    }
    return g->ev_pool[g->ev_used++];
}

struct ProfScope {
    hgt_graph* g;
    int kind;
    hipStream_t s;
    hipEvent_t a = nullptr;
    ProfScope(hgt_graph* g_, int k, hipStream_t s_) : g(g_), kind(k), s(s_) {
        if (g->prof && !t_na && !t_capture && (a = prof_event(g))) (void)hipEventRecord(a, s);
    }
    ~ProfScope() {
        if (!a) return;
        hipEvent_t b = prof_event(g);
        if (!b) return;
        (void)hipEventRecord(b, s);
        g->recs.push_back({kind, a, b});
    }
};

void refresh_view(hgt_graph* g) {
    StoreDev& s = g->st;
    s.h_off = g->h_off.as<uint64_t>();
    s.h_len = g->h_len.as<uint32_t>();
    s.h_cap = g->h_cap.as<uint32_t>();
    s.h_ts = (g->track_mask & (1u << HGT_TRIAD_TEMPORAL)) ? g->h_ts.as<int64_t>() : nullptr;
    s.h_seq = g->h_seq.as<uint64_t>();
    s.free_bm = g->free_bm.as<uint64_t>();
    s.h2v = g->h2v.as<uint32_t>();
    s.h2v_words = g->h2v.bytes / 4;
    s.v_off = g->v_off.as<uint64_t>();
    s.v_len = g->v_len.as<uint32_t>();
    s.v_cap = g->v_cap.as<uint32_t>();
    s.v2h = g->v2h.as<uint32_t>();
    s.v2h_ts = (g->track_mask & (1u << HGT_TRIAD_TEMPORAL)) ? g->v2h_ts.as<int64_t>() : nullptr;
    s.v2h_words = g->v2h.bytes / 4;
    s.mark_del = g->mark_del.as<uint64_t>();
    s.mark_ins = g->mark_ins.as<uint64_t>();
    s.sc = g->scal.as<DevScalars>();
}

GraphView view_of(hgt_graph* g) {
    GraphView v;
    v.h_off = g->st.h_off;
    v.h_len = g->st.h_len;
    v.h2v = g->st.h2v;
    v.v_off = g->st.v_off;
    v.v_len = g->st.v_len;
    v.v2h = g->st.v2h;
    v.h_ts = g->st.h_ts;
    v.h_seq = g->st.h_seq;
    v.v2h_ts = g->st.v2h_ts;
    return v;
}

// ID-indexed arrays hold id_cap entries; contents below the old capacity are kept.
int ensure_id_cap(hgt_graph* g, uint64_t need, hipStream_t s) {
    if (need <= g->st.id_cap) return HGT_OK;
    if (need > 0xfffffff0ull) return HGT_ENOMEM;
    uint64_t cap = std::max<uint64_t>(need, g->st.id_cap + g->st.id_cap / 2);
    cap = (cap + 63) & ~63ull;
    uint64_t old = g->st.id_cap;
    struct { DevBuf* b; size_t esz; } arrs[] = {{&g->h_off, 8}, {&g->h_len, 4}, {&g->h_cap, 4}, {&g->h_ts, 8},
                                                {&g->h_seq, 8}, {&g->mark_del, 8}, {&g->mark_ins, 8}};
    for (auto& a : arrs) {
        int rc = grow_keep(*a.b, cap * a.esz, old * a.esz, s);
        if (rc) return rc;
    }
    int rc = grow_keep(g->free_bm, cap / 8, (old + 7) / 8, s);
    if (rc) return rc;
    // new entries: zero (length 0, capacity 0, not free, no marks)
    HIP_OK(hipMemsetAsync(g->h_len.as<uint32_t>() + old, 0, (cap - old) * 4, s));
    HIP_OK(hipMemsetAsync(g->h_cap.as<uint32_t>() + old, 0, (cap - old) * 4, s));
    HIP_OK(hipMemsetAsync(g->mark_del.as<uint64_t>() + old, 0, (cap - old) * 8, s));
    HIP_OK(hipMemsetAsync(g->mark_ins.as<uint64_t>() + old, 0, (cap - old) * 8, s));
    HIP_OK(hipMemsetAsync((char*)g->free_bm.p + old / 8, 0, (cap - old) / 8, s));
    g->st.id_cap = cap;
    refresh_view(g);
    return HGT_OK;
}

int ensure_pool(DevBuf& pool, uint64_t used_words, uint64_t need_words, hipStream_t s) {
    uint64_t want = used_words + need_words;
    if (pool.p && pool.bytes / 4 >= want) return HGT_OK;
    uint64_t cap = std::max<uint64_t>(want + want / 4, pool.bytes / 4 * 2);
    return grow_keep(pool, cap * 4, used_words * 4, s);
}

struct Sizes {
    uint64_t n_del, n_ins, n_mem, pairs_cap, words;
};

int ensure_plan_scratch(hgt_graph* g, const Sizes& z, PlanScratch& w) {
    const uint64_t nd = std::max<uint64_t>(z.n_del, 1), ni = std::max<uint64_t>(z.n_ins, 1);
    const uint64_t nm = std::max<uint64_t>(z.n_mem, 1), pc = std::max<uint64_t>(z.pairs_cap, 1);
    const uint64_t words = std::max<uint64_t>(z.words, 1);
    int rc = 0;
    rc |= ensure(g->s_sum, sizeof(BatchSummary));
    rc |= ensure(g->s_del_bm, (g->st.id_cap / 64 + 1) * 8);
    rc |= ensure(g->s_del_card, nd * 8);
    rc |= ensure(g->s_del_poff, nd * 8);
    rc |= ensure(g->s_ins_rel, (ni + 1) * 8);
    rc |= ensure(g->s_ins_card, ni * 8);
    rc |= ensure(g->s_canon, nm * 4);
    rc |= ensure(g->s_big, ni * 4);
    rc |= ensure(g->s_small, 64 * 8);
    rc |= ensure(g->s_popc, words * 8);
    size_t scan_b = std::max({hgt_scan_tmp_bytes(words), hgt_scan_tmp_bytes(ni), hgt_scan_tmp_bytes(nd),
                              hgt_scan_tmp_bytes(pc)});
    rc |= ensure(g->s_scan, scan_b);
    rc |= ensure(g->s_assigned, ni * 4);
    rc |= ensure(g->s_h_need, ni * 8);
    rc |= ensure(g->s_h_rel, ni * 8);
    rc |= ensure(g->s_keys, pc * 8);
    rc |= ensure(g->s_keys_alt, pc * 8);
    rc |= ensure(g->s_sort, hgt_radix_tmp_bytes(pc));
    rc |= ensure(g->s_head, pc * 8);
    rc |= ensure(g->s_is_ins, pc * 8);
    rc |= ensure(g->s_tv, pc * 4);
    rc |= ensure(g->s_tseg, (pc + 1) * 8);
    rc |= ensure(g->s_D, pc * 4);
    rc |= ensure(g->s_I, pc * 4);
    rc |= ensure(g->s_It, pc * 4);
    rc |= ensure(g->s_vp, pc * (8 * 6 + 4 * 3) + 64);
    rc |= ensure(g->s_dst, pc * 8);
    if (rc) return HGT_ENOMEM;
    w.sum = g->s_sum.as<BatchSummary>();
    w.del_bm = g->s_del_bm.as<uint64_t>();
    w.del_card = g->s_del_card.as<uint64_t>();
    w.del_poff = g->s_del_poff.as<uint64_t>();
    w.ins_rel = g->s_ins_rel.as<uint64_t>();
    w.ins_card = g->s_ins_card.as<uint64_t>();
    w.canon = g->s_canon.as<uint32_t>();
    w.big_list = g->s_big.as<uint32_t>();
    uint64_t* sm = g->s_small.as<uint64_t>();
    w.big_count = (uint32_t*)(sm + 0);
    w.n_words = sm + 1;
    w.n_free = sm + 2;
    w.h2v_total = sm + 3;
    w.n_pairs = sm + 4;
    w.n_touched = sm + 5;
    w.n_ins_pairs = sm + 6;
    w.v2h_total = sm + 7;
    w.stage_total = sm + 8;
    w.popc = g->s_popc.as<uint64_t>();
    w.scan_tmp = g->s_scan.p;
    w.assigned = g->s_assigned.as<uint32_t>();
    w.h_need = g->s_h_need.as<uint64_t>();
    w.h_rel = g->s_h_rel.as<uint64_t>();
    w.pairs_cap = pc;
    w.keys = g->s_keys.as<uint64_t>();
    w.keys_alt = g->s_keys_alt.as<uint64_t>();
    w.sort_tmp = g->s_sort.p;
    w.head = g->s_head.as<uint64_t>();
    w.is_ins = g->s_is_ins.as<uint64_t>();
    w.tv = g->s_tv.as<uint32_t>();
    w.tseg = g->s_tseg.as<uint64_t>();
    w.D_all = g->s_D.as<uint32_t>();
    w.I_all = g->s_I.as<uint32_t>();
    w.I_t = g->s_It.as<uint32_t>();
    uint64_t* vp = g->s_vp.as<uint64_t>();
    w.vp.dstart = vp;
    w.vp.istart = vp + pc;
    w.vp.old_len = vp + 2 * pc;
    w.vp.need = vp + 3 * pc;
    w.vp.rel = vp + 4 * pc;
    w.vp.stage_off = vp + 5 * pc;
    uint32_t* vp32 = (uint32_t*)(vp + 6 * pc);
    w.vp.nD = vp32;
    w.vp.nI = vp32 + pc;
    w.vp.new_len = vp32 + 2 * pc;
    w.dst = g->s_dst.as<uint64_t>();
    w.staging = g->s_staging.as<uint32_t>();
    w.staging_ts = g->s_staging_ts.as<int64_t>();
    return HGT_OK;
}

// ---- triad phases ---------------------------------------------------------
void phase_ctx_free(PhaseCtx& c) {
    DevBuf* all[] = {&c.t_ctr, &c.t_whash, &c.t_big_list, &c.t_big_rank, &c.t_big_scratch, &c.t_list1, &c.t_rank1, &c.t_list2,
                     &c.t_slices, &c.t_slice_scan,
                     &c.t_rank2, &c.t_garena, &c.ent_x, &c.ent_d, &c.ent_pay, &c.bl_cnt, &c.bl_off, &c.bl_cur,
                     &c.bl_d, &c.bl_pay, &c.nb_scratch, &c.bl_scan, &c.desc, &c.iv_list, &c.iv_list2, &c.iv_garena,
                     &c.iv_garena2};
    for (DevBuf* b : all) dev_free(*b);
    for (hipEvent_t& e : c.desc_ev) {
        if (e) (void)hipEventSynchronize(e);
        if (e) (void)hipEventDestroy(e);
        e = nullptr;
    }
    if (c.desc_host) (void)hipHostFree(c.desc_host);
    c.desc_host = nullptr;
    c.desc_cap = 0;
    if (c.done) (void)hipEventDestroy(c.done);
    c.done = nullptr;
    if (c.gexec) (void)hipGraphExecDestroy(c.gexec);
    c.gexec = nullptr;
    if (c.cap_stream) (void)hipStreamDestroy(c.cap_stream);
    if (c.cap_in) (void)hipEventDestroy(c.cap_in);
    if (c.cap_out) (void)hipEventDestroy(c.cap_out);
    c.cap_stream = nullptr;
    c.cap_in = c.cap_out = nullptr;
}

std::mutex g_ctx_mu;
std::vector<PhaseCtx*> g_ctx;  // by device

// The phase scratch a call on this thread uses: the request server gives each
// of its in-flight rounds its own, so their triad phases can overlap on the
// device; every other call uses the device's shared one.
thread_local PhaseCtx* t_ph = nullptr;
PhaseCtx& ctx_of(hgt_graph* g) { return t_ph ? *t_ph : *g->ph; }

PhaseCtx* phase_ctx_acquire(int device) {
    std::lock_guard<std::mutex> lk(g_ctx_mu);
    if ((int)g_ctx.size() <= device) g_ctx.resize(device + 1, nullptr);
    PhaseCtx*& c = g_ctx[device];
    if (!c) {
        c = new (std::nothrow) PhaseCtx();
        if (!c) return nullptr;
        c->device = device;
        if (hipEventCreateWithFlags(&c->done, hipEventDisableTiming) != hipSuccess) {
            delete c;
            c = nullptr;
            return nullptr;
        }
    }
    c->refs++;
    return c;
}

// The last graph of a device frees the scratch.
void phase_ctx_release(PhaseCtx* c) {
    std::lock_guard<std::mutex> lk(g_ctx_mu);
    if (--c->refs > 0) return;
    (void)hipEventSynchronize(c->done);
    phase_ctx_free(*c);
    g_ctx[c->device] = nullptr;
    delete c;
}

// One graph's share of a phase.
struct PhaseJob {
    hgt_graph* g;
    const uint32_t* centres;  // device, n entries; the index is the batch rank
    uint64_t n;
    const uint64_t* mark;
    uint32_t epoch;
    uint64_t max_lh, sum_lh;  // over the centres (see BatchSummary)
    uint64_t n_ids;           // IDs in use during the phase
};

inline size_t desc_slot_bytes(uint64_t cap) { return cap * sizeof(HeGraph) + 2 * (cap + 1) * 8; }

// Uploads the descriptors of `G` into slot `slot` and fills M's device pointers.
int upload_multi(PhaseCtx& c, int slot, const std::vector<HeGraph>& G, const std::vector<uint64_t>& base,
                 const std::vector<uint64_t>& id_base, Multi& M, hipStream_t s) {
    const uint64_t n = G.size();
    if (t_capture) {  // uploaded before the capture
        if (!c.pre_ok[slot]) return HGT_EINVAL;
        M = c.pre[slot];
        return HGT_OK;
    }
    if (t_na) {
        // no-allocation call (one graph): the four slots live in the arena and are
        // staged from the thread's arena record; the stream orders the copies
        static_assert(sizeof(HeGraph) + 32 <= sizeof(t_na->stage[0]), "descriptor staging");
        if (n != 1) return HGT_EINVAL;
        if (int rc = ensure(c.desc, 4 * desc_slot_bytes(1))) return rc;
        char* h = t_na->stage[slot];
        char* d = (char*)c.desc.p + slot * desc_slot_bytes(1);
        const size_t bytes = sizeof(HeGraph) + 32;
        std::memcpy(h, G.data(), sizeof(HeGraph));
        std::memcpy(h + sizeof(HeGraph), base.data(), 16);
        std::memcpy(h + sizeof(HeGraph) + 16, id_base.data(), 16);
        HIP_OK(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s));
        M.graphs = (const HeGraph*)d;
        M.base = (const uint64_t*)(d + sizeof(HeGraph));
        M.id_base = (const uint64_t*)(d + sizeof(HeGraph) + 16);
        M.n_graphs = 1;
        M.total = base[1];
        M.total_ids = id_base[1];
        return HGT_OK;
    }
    if (n > c.desc_cap) {
        for (hipEvent_t e : c.desc_ev)
            if (e) HIP_OK(hipEventSynchronize(e));
        HIP_OK(hipStreamSynchronize(s));
        uint64_t cap = std::max<uint64_t>(n, 2 * c.desc_cap);
        cap = std::max<uint64_t>(cap, 4);
        if (c.desc_host) (void)hipHostFree(c.desc_host);
        c.desc_host = nullptr;
        c.desc_cap = 0;
        if (hipHostMalloc((void**)&c.desc_host, 4 * desc_slot_bytes(cap), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            c.desc_host = nullptr;
            return HGT_ENOMEM;
        }
        dev_free(c.desc);
        if (dev_alloc(c.desc, 4 * desc_slot_bytes(cap))) return HGT_ENOMEM;
        c.desc_cap = cap;
    }
    if (!c.desc_ev[slot] && hipEventCreateWithFlags(&c.desc_ev[slot], hipEventDisableTiming) != hipSuccess) {
        c.desc_ev[slot] = nullptr;
        return HGT_EDEVICE;
    }
    HIP_OK(hipEventSynchronize(c.desc_ev[slot]));  // the slot's previous upload has been read
    const size_t sb = desc_slot_bytes(c.desc_cap);
    char* h = c.desc_host + slot * sb;
    char* d = (char*)c.desc.p + slot * sb;
    std::memcpy(h, G.data(), n * sizeof(HeGraph));
    std::memcpy(h + n * sizeof(HeGraph), base.data(), (n + 1) * 8);
    std::memcpy(h + n * sizeof(HeGraph) + (n + 1) * 8, id_base.data(), (n + 1) * 8);
    const size_t bytes = n * sizeof(HeGraph) + 2 * (n + 1) * 8;
    HIP_OK(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, s));
    HIP_OK(hipEventRecord(c.desc_ev[slot], s));
    M.graphs = (const HeGraph*)d;
    M.base = (const uint64_t*)(d + n * sizeof(HeGraph));
    M.id_base = (const uint64_t*)(d + n * sizeof(HeGraph) + (n + 1) * 8);
    M.n_graphs = (uint32_t)n;
    M.total = base[n];
    M.total_ids = id_base[n];
    return HGT_OK;
}

// Builds the descriptors of the jobs whose graph tracks `family`.
void collect(const PhaseJob* jobs, uint32_t nj, int family, bool minus, std::vector<HeGraph>& G,
             std::vector<uint64_t>& base, std::vector<uint64_t>& id_base, uint64_t& max_lh, uint64_t& sum_lh) {
    G.clear();
    base.assign(1, 0);
    id_base.assign(1, 0);
    max_lh = sum_lh = 0;
    for (uint32_t j = 0; j < nj; j++) {
        const PhaseJob& J = jobs[j];
        hgt_graph* g = J.g;
        if (J.n == 0 || !(g->track_mask & (1u << family))) continue;
        HeGraph h{};
        h.g = view_of(g);
        h.centres = J.centres;
        h.n_centres = J.n;
        h.mark = J.mark;
        h.epoch = J.epoch;
        h.window = g->window;
        h.status = &g->st.sc->status;
        uint64_t* cnt = g->counts.as<uint64_t>();
        h.out_he = cnt + (minus ? ACC_HE_M : ACC_HE_P);
        h.out_tmp = cnt + (minus ? ACC_TMP_M : ACC_TMP_P);
        h.hpool = g->hpool.as<uint32_t>();
        h.id_base = id_base.back();
        G.push_back(h);
        base.push_back(base.back() + J.n);
        id_base.push_back(id_base.back() + std::max<uint64_t>(J.n_ids, 1));
        max_lh = std::max(max_lh, J.max_lh);
        sum_lh += J.sum_lh;
    }
}

// Launch shapes and scratch sizes of one family's phase, from its centre count
// and neighbourhood sizes.  `lean` (the no-allocation entry point) keeps the
// grids of the kernels with per-workgroup global tables small.
struct PhaseShape {
    uint64_t n, lhm, max_card, ecap, total_ids;
    BigLayout L;
    uint64_t grid_big, grid_small, grid_tmp, grid_2hop, grid_s0, grid_s1, grid_g, nb_grid, nb_words;
    uint32_t wave_slots;
};

constexpr uint64_t kGarenaWords = 1ull << 18;  // 1 MB global arena per workgroup of the global stage

PhaseShape phase_shape(const hgt_graph* owner, uint64_t n, uint64_t max_lh, uint64_t sum_lh, uint64_t total_ids,
                       bool lean) {
    const uint64_t n_cu = (uint64_t)owner->n_cu;
    PhaseShape z{};
    z.n = n;
    z.lhm = std::max<uint64_t>(max_lh, 1);
    z.max_card = std::min<uint64_t>(HGT_MAX_CARD, z.lhm);
    z.L = triad_big_layout(z.lhm, z.max_card);
    // at most ~1 GiB of global tables for the large-centre kernels
    z.grid_big = std::max<uint64_t>(1, std::min<uint64_t>(lean ? 8 : n_cu * 2, (1ull << 28) / z.L.words_per_wg));
    z.grid_small = std::min<uint64_t>(n_cu * 2, n);
    z.grid_tmp = std::min<uint64_t>(lean ? 32 : n_cu * 3, n);
    // 2-hop hashes in global memory, one per wave of the 2-hop kernels (64 KB each)
    z.wave_slots = t_tune ? t_tune->wave_slots : owner->wave_slots;
    z.grid_2hop = std::max<uint64_t>(z.grid_big, z.grid_tmp);
    z.ecap = std::max<uint64_t>(sum_lh, 1);
    z.nb_words = 2 * pow2ceil64(2 * std::max<uint64_t>(z.lhm, 32)) + 3 * z.max_card + 8;
    z.nb_grid = std::max<uint64_t>(1, std::min<uint64_t>(lean ? 8 : 256, (1ull << 27) / z.nb_words));
    z.grid_s0 = std::min<uint64_t>(n_cu * 4, n);
    z.grid_s1 = std::min<uint64_t>(n_cu, n);
    // the global stage holds little LDS, so several workgroups share a CU and hide
    // each other's memory latency
    const int wg_per_cu = t_tune ? t_tune->wg_per_cu : owner->global_wg_per_cu;
    z.grid_g = std::min<uint64_t>(lean ? 16 : n_cu * (uint64_t)wg_per_cu, n);
    z.total_ids = total_ids;
    return z;
}

// Every scratch buffer of one family's phase at the shape's sizes.
int phase_reserve(PhaseCtx& c, int family, const PhaseShape& z) {
    const uint64_t n = z.n;
    int rc = 0;
    rc |= ensure(c.t_ctr, 128);
    rc |= ensure(c.t_big_list, n * 8);
    rc |= ensure(c.t_big_rank, n * 4);
    rc |= ensure(c.t_list1, n * 8);
    rc |= ensure(c.t_rank1, n * 4);
    rc |= ensure(c.t_list2, n * 8);
    rc |= ensure(c.t_rank2, n * 4);
    rc |= ensure(c.t_big_scratch, z.grid_big * z.L.words_per_wg * 4);
    rc |= ensure(c.t_whash, z.grid_2hop * 4 * 2ull * z.wave_slots * 4);
    rc |= ensure(c.t_slices, (n + 2) * 8);
    rc |= ensure(c.t_slice_scan, hgt_scan_tmp_bytes(n));
    if (family == HGT_TRIAD_HYPEREDGE) {
        const uint64_t ids = z.total_ids;
        rc |= ensure(c.ent_x, z.ecap * 4);
        rc |= ensure(c.ent_d, z.ecap * 4);
        rc |= ensure(c.ent_pay, z.ecap * 8);
        rc |= ensure(c.bl_d, z.ecap * 4);
        rc |= ensure(c.bl_pay, z.ecap * 8);
        rc |= ensure(c.bl_cnt, ids * 8);
        rc |= ensure(c.bl_off, ids * 8);
        rc |= ensure(c.bl_cur, ids * 8);
        rc |= ensure(c.bl_scan, hgt_scan_tmp_bytes(ids));
        rc |= ensure(c.nb_scratch, z.nb_grid * z.nb_words * 4);
        rc |= ensure(c.t_garena, z.grid_g * kGarenaWords * 4);
    }
    return rc ? HGT_ENOMEM : HGT_OK;
}

// One phase (deltas of the deleted hyperedges on the old graphs, or of the
// inserted ones on the new graphs) for every job, in one launch per kernel.
// Counter slots in t_ctr: 0-2 neighbour pass, 5 2-hop queue for the centres the
// histogram stages pass on, 6-8 temporal, 10-11 entry count, 16-18 stage queues,
// 19-21 stage hand-over counts.
int run_phase(hgt_graph* owner, const PhaseJob* jobs, uint32_t nj, bool minus, bool full, hipStream_t s) {
    PhaseCtx& c = ctx_of(owner);
    uint64_t* stats = owner->prof ? owner->stats.as<uint64_t>() : nullptr;
    std::vector<HeGraph> G;
    std::vector<uint64_t> base, id_base;
    for (int family : {HGT_TRIAD_HYPEREDGE, HGT_TRIAD_TEMPORAL}) {
        uint64_t max_lh, sum_lh;
        collect(jobs, nj, family, minus, G, base, id_base, max_lh, sum_lh);
        const uint64_t n = base.back();
        if (n == 0) continue;
        if (id_base.back() > 0xfffffff0ull) return HGT_EINVAL;  // entry slots are u32
        const PhaseShape z = phase_shape(owner, n, max_lh, sum_lh, id_base.back(), t_na != nullptr);
        int rc = phase_reserve(c, family, z);
        if (rc) return rc;
        const BigLayout& L = z.L;
        const uint64_t grid_big = z.grid_big;
        Multi M{};
        rc = upload_multi(c, (minus ? 0 : 2) + (family == HGT_TRIAD_TEMPORAL ? 1 : 0), G, base, id_base, M, s);
        if (rc) return rc;
        uint32_t* ctr = c.t_ctr.as<uint32_t>();
        TriadParams P{};
        P.M = M;
        P.he_tab = owner->tabs.as<uint8_t>();
        P.tmp_tab = owner->tabs.as<uint8_t>() + 128;
        P.big_list = c.t_big_list.as<uint64_t>();
        P.big_rank = c.t_big_rank.as<uint32_t>();
        P.big_scratch = c.t_big_scratch.as<uint32_t>();
        P.wave_hash = c.t_whash.as<uint32_t>();
        P.wave_slots = z.wave_slots;
        P.slice_pre = c.t_slices.as<uint64_t>();
        P.slice_cap = n;
        P.slice_scan_tmp = c.t_slice_scan.p;
        P.slice_lh = owner->slice_lh;
        P.big = L;
        P.stats = stats;
        const unsigned grid_small = (unsigned)z.grid_small;
        if (family == HGT_TRIAD_HYPEREDGE) {
            // neighbour pass: batch-neighbour entries; histogram updates for inserts
            const uint64_t ecap = z.ecap, nb_words = z.nb_words, nb_grid = z.nb_grid;
            NbrParams N{};
            N.M = M;
            N.inserting = minus ? 0 : 1;
            N.emit_entries = full ? 0 : 1;
            N.n_entries = (uint64_t*)(ctr + 10);  // 8-byte aligned slot
            N.entries_cap = ecap;
            N.ent_x = c.ent_x.as<uint32_t>();
            N.ent_d = c.ent_d.as<uint32_t>();
            N.ent_pay = c.ent_pay.as<uint64_t>();
            N.queue = ctr;
            N.big_queue = ctr + 1;
            N.big_count = ctr + 2;
            N.big_list = P.big_list;
            N.big_rank = P.big_rank;
            N.big_scratch = c.nb_scratch.as<uint32_t>();
            N.big_words = nb_words;
            {
                ProfScope ps_nbr(owner, PK_NBR, s);
                he2_nbr_launch(N, grid_small, (unsigned)nb_grid, s);
                if (!full)
                    he2_lists_build(N, c.bl_cnt.as<uint64_t>(), c.bl_off.as<uint64_t>(), c.bl_cur.as<uint64_t>(),
                                    c.bl_d.as<uint32_t>(), c.bl_pay.as<uint64_t>(), c.bl_scan.p, s);
            }
            He2Params E{};
            E.M = M;
            E.he_tab = P.he_tab;
            E.bl_off = c.bl_off.as<uint64_t>();
            E.bl_cnt = c.bl_cnt.as<uint64_t>();
            E.bl_d = c.bl_d.as<uint32_t>();
            E.bl_pay = c.bl_pay.as<uint64_t>();
            E.queue = ctr + 16;
            E.count = ctr + 19;
            E.list[0] = c.t_list1.as<uint64_t>();
            E.rank[0] = c.t_rank1.as<uint32_t>();
            E.list[1] = c.t_list2.as<uint64_t>();
            E.rank[1] = c.t_rank2.as<uint32_t>();
            E.list[2] = P.big_list;
            E.rank[2] = P.big_rank;
            const unsigned grid_g = (unsigned)z.grid_g;
            E.garena = c.t_garena.as<uint32_t>();
            E.garena_words = kGarenaWords;
            E.stats = stats;
            E.phase_ticks = (stats && owner->prof_phases) ? 1 : 0;
            // read again at every phase, so that a test can force the stages of a batch
            // without forcing those of the build's full count
            const char* fs = std::getenv("HGT_FORCE_STAGE");
            E.force_stage = fs ? std::atoi(fs) : owner->force_stage;
            E.pair_agg = owner->pair_agg;
            E.skip_lds148 = t_tune ? t_tune->skip_lds148 : owner->skip_lds148;
            E.e2_2hop = t_tune && t_tune->e2_2hop ? t_tune->e2_2hop : owner->e2_2hop;
            E.w_2hop = owner->w_2hop;
            E.static_mode = full ? 1 : 0;
            hgt_fill_u32(ctr + 16, 0, 6, s);
            hgt_fill_u32(ctr + 5, 0, 1, s);
            {
                ProfScope ps(owner, PK_DELTA_SMALL, s);
                he2_launch_stage(E, 0, (unsigned)z.grid_s0, s);
            }
            {
                ProfScope ps(owner, PK_DELTA_MED, s);
                he2_launch_stage(E, 1, (unsigned)z.grid_s1, s);
            }
            {
                ProfScope ps(owner, PK_DELTA_GLOBAL, s);
                he2_launch_stage(E, 2, grid_g, s);
            }
            // centres too large for every arena: the 2-hop kernel
            TriadParams B = P;
            B.do_he = 1;
            B.do_tmp = 0;
            B.big_count = ctr + 21;
            B.big_queue = ctr + 5;
            B.static_he = full ? 1 : 0;
            {
                ProfScope ps(owner, PK_DELTA_BIG, s);
                triad_he_slices(B, s);
                triad_he_launch_big(B, (unsigned)grid_big, s);
            }
            if (minus) he2_remove_deleted(N, s);
        } else {
            TriadParams Q = P;
            Q.do_he = 0;
            Q.do_tmp = 1;
            Q.queue = ctr + 6;
            Q.big_queue = ctr + 7;
            Q.big_count = ctr + 8;
            Q.stats = stats ? stats + ST_TMP0 : nullptr;
            triad_he_prepare(Q, s);
            ProfScope ps(owner, PK_TMP, s);
            triad_he_launch_small(Q, (unsigned)z.grid_tmp, s);
            triad_he_slices(Q, s);
            triad_he_launch_big(Q, (unsigned)grid_big, s);
        }
    }
    return HGT_OK;
}

// IV pair list: unique vertex pairs inside the changed hyperedges.
__global__ void k_iv_gen(const uint32_t* __restrict__ ids, uint64_t n, const uint64_t* __restrict__ h_off,
                         const uint32_t* __restrict__ h_len, const uint32_t* __restrict__ h2v,
                         const uint32_t* __restrict__ canon, const uint64_t* __restrict__ rel,
                         const uint64_t* __restrict__ p2off, uint64_t base, int vb, uint64_t* keys, uint64_t* t1,
                         const DevScalars* sc) {
    if (sc->status) return;
    const int lane = threadIdx.x & 63;
    uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (i >= n) return;
    const uint32_t* m;
    uint64_t d;
    if (ids) {
        m = h2v + h_off[ids[i]];
        d = h_len[ids[i]];
    } else {
        m = canon + rel[i];
        d = rel[i + 1] - rel[i];
    }
    uint64_t o = base + p2off[i];
    for (uint64_t a = lane; a < d; a += 64) {
        uint64_t start = o + a * (2 * d - a - 1) / 2;
        uint64_t ua = m[a];
        for (uint64_t b = a + 1; b < d; b++) keys[start + (b - a - 1)] = (ua << vb) | m[b];
    }
    if (lane == 0) atomicAdd((unsigned long long*)t1, (unsigned long long)choose3(d));
}

__global__ void k_c2(const uint64_t* __restrict__ card, uint64_t n, uint64_t* out) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = choose2(card[i]);
}

__global__ void k_uniq_heads(const uint64_t* __restrict__ keys, uint64_t n, uint64_t* head) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) head[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

__global__ void k_uniq_write(const uint64_t* __restrict__ keys, uint64_t n, const uint64_t* __restrict__ pos, int vb,
                             uint64_t* out) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (i == 0 || keys[i] != keys[i - 1]) {
        uint64_t k = keys[i];
        out[pos[i]] = ((k >> vb) << 32) | (k & ((1ull << vb) - 1));
    }
}

// Owner of a touched pair: the endpoint of higher degree (ties: the smaller ID).
// The owner's weighted clique map is built once and the other endpoint's
// hyperedges are scanned per pair, so hubs are scanned as rarely as possible.
__global__ void k_iv_orient(const uint64_t* __restrict__ canon, const uint64_t* n_p, const uint32_t* __restrict__ v_len,
                            uint64_t* out) {
    const uint64_t n = *n_p;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t k = canon[i];
        const uint32_t lo = (uint32_t)(k >> 32), hi = (uint32_t)k;
        out[i] = v_len[hi] > v_len[lo] ? ((uint64_t)hi << 32 | lo) : k;
    }
}

__global__ void k_iv_update(uint64_t* cnt, int iv, int m, int p, int t1) {
    if (threadIdx.x || blockIdx.x) return;
    uint64_t d1 = cnt[t1 + 1] - cnt[t1];           // change of type 1
    uint64_t ds = cnt[p] - cnt[m];                 // change of sum m_p w_p
    uint64_t dx = cnt[p + 1] - cnt[m + 1];         // change of the triangle sum
    uint64_t d2 = ds - 3 * d1;
    cnt[iv] += d1;
    cnt[iv + 1] += d2;
    cnt[iv + 2] += dx - d1 - d2;
}

inline unsigned nblk(uint64_t n, unsigned per = 256) {
    uint64_t b = (n + per - 1) / per;
    return (unsigned)(b ? b : 1);
}

struct IvPlan {
    uint64_t n_keys = 0;
    uint64_t* uniq = nullptr;     // touched pairs (lo << 32 | hi), sorted
    uint64_t* own = nullptr;      // the same as (owner << 32 | other), sorted
    uint64_t* n_uniq = nullptr;
    uint64_t tab_slots = 0;
};

int iv_prepare(hgt_graph* g, const BatchIn& b, const PlanScratch& w, const BatchSummary& sum, IvPlan& ip,
               hipStream_t s) {
    uint64_t nk = sum.del_pairs2 + sum.ins_pairs2;
    ip.n_keys = nk;
    uint64_t nmax = std::max<uint64_t>(nk, 1);
    uint64_t nh = std::max<uint64_t>(std::max(b.n_del, b.n_ins), 1);
    int rc = 0;
    rc |= ensure(g->iv_keys, nmax * 8);
    rc |= ensure(g->iv_alt, nmax * 8);
    rc |= ensure(g->iv_sort, hgt_radix_tmp_bytes(nmax));
    rc |= ensure(g->iv_head, nmax * 8);
    rc |= ensure(g->iv_uniq, nmax * 8 + 64);
    rc |= ensure(g->iv_p2, (nh + 1) * 8);
    rc |= ensure(g->iv_scan, std::max(hgt_scan_tmp_bytes(nmax), hgt_scan_tmp_bytes(nh)));
    if (rc) return HGT_ENOMEM;
    uint64_t* cnt = g->counts.as<uint64_t>();
    uint64_t* keys = g->iv_keys.as<uint64_t>();
    uint64_t* p2 = g->iv_p2.as<uint64_t>();
    int vb = g->st.vb;
    if (b.n_del) {
        k_c2<<<nblk(b.n_del), 256, 0, s>>>(w.del_card, b.n_del, p2);
        hgt_scan_u64(p2, p2, b.n_del, nullptr, nullptr, g->iv_scan.p, s);
        k_iv_gen<<<nblk(b.n_del * 64), 256, 0, s>>>(b.del, b.n_del, g->st.h_off, g->st.h_len, g->st.h2v, nullptr,
                                                    nullptr, p2, 0, vb, keys, cnt + ACC_T1, g->st.sc);
    }
    if (b.n_ins) {
        k_c2<<<nblk(b.n_ins), 256, 0, s>>>(w.ins_card, b.n_ins, p2);
        hgt_scan_u64(p2, p2, b.n_ins, nullptr, nullptr, g->iv_scan.p, s);
        k_iv_gen<<<nblk(b.n_ins * 64), 256, 0, s>>>(nullptr, b.n_ins, nullptr, nullptr, nullptr, w.canon, w.ins_rel,
                                                    p2, sum.del_pairs2, vb, keys, cnt + ACC_T1 + 1, g->st.sc);
    }
    ip.uniq = g->iv_uniq.as<uint64_t>() + 1;
    ip.n_uniq = g->iv_uniq.as<uint64_t>();
    if (nk == 0) {
        hgt_fill_u64(ip.n_uniq, 0, 1, s);
        return HGT_OK;
    }
    hgt_radix_sort_u64(keys, g->iv_alt.as<uint64_t>(), nk, nullptr, 2 * vb, g->iv_sort.p, s);
    uint64_t* head = g->iv_head.as<uint64_t>();
    k_uniq_heads<<<nblk(nk), 256, 0, s>>>(keys, nk, head);
    hgt_scan_u64(head, head, nk, nullptr, ip.n_uniq, g->iv_scan.p, s);
    k_uniq_write<<<nblk(nk), 256, 0, s>>>(keys, nk, head, vb, ip.uniq);
    // pairs by owner (the buffer of the unsorted keys is free now)
    ip.own = keys;
    k_iv_orient<<<nblk(nk > 262144 ? 262144 : nk), 256, 0, s>>>(ip.uniq, ip.n_uniq, g->st.v_len, ip.own);
    hgt_radix_sort_u64(ip.own, g->iv_alt.as<uint64_t>(), nk, ip.n_uniq, 32 + vb, g->iv_sort.p, s);
    // hash of the touched pairs and the owner segments
    ip.tab_slots = pow2ceil64(2 * nk + 64);
    if (ensure(g->iv_tab, ip.tab_slots * 8) || ensure(g->iv_owner, (nk + 2) * 8) || ensure(g->iv_ctr, 64))
        return HGT_ENOMEM;
    uint64_t* ictr = g->iv_ctr.as<uint64_t>();
    iv_touched_build(ip.uniq, ip.own, ip.n_uniq, g->iv_tab.as<uint64_t>(), ip.tab_slots, head,
                     g->iv_owner.as<uint64_t>(), ictr, nk, g->iv_scan.p, s);
    return HGT_OK;
}

// Incident-vertex global stages: 1 MB per workgroup (maps of up to 65536 slots:
// owners whose hyperedges hold up to about 43k members in all), four
// workgroups per CU; then 16 MB per workgroup (owners up to about 700k
// members), 32 workgroups.  The no-allocation entry point runs 16 and 2.
constexpr uint64_t kIvGarenaWords = 1ull << 18;
constexpr uint64_t kIvGarena2Words = 1ull << 22;
inline unsigned iv_grid_global(const hgt_graph* g) { return t_na ? 16u : (unsigned)(g->n_cu * g->iv_wg_per_cu); }
inline unsigned iv_grid_global2() { return t_na ? 2u : 32u; }

int iv_reserve(hgt_graph* g, const IvPlan& ip) {
    PhaseCtx& c = ctx_of(g);
    if (ensure(c.iv_list, (ip.n_keys + 1) * 4) || ensure(c.iv_list2, (ip.n_keys + 1) * 4) ||
        ensure(c.iv_garena, (uint64_t)iv_grid_global(g) * kIvGarenaWords * 4) ||
        ensure(c.iv_garena2, (uint64_t)iv_grid_global2() * kIvGarena2Words * 4))
        return HGT_ENOMEM;
    return HGT_OK;
}

int iv_phase(hgt_graph* g, const IvPlan& ip, bool minus, hipStream_t s) {
    if (ip.n_keys == 0) return HGT_OK;
    const uint64_t gwords = kIvGarenaWords;
    const unsigned grid_g = iv_grid_global(g);
    PhaseCtx& c = ctx_of(g);
    if (int rc = iv_reserve(g, ip)) return rc;
    IvParams P{};
    P.g = view_of(g);
    P.pairs = ip.own;
    P.n_pairs = ip.n_uniq;
    uint64_t* ictr = g->iv_ctr.as<uint64_t>();
    P.n_owners = ictr;
    P.owner_start = g->iv_owner.as<uint64_t>();
    P.tab = g->iv_tab.as<uint64_t>();
    P.tab_mask = ip.tab_slots - 1;
    P.out = g->counts.as<uint64_t>() + (minus ? ACC_IV_M : ACC_IV_P);
    P.status = &g->st.sc->status;
    P.queue = (uint32_t*)(ictr + 2);
    P.count = P.queue + 3;
    P.list = c.iv_list.as<uint32_t>();
    P.list2 = c.iv_list2.as<uint32_t>();
    P.garena = c.iv_garena.as<uint32_t>();
    P.garena_words = gwords;
    P.garena2 = c.iv_garena2.as<uint32_t>();
    P.garena2_words = kIvGarena2Words;
    P.stats = g->prof ? g->stats.as<uint64_t>() : nullptr;
    P.force_direct = g->iv_direct;
    P.force_stage = g->iv_force_stage;
    ProfScope ps(g, PK_IV_PAIRS, s);
    triad_iv_launch(P, (unsigned)std::min<uint64_t>((uint64_t)g->n_cu * 4, ip.n_keys), grid_g, iv_grid_global2(), s);
    return HGT_OK;
}

__global__ void k_he_tmp_update(uint64_t* cnt) {
    int i = threadIdx.x;
    if (i < 30) cnt[CNT_HE + i] += cnt[ACC_HE_P + i] - cnt[ACC_HE_M + i];
    if (i < 96) cnt[CNT_TMP + i] += cnt[ACC_TMP_P + i] - cnt[ACC_TMP_M + i];
}

// A batch in flight: the steps before and after the one host synchronisation.
struct Pending {
    hgt_graph* g = nullptr;
    BatchIn b{};
    PlanScratch w{};
    BatchSummary sum{};
    IvPlan ip;
    uint64_t n_mem = 0;
    uint32_t* out_ids = nullptr;
    int check_order = 1;
    int is_build = 0;                       // the build: counts by the static mode of the kernels
    const uint32_t* forced_ids = nullptr;   // horizontal operations: the IDs the inserts take
    int keep_seq = 0;                       // horizontal operations: arrival sequences kept
    int rc = HGT_OK;  // this batch's result so far
};

// Moves every live list into fresh pools: the blocks of free IDs and the
// blocks that relocated lists left behind are dropped (the pools otherwise
// only grow).  Queued on s after the graph's earlier work; waits for s.
int compact_pools(hgt_graph* g, hipStream_t s) {
    if (g->last_stream != s) HIP_OK(hipStreamSynchronize(g->last_stream));
    const uint64_t n_ids = g->next_id, V = g->st.n_vertices;
    const uint64_t nmax = std::max<uint64_t>(n_ids, V) + 1;
    DevBuf need_h, need_v, off_h, off_v, tmp, tot;
    DevBuf h2v_new, hpool_new, v2h_new, ts_new;
    auto cleanup = [&] {
        for (DevBuf* b : {&need_h, &need_v, &off_h, &off_v, &tmp, &tot, &h2v_new, &hpool_new, &v2h_new, &ts_new})
            dev_free(*b);
    };
    int rc = 0;
    rc |= dev_alloc(need_h, nmax * 8);
    rc |= dev_alloc(need_v, nmax * 8);
    rc |= dev_alloc(off_h, nmax * 8);
    rc |= dev_alloc(off_v, nmax * 8);
    rc |= dev_alloc(tmp, hgt_scan_tmp_bytes(nmax));
    rc |= dev_alloc(tot, 64);
    if (rc) { cleanup(); return HGT_ENOMEM; }
    uint64_t* t = tot.as<uint64_t>();
    hgt_fill_u64(t, 0, 2, s);
    store_compact_need(g->st, n_ids, need_h.as<uint64_t>(), need_v.as<uint64_t>(), s);
    if (n_ids) hgt_scan_u64(need_h.as<uint64_t>(), off_h.as<uint64_t>(), n_ids, nullptr, t, tmp.p, s);
    hgt_scan_u64(need_v.as<uint64_t>(), off_v.as<uint64_t>(), V, nullptr, t + 1, tmp.p, s);
    uint64_t totals[2] = {0, 0};
    if (hip_failed(hipMemcpyAsync(totals, t, 16, hipMemcpyDeviceToHost, s), "compact totals", __LINE__) ||
        hip_failed(hipStreamSynchronize(s), "compact sync", __LINE__)) {
        cleanup();
        return HGT_EDEVICE;
    }
    const uint64_t hw = totals[0] + totals[0] / 4 + 1024, vw = totals[1] + totals[1] / 4 + 1024;
    const bool he = g->track_mask & (1u << HGT_TRIAD_HYPEREDGE), tm = g->track_mask & (1u << HGT_TRIAD_TEMPORAL);
    rc |= dev_alloc(h2v_new, hw * 4);
    rc |= dev_alloc(v2h_new, vw * 4);
    if (he) rc |= dev_alloc(hpool_new, hw * 8);
    if (tm) rc |= dev_alloc(ts_new, vw * 8);
    if (rc) { cleanup(); return HGT_ENOMEM; }
    store_compact_h2v(g->st, n_ids, need_h.as<uint64_t>(), off_h.as<uint64_t>(), h2v_new.as<uint32_t>(),
                      he ? g->hpool.as<uint32_t>() : nullptr, he ? hpool_new.as<uint32_t>() : nullptr, s);
    store_compact_v2h(g->st, need_v.as<uint64_t>(), off_v.as<uint64_t>(), v2h_new.as<uint32_t>(),
                      tm ? ts_new.as<int64_t>() : nullptr, s);
    store_compact_scalars(g->st.sc, t, t + 1, s);
    if (hip_failed(hipStreamSynchronize(s), "compact copy", __LINE__)) { cleanup(); return HGT_EDEVICE; }
    std::swap(g->h2v, h2v_new);
    std::swap(g->v2h, v2h_new);
    if (he) std::swap(g->hpool, hpool_new);
    if (tm) std::swap(g->v2h_ts, ts_new);
    cleanup();  // frees the old pools (now in the *_new buffers) and the scratch
    g->h_bump = totals[0];
    g->v_bump = totals[1];
    g->compactions++;
    refresh_view(g);
    return HGT_OK;
}

// The pools hold more than twice what their live lists need (power-of-two
// blocks of at least 4 words), plus 1M words of slack.
bool pools_bloated(const hgt_graph* g) {
    const uint64_t h_est = 2 * g->n_inc + 4 * g->n_live;
    const uint64_t v_est = 2 * g->n_inc + 4 * std::min<uint64_t>(g->st.n_vertices, g->n_inc);
    return g->h_bump > 2 * h_est + (1ull << 20) || g->v_bump > 2 * v_est + (1ull << 20);
}

// Host checks, scratch, and the non-mutating planning pass; the summary is
// copied to pinned memory, read after the caller synchronises.
int plan_begin(Pending& p, const uint32_t* del, uint64_t n_del, const uint64_t* ins_off, const uint32_t* ins_mem,
               uint64_t n_mem, const int64_t* ins_ts, uint64_t n_ins, hipStream_t s) {
    hgt_graph* g = p.g;
    const bool tmp = g->track_mask & (1u << HGT_TRIAD_TEMPORAL);
    if ((n_del && !del) || (n_ins && !ins_off) || (n_mem && !ins_mem)) return HGT_EINVAL;
    if (tmp && n_ins && !ins_ts) return HGT_EINVAL;
    if (n_ins > 0xfffffff0ull || n_del > 0xfffffff0ull) return HGT_EINVAL;
    if (n_mem > n_ins * (uint64_t)HGT_MAX_CARD) return HGT_EINVAL;
    if (n_del > g->n_live) return HGT_ENOENT;
    int rc;
    if (!t_na && pools_bloated(g) && (rc = compact_pools(g, s))) return rc;
    g->last_stream = s;
    rc = ensure_id_cap(g, g->next_id + n_ins + 1, s);
    if (rc) return rc;
    g->st.next_id_host = g->next_id;
    g->st.hb = bits_for(g->next_id + n_ins);
    g->st.vb = bits_for(g->st.n_vertices ? g->st.n_vertices - 1 : 0);
    if (g->st.hb + 1 + g->st.vb > 64) return HGT_EINVAL;
    Sizes z{n_del, n_ins, n_mem, g->n_inc + n_mem, (g->next_id + 63) / 64 + 1};
    rc = ensure_plan_scratch(g, z, p.w);
    if (rc) return rc;
    p.b = BatchIn{del, n_del, ins_off, ins_mem, n_mem, ins_ts, n_ins, g->epoch + 1, g->epoch + 2, p.check_order,
                  p.forced_ids, p.keep_seq};
    p.n_mem = n_mem;
    g->epoch += 2;
    uint64_t* cnt = g->counts.as<uint64_t>();
    store_batch_begin(g->st.sc, p.w.sum, s);
    hgt_fill_u64(cnt + CNT_N, 0, ACC_N - CNT_N, s);
    {
        ProfScope ps(g, PK_PLAN, s);
        store_plan(g->st, p.b, p.w, s);
    }
    HIP_OK(hipMemcpyAsync(g->h_sum, p.w.sum, sizeof(BatchSummary), hipMemcpyDeviceToHost, s));
    return HGT_OK;
}

// After the synchronisation: the batch's verdict, then capacities for the commit
// and the incident-vertex pair list.
int plan_end(Pending& p, hipStream_t s) {
    hgt_graph* g = p.g;
    p.sum = *g->h_sum;
    if (p.sum.status != HGT_OK) return p.sum.status;
    const BatchSummary& sum = p.sum;
    int rc = ensure_pool(g->h2v, g->h_bump, sum.h2v_need, s);
    if (!rc && (g->track_mask & (1u << HGT_TRIAD_HYPEREDGE)) && g->hpool.bytes < 2 * g->h2v.bytes)
        rc = grow_keep(g->hpool, 2 * g->h2v.bytes, 2 * g->h_bump * 4, s);
    if (!rc) rc = ensure_pool(g->v2h, g->v_bump, sum.v2h_need, s);
    const bool tmp = g->track_mask & (1u << HGT_TRIAD_TEMPORAL);
    // the timestamp pool follows the v2h pool word for word
    if (!rc && tmp && g->v2h_ts.bytes < 2 * g->v2h.bytes)
        rc = grow_keep(g->v2h_ts, 2 * g->v2h.bytes, g->v_bump * 8, s);
    if (!rc) rc = ensure(g->s_staging, std::max<uint64_t>(sum.stage_words, 1) * 4);
    if (!rc && tmp) rc = ensure(g->s_staging_ts, std::max<uint64_t>(sum.stage_words, 1) * 8);
    if (rc) return rc;
    refresh_view(g);
    p.w.staging = g->s_staging.as<uint32_t>();
    p.w.staging_ts = g->s_staging_ts.as<int64_t>();
    if (g->track_mask & (1u << HGT_TRIAD_INCIDENT_VERTEX)) {
        ProfScope ps(g, PK_IV_PREP, s);
        rc = iv_prepare(g, p.b, p.w, sum, p.ip, s);
        if (rc) return rc;
    }
    return HGT_OK;
}

PhaseJob job_minus(const Pending& p) {
    hgt_graph* g = p.g;
    return PhaseJob{g, p.b.del, p.b.n_del, g->st.mark_del, p.b.epoch_del, p.sum.max_lh_del, p.sum.sum_lh_del,
                    g->next_id};
}

PhaseJob job_plus(const Pending& p) {
    hgt_graph* g = p.g;
    return PhaseJob{g, p.w.assigned, p.b.n_ins, g->st.mark_ins, p.b.epoch_ins, p.sum.max_lh_ins, p.sum.sum_lh_ins,
                    p.sum.next_id_new};
}

// Every scratch buffer of both phases, reserved before the first kernel that
// changes the graph.  In a no-allocation call they come from the arena, so a
// batch whose scratch does not fit is rejected with nothing changed.  With
// upload set the descriptors of every (phase, family) are uploaded too (on
// stream s, which may be the null stream), for a round that is then captured
// into a HIP graph (a second pass if the descriptor buffer had to grow under the
// first, which moves it).
int reserve_all_phases(hgt_graph* owner, std::vector<Pending*>& ps, bool upload = false, hipStream_t s = nullptr) {
    PhaseCtx& c = ctx_of(owner);
    std::vector<HeGraph> G;
    std::vector<uint64_t> base, id_base;
    const uint64_t cap0 = c.desc_cap;
    for (int slot = 0; slot < 4; slot++) c.pre_ok[slot] = false;
    for (int phase = 0; phase < 2; phase++) {
        std::vector<PhaseJob> jobs;
        for (Pending* p : ps) jobs.push_back(phase == 0 ? job_minus(*p) : job_plus(*p));
        for (int family : {HGT_TRIAD_HYPEREDGE, HGT_TRIAD_TEMPORAL}) {
            uint64_t max_lh, sum_lh;
            collect(jobs.data(), (uint32_t)jobs.size(), family, phase == 0, G, base, id_base, max_lh, sum_lh);
            if (base.back() == 0) continue;
            const PhaseShape z = phase_shape(owner, base.back(), max_lh, sum_lh, id_base.back(), t_na != nullptr);
            if (int rc = phase_reserve(c, family, z)) return rc;
            if (upload) {
                const int slot = (phase == 0 ? 0 : 2) + (family == HGT_TRIAD_TEMPORAL ? 1 : 0);
                if (int rc = upload_multi(c, slot, G, base, id_base, c.pre[slot], s)) return rc;
                c.pre_ok[slot] = true;
            }
        }
    }
    if (upload && c.desc_cap != cap0) return reserve_all_phases(owner, ps, upload, s);
    if (t_na)
        if (int rc = ensure(c.desc, 4 * desc_slot_bytes(1))) return rc;
    for (Pending* p : ps)
        if ((p->g->track_mask & (1u << HGT_TRIAD_INCIDENT_VERTEX)) && p->ip.n_keys)
            if (int rc = iv_reserve(p->g, p->ip)) return rc;
    return HGT_OK;
}

// Applies the planned batches of `ps` (all with rc == 0) on stream s: deltas on
// the old graphs, delete + insert, deltas on the new graphs, count update.  The
// hyperedge and temporal phases of all graphs share one launch per kernel.
// Changes no host state, so a round whose capture failed can be launched again.
// HGT_INJECT_FAULT=1 (tests): a batch that passed validation stops right after
// its store update has been queued and fails as a HIP launch would, leaving
// the graph part-way (every kernel queued so far still runs to completion).
bool fault_injected() {
    const char* f = std::getenv("HGT_INJECT_FAULT");
    return f && std::atoi(f) == 1;
}

// *began is set once the first kernel that changes graph state or counts may
// have been queued: a failure after that leaves the graphs of `ps` part-way.
int apply_locked(hgt_graph* owner, std::vector<Pending*>& ps, hipStream_t s, bool* began) {
    int rc;
    if (t_na && (rc = reserve_all_phases(owner, ps))) return rc;
    *began = true;
    std::vector<PhaseJob> jobs;
    jobs.reserve(ps.size());
    for (Pending* p : ps) jobs.push_back(job_minus(*p));
    bool full = !ps.empty() && ps[0]->is_build;
    // step 2: deltas on the old graph
    rc = run_phase(owner, jobs.data(), (uint32_t)jobs.size(), true, false, s);
    if (rc) return rc;
    for (Pending* p : ps)
        if ((p->g->track_mask & (1u << HGT_TRIAD_INCIDENT_VERTEX)) && (rc = iv_phase(p->g, p->ip, true, s)))
            return rc;
    // step 3: delete, then insert
    for (Pending* p : ps) {
        hgt_graph* g = p->g;
        {
            ProfScope sc(g, PK_COMMIT, s);
            store_commit(g->st, p->b, p->w, p->sum, g->h_bump, g->v_bump, g->next_seq, s);
        }
        if (p->out_ids && p->b.n_ins)
            HIP_OK(hipMemcpyAsync(p->out_ids, p->w.assigned, p->b.n_ins * 4, hipMemcpyDeviceToDevice, s));
    }
    if (!t_capture && fault_injected()) return HGT_EDEVICE;
    // step 5: deltas on the new graph
    jobs.clear();
    for (Pending* p : ps) jobs.push_back(job_plus(*p));
    rc = run_phase(owner, jobs.data(), (uint32_t)jobs.size(), false, full, s);
    if (rc) return rc;
    for (Pending* p : ps)
        if ((p->g->track_mask & (1u << HGT_TRIAD_INCIDENT_VERTEX)) && (rc = iv_phase(p->g, p->ip, false, s)))
            return rc;
    // step 6
    for (Pending* p : ps) {
        hgt_graph* g = p->g;
        uint64_t* cnt = g->counts.as<uint64_t>();
        k_he_tmp_update<<<1, 128, 0, s>>>(cnt);
        if (g->track_mask & (1u << HGT_TRIAD_INCIDENT_VERTEX))
            k_iv_update<<<1, 64, 0, s>>>(cnt, CNT_IV, ACC_IV_M, ACC_IV_P, ACC_T1);
    }
    HIP_OK(hipGetLastError());
    return HGT_OK;
}

// The host mirrors of the graphs, once the round's work is queued.
void commit_mirrors(std::vector<Pending*>& ps) {
    for (Pending* p : ps) {
        hgt_graph* g = p->g;
        g->next_id = p->sum.next_id_new;
        g->h_bump += p->sum.h2v_need;
        g->v_bump += p->sum.v2h_need;
        if (!p->b.keep_seq) g->next_seq += p->b.n_ins;
        g->n_live = g->n_live + p->b.n_ins - p->b.n_del;
        g->n_inc = g->n_inc + p->n_mem - p->sum.del_members;
        g->batches++;
        // algorithmic bytes of the store update: an insert of cardinality d reads its
        // input (4d + 8) and writes its h2v block (4d) and v2h entries (4d, locating
        // them reads 4d); a delete reads its h2v block (4d) and rewrites its v2h
        // entries (8d)
        if (g->prof) g->store_bytes += 16 * p->n_mem + 16 * p->b.n_ins + 12 * p->sum.del_members + 8 * p->b.n_del;
    }
}

// The post-planning half of a round captured into a HIP graph and launched as
// one: every scratch buffer is reserved and every descriptor uploaded before
// the capture.  The executable graph of the previous round on this phase
// context is updated in place when the shapes agree, else instantiated anew.
// kCaptureFailed: the capture did not succeed and nothing was launched.
constexpr int kCaptureFailed = 1;
// HGT_GRAPH_DEBUG=1: say on stderr why a capture fell back to the launch kernel by kernel
void capture_note(const char* what, int code) {
    static const bool on = std::getenv("HGT_GRAPH_DEBUG") != nullptr;
    if (on) std::fprintf(stderr, "[hgt] graph launch fell back: %s (%d)\n", what, code);
}
int apply_graph(hgt_graph* owner, std::vector<Pending*>& ps, hipStream_t s, bool* began) {
    PhaseCtx& c = ctx_of(owner);
    int rc = reserve_all_phases(owner, ps, true, s);
    if (rc) return rc;
    hipStream_t cs = s;  // the stream captured and launched on
    if (!s) {
        if (!c.cap_stream) {
            hipStream_t st = nullptr;
            hipEvent_t e_in = nullptr, e_out = nullptr;
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&e_in, hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&e_out, hipEventDisableTiming) != hipSuccess) {
                (void)hipGetLastError();
                if (st) (void)hipStreamDestroy(st);
                if (e_in) (void)hipEventDestroy(e_in);
                return kCaptureFailed;
            }
            c.cap_stream = st;
            c.cap_in = e_in;
            c.cap_out = e_out;
        }
        cs = c.cap_stream;
        HIP_OK(hipEventRecord(c.cap_in, s));
        HIP_OK(hipStreamWaitEvent(cs, c.cap_in, 0));
    }
    if (hipError_t be = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed); be != hipSuccess) {
        (void)hipGetLastError();
        capture_note("begin capture", (int)be);
        return kCaptureFailed;
    }
    t_capture = 1;
    bool captured_only = false;  // nothing runs while the stream is captured
    rc = apply_locked(owner, ps, cs, &captured_only);
    t_capture = 0;
    hipGraph_t gr = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &gr);
    for (int slot = 0; slot < 4; slot++) c.pre_ok[slot] = false;
    if (rc || e != hipSuccess || !gr) {
        (void)hipGetLastError();
        if (gr) (void)hipGraphDestroy(gr);
        capture_note(rc ? "launch under capture" : "end capture", rc ? rc : (int)e);
        return kCaptureFailed;
    }
    bool updated = false;
    if (c.gexec) {
        hipGraphNode_t err_node = nullptr;
        hipGraphExecUpdateResult res;
        updated = hipGraphExecUpdate(c.gexec, gr, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess;
        if (!updated) {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(c.gexec);
            c.gexec = nullptr;
        }
    }
    if (!updated && hipGraphInstantiate(&c.gexec, gr, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        capture_note("instantiate", 0);
        c.gexec = nullptr;
        (void)hipGraphDestroy(gr);
        return kCaptureFailed;
    }
    (void)hipGraphDestroy(gr);
    *began = true;
    HIP_OK(hipGraphLaunch(c.gexec, cs));
    if (cs != s) {
        HIP_OK(hipEventRecord(c.cap_out, cs));
        HIP_OK(hipStreamWaitEvent(s, c.cap_out, 0));
    }
    owner->graph_launches++;
    return HGT_OK;
}

int apply_planned(hgt_graph* owner, std::vector<Pending*>& ps, hipStream_t s, bool graph = false) {
    PhaseCtx& c = ctx_of(owner);
    std::lock_guard<std::mutex> lk(c.mu);
    HIP_OK(hipStreamWaitEvent(s, c.done, 0));
    if (t_tune_ev[0]) (void)hipEventRecord(t_tune_ev[0], s);
    int rc = kCaptureFailed;
    bool began = false;
    if (graph && !t_na && !fault_injected()) rc = apply_graph(owner, ps, s, &began);
    if (rc == kCaptureFailed) rc = apply_locked(owner, ps, s, &began);  // launched one by one
    if (rc == HGT_OK) commit_mirrors(ps);
    if (t_tune_ev[1]) (void)hipEventRecord(t_tune_ev[1], s);
    if (hipEventRecord(c.done, s) != hipSuccess && rc == HGT_OK) rc = HGT_EDEVICE;
    if (rc != HGT_OK && began) {
        // part of the round may have run: its graphs' device state no longer
        // matches their host mirrors or their counts
        for (Pending* p : ps) {
            p->g->poisoned = true;
            p->g->sticky = HGT_EPOISONED;
        }
        rc = HGT_EPOISONED;
    }
    return rc;
}

void set_sticky(hgt_graph* g, int rc) {
    if (rc && !g->sticky) g->sticky = rc;
}

// What a batch is: an update batch, the build (every hyperedge inserted into
// the empty graph, counted by the static mode), or horizontal operations
// (the modified hyperedges deleted and reinserted under the same IDs with
// their timestamps and arrival sequences kept).
enum ApplyMode { MODE_BATCH = 0, MODE_BUILD, MODE_VOPS };

// One batch.
int apply(hgt_graph* g, const uint32_t* del, uint64_t n_del, const uint64_t* ins_off, const uint32_t* ins_mem,
          uint64_t n_mem, const int64_t* ins_ts, uint64_t n_ins, uint32_t* out_ids, hipStream_t s,
          ApplyMode mode = MODE_BATCH, const uint32_t* forced_ids = nullptr) {
    Pending p;
    p.g = g;
    p.out_ids = out_ids;
    p.check_order = mode == MODE_BATCH ? 1 : 0;
    p.is_build = mode == MODE_BUILD ? 1 : 0;
    p.forced_ids = forced_ids;
    p.keep_seq = mode == MODE_VOPS ? 1 : 0;
    int rc = plan_begin(p, del, n_del, ins_off, ins_mem, n_mem, ins_ts, n_ins, s);
    if (rc == HGT_ENOENT) set_sticky(g, rc);
    if (rc) return rc;
    HIP_OK(hipStreamSynchronize(s));
    rc = plan_end(p, s);
    if (rc) {
        set_sticky(g, rc);
        return rc;
    }
    std::vector<Pending*> ps{&p};
    return apply_planned(g, ps, s);
}

void destroy_graph(hgt_graph* g) {
    if (!g) return;
    DevBuf* all[] = {&g->h_off, &g->h_len, &g->h_cap, &g->h_ts, &g->h_seq, &g->free_bm, &g->mark_del, &g->mark_ins,
                     &g->h2v, &g->v_off, &g->v_len, &g->v_cap, &g->v2h, &g->scal, &g->counts, &g->tabs,
                     &g->s_sum, &g->s_del_bm, &g->s_del_card, &g->s_del_poff, &g->s_ins_rel, &g->s_ins_card,
                     &g->s_canon, &g->s_big, &g->s_small, &g->s_popc, &g->s_scan, &g->s_assigned, &g->s_h_need,
                     &g->s_h_rel, &g->s_keys, &g->s_keys_alt, &g->s_sort, &g->s_head, &g->s_is_ins, &g->s_tv,
                     &g->s_tseg, &g->s_D, &g->s_I, &g->s_It, &g->s_vp, &g->s_staging, &g->s_dst,
                     &g->s_staging_ts, &g->v2h_ts, &g->iv_keys, &g->iv_alt, &g->iv_sort,
                     &g->iv_head, &g->iv_uniq, &g->iv_p2, &g->iv_scan, &g->iv_tab, &g->iv_owner, &g->iv_ctr,
                     &g->hpool, &g->vo_sum, &g->vo_keys, &g->vo_alt, &g->vo_sort, &g->vo_scan, &g->vo_head,
                     &g->vo_ins, &g->vo_nmod, &g->vo_mod, &g->vo_seg, &g->vo_card, &g->vo_ts, &g->vo_off, &g->vo_mem};
    for (DevBuf* b : all) dev_free(*b);
    if (g->ph) phase_ctx_release(g->ph);
    dev_free(g->stats);
    for (hipEvent_t e : g->ev_pool) (void)hipEventDestroy(e);
    if (g->h_sum) (void)hipHostFree(g->h_sum);
    if (g->h_sc) (void)hipHostFree(g->h_sc);
    delete g;
}

}  // namespace

// ---- hooks for the request server (internal.h) -----------------------------
PhaseCtx* hgt_phase_ctx_create(int device) {
    PhaseCtx* c = new (std::nothrow) PhaseCtx();
    if (!c) return nullptr;
    c->device = device;
    if (hipEventCreateWithFlags(&c->done, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return nullptr;
    }
    return c;
}

void hgt_phase_ctx_destroy(PhaseCtx* c) {
    if (!c) return;
    (void)hipEventSynchronize(c->done);
    phase_ctx_free(*c);
    delete c;
}

void hgt_use_phase_ctx(PhaseCtx* c) { t_ph = c; }

int hgt_counts_async(hgt_graph* g, uint64_t* dst, hipStream_t s) {
    static_assert(CNT_N == HGT_COUNT_WORDS, "count layout");
    HIP_OK(hipMemcpyAsync(dst, g->counts.p, CNT_N * 8, hipMemcpyDeviceToHost, s));
    return HGT_OK;
}

HgtSizes hgt_sizes(hgt_graph* g) {
    HgtSizes z;
    z.n_vertices = g->st.n_vertices;
    z.track_mask = g->track_mask;
    z.n_live = g->n_live;
    z.n_inc = g->n_inc;
    z.device = g->device;
    return z;
}

// ---------------------------------------------------------------------------
// scratch of the no-allocation entry point
// ---------------------------------------------------------------------------
// One copy per GPU, held until the process ends.  In host code the array's
// name is not a device address: its address on a device comes from
// hipGetSymbolAddress (once per device, with that device current) and only
// that address is handed to kernels.
constexpr uint64_t kNoAllocScratchBytes = 256ull << 20;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_na_mu;
char* g_na_base[kMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current).
int noalloc_base(int device, char** out) {
    if (device < 0 || device >= kMaxDevices) return HGT_EINVAL;
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_base[device]) {
        void* ptr = nullptr;
        if (hip_failed(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress", __LINE__) || !ptr)
            return HGT_EDEVICE;
        g_na_base[device] = (char*)ptr;
    }
    *out = g_na_base[device];
    return HGT_OK;
}
}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* hgt_status_str(int status) {
    switch (status) {
        case HGT_OK: return "ok";
        case HGT_EINVAL: return "invalid argument or member list";
        case HGT_ENOENT: return "deleted ID is not live";
        case HGT_EDUP: return "ID repeated in a deletion list";
        case HGT_EORDER: return "temporal insert out of order";
        case HGT_ENOMEM: return "device memory exhausted";
        case HGT_ENOTTRACKED: return "triad family or window not tracked";
        case HGT_EDEVICE: return "HIP runtime failure";
        case HGT_EPOISONED: return "graph left part-way through a batch: restore a snapshot or destroy it";
        default: return "unknown status";
    }
}

int hgt_class_codes(int type, int32_t* out_host, uint32_t n) {
    const ClassTables& t = tables();
    const std::vector<int32_t>* v = type == HGT_TRIAD_HYPEREDGE ? &t.he_codes
                                    : type == HGT_TRIAD_TEMPORAL ? &t.tmp_codes
                                                                 : nullptr;
    if (!v) return HGT_EINVAL;
    if (out_host) {
        if (n < v->size()) return HGT_EINVAL;
        std::memcpy(out_host, v->data(), v->size() * 4);
    }
    return (int)v->size();
}

int hgt_build(const hgt_build_desc* d, hgt_graph** out) {
    if (!d || !out) return HGT_EINVAL;
    *out = nullptr;
    if (d->n_vertices == 0 || d->n_vertices > 0x7fffffffu) return HGT_EINVAL;
    if (d->n_edges && (!d->offsets || !d->members)) return HGT_EINVAL;
    if (d->track_mask & ~7u) return HGT_EINVAL;
    const bool tmp = d->track_mask & (1u << HGT_TRIAD_TEMPORAL);
    if (tmp && d->n_edges && !d->timestamps) return HGT_EINVAL;
    if (d->temporal_window < 0) return HGT_EINVAL;
    if (d->n_edges > 0xfffffff0ull) return HGT_EINVAL;
    hipStream_t s = (hipStream_t)d->stream;
    hgt_graph* g = new (std::nothrow) hgt_graph();
    if (!g) return HGT_ENOMEM;
    g->track_mask = d->track_mask;
    g->window = d->temporal_window;
    g->last_stream = s;
    if (const char* fs = std::getenv("HGT_FORCE_STAGE")) g->force_stage = std::atoi(fs);
    if (const char* pa = std::getenv("HGT_PAIR_AGG")) g->pair_agg = std::atoi(pa) != 0;
    if (const char* gw = std::getenv("HGT_GLOBAL_WG_PER_CU")) g->global_wg_per_cu = std::max(1, std::min(16, std::atoi(gw)));
    if (const char* sk = std::getenv("HGT_SKIP_LDS148")) g->skip_lds148 = std::atoi(sk) != 0;
    if (const char* iw = std::getenv("HGT_IV_WG_PER_CU")) g->iv_wg_per_cu = std::max(1, std::min(16, std::atoi(iw)));
    if (const char* sl = std::getenv("HGT_SLICE_LH")) g->slice_lh = (uint32_t)std::max(1, std::atoi(sl));
    if (const char* e2 = std::getenv("HGT_E2_2HOP")) g->e2_2hop = std::strtoull(e2, nullptr, 10);
    if (const char* w2 = std::getenv("HGT_W_2HOP")) g->w_2hop = (uint32_t)std::min<uint64_t>(std::strtoull(w2, nullptr, 10), 1u << 21);
    if (const char* iv = std::getenv("HGT_IV_DIRECT")) g->iv_direct = std::atoi(iv) != 0;
    if (const char* fs = std::getenv("HGT_IV_FORCE_STAGE")) g->iv_force_stage = std::atoi(fs);
    if (const char* ws = std::getenv("HGT_WAVE_SLOTS")) {  // a power of two, 64 .. 2^20
        const long v = std::atol(ws);
        if (v >= 64 && v <= (1l << 20) && (v & (v - 1)) == 0) g->wave_slots = (uint32_t)v;
    }
    int rc = HGT_OK;
    do {
        HIP_BRK(hipGetDevice(&g->device));
        if (!(g->ph = phase_ctx_acquire(g->device))) { rc = HGT_ENOMEM; break; }
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, g->device) == hipSuccess && ncu > 0)
            g->n_cu = ncu;
        if (hipHostMalloc((void**)&g->h_sum, sizeof(BatchSummary), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&g->h_sc, sizeof(DevScalars), hipHostMallocDefault) != hipSuccess) {
            rc = HGT_ENOMEM;
            break;
        }
        g->st.n_vertices = d->n_vertices;
        g->st.id_cap = 0;
        uint64_t cap = std::max<uint64_t>(d->edge_capacity, d->n_edges + d->n_edges / 4 + 64);
        if ((rc = ensure_id_cap(g, cap, s))) break;
        uint64_t V = d->n_vertices;
        if ((rc = dev_alloc(g->v_off, V * 8)) || (rc = dev_alloc(g->v_len, V * 4)) || (rc = dev_alloc(g->v_cap, V * 4)))
            break;
        HIP_BRK(hipMemsetAsync(g->v_off.p, 0, V * 8, s));
        HIP_BRK(hipMemsetAsync(g->v_len.p, 0, V * 4, s));
        HIP_BRK(hipMemsetAsync(g->v_cap.p, 0, V * 4, s));
        uint64_t pw = d->pool_words ? d->pool_words : 1 << 20;
        if ((rc = dev_alloc(g->h2v, pw * 4)) || (rc = dev_alloc(g->v2h, pw * 4))) break;
        if (tmp && (rc = dev_alloc(g->v2h_ts, pw * 8))) break;
        if ((d->track_mask & (1u << HGT_TRIAD_HYPEREDGE)) && (rc = dev_alloc(g->hpool, pw * 8))) break;
        if ((rc = dev_alloc(g->scal, sizeof(DevScalars))) || (rc = dev_alloc(g->counts, ACC_N * 8)) ||
            (rc = dev_alloc(g->tabs, 256)))
            break;
        DevScalars z{};
        z.last_ts = INT64_MIN;
        const ClassTables& t = tables();
        uint8_t tb[256];
        std::memcpy(tb, t.he, 128);
        std::memcpy(tb + 128, t.tmp, 128);
        HIP_BRK(hipMemcpyAsync(g->scal.p, &z, sizeof z, hipMemcpyHostToDevice, s));
        HIP_BRK(hipMemsetAsync(g->counts.p, 0, ACC_N * 8, s));
        HIP_BRK(hipMemcpyAsync(g->tabs.p, tb, 256, hipMemcpyHostToDevice, s));
        HIP_BRK(hipStreamSynchronize(s));
        refresh_view(g);
        if (d->n_edges) {
            // build = insert every hyperedge into the empty graph; the inserted
            // hyperedges' deltas are the initial counts
            uint64_t first = 0, last = 0;
            HIP_BRK(hipMemcpy(&first, d->offsets, 8, hipMemcpyDeviceToHost));
            HIP_BRK(hipMemcpy(&last, d->offsets + d->n_edges, 8, hipMemcpyDeviceToHost));
            if (last < first) { rc = HGT_EINVAL; break; }
            if (tmp) store_max_ts(d->timestamps, d->n_edges, g->st.sc, s);
            rc = apply(g, nullptr, 0, d->offsets, d->members, last - first, tmp ? d->timestamps : nullptr, d->n_edges,
                       nullptr, s, MODE_BUILD);
            if (rc) break;
            HIP_BRK(hipStreamSynchronize(s));
        }
    } while (0);
    if (rc) {
        destroy_graph(g);
        return rc;
    }
    g->sticky = HGT_OK;
    *out = g;
    return HGT_OK;
}

int hgt_apply_batch(hgt_graph* g, const uint32_t* del_ids, uint64_t n_del, const uint64_t* ins_offsets,
                    const uint32_t* ins_members, uint64_t n_ins_members, const int64_t* ins_ts, uint64_t n_ins,
                    uint32_t* out_ins_ids, void* stream) {
    if (!g) return HGT_EINVAL;
    if (g->poisoned) return HGT_EPOISONED;
    if (n_del == 0 && n_ins == 0) return HGT_OK;
    int rc = apply(g, del_ids, n_del, ins_offsets, ins_members, n_ins_members, ins_ts, n_ins, out_ins_ids,
                   (hipStream_t)stream);
    if (rc && !g->sticky) g->sticky = rc;
    return rc;
}

int hgt_apply_vertex_ops(hgt_graph* g, const uint32_t* edge_ids, const uint32_t* vertices, const uint8_t* insert,
                         uint64_t n_ops, void* stream) {
    if (!g) return HGT_EINVAL;
    if (g->poisoned) return HGT_EPOISONED;
    if (n_ops == 0) return HGT_OK;
    if (!edge_ids || !vertices || !insert || n_ops > 0xfffffff0ull) return HGT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    g->last_stream = s;
    const bool tmp = g->track_mask & (1u << HGT_TRIAD_TEMPORAL);
    VopIn in{};
    in.edge_ids = edge_ids;
    in.vertices = vertices;
    in.insert = insert;
    in.n = n_ops;
    in.hb = bits_for(g->next_id);
    in.vb = bits_for(g->st.n_vertices ? g->st.n_vertices - 1 : 0);
    if (in.hb + in.vb + 1 > 64) return HGT_EINVAL;
    in.n_vertices = g->st.n_vertices;
    in.free_bm = g->st.free_bm;
    in.h_off = g->st.h_off;
    in.h_len = g->st.h_len;
    in.h2v = g->st.h2v;
    in.h_ts = tmp ? g->st.h_ts : nullptr;
    in.sc = g->st.sc;
    const uint64_t n = n_ops;
    int rc = 0;
    rc |= ensure(g->vo_sum, sizeof(VopSummary));
    rc |= ensure(g->vo_keys, n * 8);
    rc |= ensure(g->vo_alt, n * 8);
    rc |= ensure(g->vo_sort, hgt_radix_tmp_bytes(n));
    rc |= ensure(g->vo_scan, hgt_scan_tmp_bytes(n + 1));
    rc |= ensure(g->vo_head, n * 8);
    rc |= ensure(g->vo_ins, (n + 1) * 8);
    rc |= ensure(g->vo_nmod, 64);
    rc |= ensure(g->vo_mod, n * 4);
    rc |= ensure(g->vo_seg, (n + 1) * 8);
    rc |= ensure(g->vo_card, n * 8);
    rc |= ensure(g->vo_ts, n * 8);
    rc |= ensure(g->vo_off, (n + 1) * 8);
    if (rc) return HGT_ENOMEM;
    VopScratch w{};
    w.sum = g->vo_sum.as<VopSummary>();
    w.keys = g->vo_keys.as<uint64_t>();
    w.keys_alt = g->vo_alt.as<uint64_t>();
    w.sort_tmp = g->vo_sort.p;
    w.scan_tmp = g->vo_scan.p;
    w.head = g->vo_head.as<uint64_t>();
    w.ins_pre = g->vo_ins.as<uint64_t>();
    w.n_mod = g->vo_nmod.as<uint64_t>();
    w.mod_ids = g->vo_mod.as<uint32_t>();
    w.seg = g->vo_seg.as<uint64_t>();
    w.card = g->vo_card.as<uint64_t>();
    w.ts = tmp ? g->vo_ts.as<int64_t>() : nullptr;
    w.new_off = g->vo_off.as<uint64_t>();
    vops_plan(in, w, s);
    static_assert(sizeof(VopSummary) <= sizeof(BatchSummary), "summary staging");
    VopSummary* hs = (VopSummary*)g->h_sum;  // pinned; the batch below rewrites it after its own plan
    HIP_OK(hipMemcpyAsync(hs, w.sum, sizeof(VopSummary), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    const VopSummary sum = *hs;
    if (sum.status) {
        if (!g->sticky) g->sticky = sum.status;
        return sum.status;
    }
    if (ensure(g->vo_mem, std::max<uint64_t>(sum.n_members, 1) * 4)) return HGT_ENOMEM;
    w.members = g->vo_mem.as<uint32_t>();
    vops_rows(in, w, sum.n_mod, s);
    rc = apply(g, w.mod_ids, sum.n_mod, w.new_off, w.members, sum.n_members, w.ts, sum.n_mod, nullptr, s, MODE_VOPS,
               w.mod_ids);
    if (rc && !g->sticky) g->sticky = rc;
    return rc;
}

int hgt_apply_batch_noalloc(hgt_graph* g, const uint32_t* del_ids, uint64_t n_del, const uint64_t* ins_offsets,
                            const uint32_t* ins_members, uint64_t n_ins_members, const int64_t* ins_ts,
                            uint64_t n_ins, uint32_t* out_ins_ids, void* stream) {
    if (!g) return HGT_EINVAL;
    if (g->poisoned) return HGT_EPOISONED;
    if (n_del == 0 && n_ins == 0) return HGT_OK;
    int cur = -1;
    HIP_OK(hipGetDevice(&cur));
    if (cur != g->device) return HGT_EINVAL;  // the scratch copy must be the graph's GPU's
    char* base = nullptr;
    int rc = noalloc_base(g->device, &base);
    if (rc) return rc;
    NoAllocArena a;
    a.base = base;
    a.cap = kNoAllocScratchBytes;
    t_na = &a;
    rc = apply(g, del_ids, n_del, ins_offsets, ins_members, n_ins_members, ins_ts, n_ins, out_ins_ids,
               (hipStream_t)stream);
    t_na = nullptr;
    // the graph's own scratch buffers are its again (queued kernels keep using the
    // arena regions they were given; the arena is never freed)
    for (int i = a.n_undo - 1; i >= 0; i--) *a.undo[i].b = a.undo[i].old;
    if (rc && !g->sticky) g->sticky = rc;
    return rc;
}

namespace {

// Online autotuner of the batched form.  A round's key bins it by the tracked
// families, the number of graphs (log2), the changes and the 2-hop load of its
// heaviest centre (log4 buckets).  Each round is timed by two events around
// its launches, read back without a wait at a later call.  The choices are
// tried in turn; one whose quickest trial is more than kTuneDrop times the
// best choice's is dropped, and once every remaining choice has kTuneTrials
// trials the fastest (by its quickest trial) is kept for the key and appended
// to the cache file, which later processes read first.
constexpr TuneChoice kTune[] = {{4, 1, 8192, 0},       {2, 1, 8192, 0},       {8, 1, 8192, 0},
                                {4, 0, 8192, 0},       {4, 1, 32768, 0},      {4, 1, 8192, 1u << 18},
                                {4, 1, 8192, 1u << 21}};
constexpr int kTuneN = (int)(sizeof(kTune) / sizeof(kTune[0]));
constexpr int kTuneTrials = 2;
constexpr float kTuneDrop = 1.25f;

struct TuneEntry {
    float best_ms[kTuneN];
    int trials[kTuneN];
    int pick = -1;
    TuneEntry() {
        for (int i = 0; i < kTuneN; i++) best_ms[i] = 1e30f, trials[i] = 0;
    }
};

struct Tuner {
    std::mutex mu;
    std::map<uint64_t, TuneEntry> tab;
    bool loaded = false;
    std::string path;  // empty: no cache file
    struct Open {
        uint64_t key;
        int choice;
        hipEvent_t a, b;
    };
    std::vector<Open> open;
};

Tuner& tuner() {
    static Tuner* t = new Tuner();  // outlives every graph (never destroyed)
    return *t;
}

inline int ilog2_bucket(uint64_t x) { return x ? 64 - __builtin_clzll(x) : 0; }

uint64_t tune_key(const std::vector<Pending*>& ps, int n_cu) {
    uint64_t changes = 0, lh = 0;
    uint32_t mask = 0;
    for (const Pending* p : ps) {
        changes += p->b.n_del + p->b.n_ins;
        lh = std::max(lh, std::max(p->sum.max_lh_del, p->sum.max_lh_ins));
        mask |= p->g->track_mask;
    }
    return ((uint64_t)(n_cu & 0xffff) << 40) | ((uint64_t)(mask & 0xff) << 32) |
           ((uint64_t)ilog2_bucket(ps.size()) << 24) | ((uint64_t)(ilog2_bucket(changes) / 2) << 16) |
           ((uint64_t)(ilog2_bucket(lh) / 2) << 8);
}

// Cache file: one line per settled key, "key choice wg_per_cu skip_lds148
// wave_slots e2_2hop best_ms"; lines whose choice does not match this library's
// table are ignored.
void tune_load(Tuner& T) {
    if (T.loaded) return;
    T.loaded = true;
    const char* e = std::getenv("HGT_TUNE_CACHE");
    if (e) {
        T.path = e;
    } else if (const char* home = std::getenv("HOME")) {
        T.path = std::string(home) + "/.cache/hgt_tune.txt";
    }
    if (T.path.empty() || T.path == "off") {
        T.path.clear();
        return;
    }
    FILE* f = std::fopen(T.path.c_str(), "r");
    if (!f) return;
    unsigned long long key, e2;
    int choice, wg, skip;
    unsigned slots;
    float ms;
    while (std::fscanf(f, "%llx %d %d %d %u %llu %f", &key, &choice, &wg, &skip, &slots, &e2, &ms) == 7) {
        if (choice < 0 || choice >= kTuneN || kTune[choice].wg_per_cu != wg || kTune[choice].skip_lds148 != skip ||
            kTune[choice].wave_slots != slots || kTune[choice].e2_2hop != e2)
            continue;
        TuneEntry& t = T.tab[(uint64_t)key];
        t.pick = choice;
        t.best_ms[choice] = ms;
    }
    std::fclose(f);
}

// Whether choice c is still in the running: untried, or within kTuneDrop of
// the best quickest trial so far.
bool tune_live(const TuneEntry& t, int c) {
    float best = 1e30f;
    for (int i = 0; i < kTuneN; i++) best = std::min(best, t.best_ms[i]);
    return t.trials[c] == 0 || t.best_ms[c] <= kTuneDrop * best;
}

void tune_settle(Tuner& T, uint64_t key, TuneEntry& t) {
    int best = 0;
    for (int i = 1; i < kTuneN; i++)
        if (t.best_ms[i] < t.best_ms[best]) best = i;
    t.pick = best;
    if (T.path.empty()) return;
    if (FILE* f = std::fopen(T.path.c_str(), "a")) {
        const TuneChoice& c = kTune[best];
        std::fprintf(f, "%llx %d %d %d %u %llu %.4f\n", (unsigned long long)key, best, c.wg_per_cu, c.skip_lds148,
                     c.wave_slots, (unsigned long long)c.e2_2hop, t.best_ms[best]);
        std::fclose(f);
    }
}

// Reads back the timed rounds whose second event has passed (all of them,
// waiting, when wait is set).
void tune_harvest(Tuner& T, bool wait) {
    size_t kept = 0;
    for (size_t i = 0; i < T.open.size(); i++) {
        Tuner::Open& o = T.open[i];
        if (wait) (void)hipEventSynchronize(o.b);
        const hipError_t q = hipEventQuery(o.b);
        if (q == hipErrorNotReady) {
            T.open[kept++] = o;
            continue;
        }
        float ms = 0.f;
        if (q == hipSuccess && hipEventElapsedTime(&ms, o.a, o.b) == hipSuccess) {
            TuneEntry& t = T.tab[o.key];
            if (t.pick < 0) {
                t.best_ms[o.choice] = std::min(t.best_ms[o.choice], ms);
                t.trials[o.choice]++;
                bool done = true;
                for (int c = 0; c < kTuneN; c++) done &= !tune_live(t, c) || t.trials[c] >= kTuneTrials;
                if (done) tune_settle(T, o.key, t);
            }
        }
        (void)hipGetLastError();
        (void)hipEventDestroy(o.a);
        (void)hipEventDestroy(o.b);
    }
    T.open.resize(kept);
}

// The choice for a round's key: the settled one, else the one with the fewest
// trials (HGT_TUNE_FORCE=k, for tests, forces choice k).
int tune_pick(Tuner& T, uint64_t key) {
    if (const char* f = std::getenv("HGT_TUNE_FORCE")) {
        const int k = std::atoi(f);
        if (k >= 0 && k < kTuneN) return k;
    }
    TuneEntry& t = T.tab[key];
    if (t.pick >= 0) return t.pick;
    int c = -1, pending[kTuneN] = {};
    for (const Tuner::Open& o : T.open)
        if (o.key == key) pending[o.choice]++;
    for (int i = 0; i < kTuneN; i++)
        if (tune_live(t, i) && (c < 0 || t.trials[i] + pending[i] < t.trials[c] + pending[c])) c = i;
    return c < 0 ? 0 : c;
}

int apply_batches(hgt_batch* bs, uint32_t n, void* stream, uint32_t flags) {
    if (n == 0) return HGT_OK;
    if (!bs || (flags & ~(uint32_t)(HGT_BATCHES_GRAPH | HGT_BATCHES_AUTOTUNE))) return HGT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    {
        std::vector<hgt_graph*> gs;
        for (uint32_t i = 0; i < n; i++) {
            if (!bs[i].graph || bs[i].graph->device != bs[0].graph->device) return HGT_EINVAL;
            gs.push_back(bs[i].graph);
        }
        std::sort(gs.begin(), gs.end());
        if (std::adjacent_find(gs.begin(), gs.end()) != gs.end()) return HGT_EINVAL;
    }
    std::vector<Pending> P(n);
    bool any = false;
    for (uint32_t i = 0; i < n; i++) {
        hgt_batch& b = bs[i];
        b.status = HGT_OK;
        P[i].g = b.graph;
        P[i].out_ids = b.out_ins_ids;
        P[i].rc = 1;  // nothing to apply
        if (b.graph->poisoned) {
            P[i].rc = HGT_EPOISONED;
            continue;
        }
        if (b.n_del == 0 && b.n_ins == 0) continue;
        P[i].rc = plan_begin(P[i], b.del_ids, b.n_del, b.ins_offsets, b.ins_members, b.n_ins_members, b.ins_ts,
                             b.n_ins, s);
        if (P[i].rc == HGT_OK) any = true;
    }
    if (any) HIP_OK(hipStreamSynchronize(s));
    std::vector<Pending*> act;
    for (uint32_t i = 0; i < n; i++) {
        if (P[i].rc != HGT_OK) continue;
        P[i].rc = plan_end(P[i], s);
        if (P[i].rc == HGT_OK) act.push_back(&P[i]);
    }
    if (!act.empty()) {
        hgt_graph* owner = act[0]->g;
        const bool graph = flags & HGT_BATCHES_GRAPH;
        int rc;
        if (flags & HGT_BATCHES_AUTOTUNE) {
            Tuner& T = tuner();
            std::lock_guard<std::mutex> lk(T.mu);
            tune_load(T);
            tune_harvest(T, false);
            const uint64_t key = tune_key(act, owner->n_cu);
            const int choice = tune_pick(T, key);
            const bool timed = T.tab[key].pick < 0;
            Tuner::Open o{key, choice, nullptr, nullptr};
            if (timed && (hipEventCreate(&o.a) != hipSuccess || hipEventCreate(&o.b) != hipSuccess)) {
                (void)hipGetLastError();
                if (o.a) (void)hipEventDestroy(o.a);
                o.a = o.b = nullptr;
            }
            // the first event after the wait for the context's previous round
            t_tune = &kTune[choice];
            t_tune_ev[0] = o.a;
            t_tune_ev[1] = o.b;
            rc = apply_planned(owner, act, s, graph);
            t_tune = nullptr;
            t_tune_ev[0] = t_tune_ev[1] = nullptr;
            if (o.a && rc == HGT_OK) {
                T.open.push_back(o);
            } else if (o.a) {
                (void)hipEventDestroy(o.a);
                (void)hipEventDestroy(o.b);
            }
        } else {
            rc = apply_planned(owner, act, s, graph);
        }
        if (rc)
            for (Pending* p : act) p->rc = rc;
    }
    int first = HGT_OK;
    for (uint32_t i = 0; i < n; i++) {
        int rc = P[i].rc == 1 ? HGT_OK : P[i].rc;
        bs[i].status = rc;
        set_sticky(bs[i].graph, rc);
        if (rc && first == HGT_OK) first = rc;
    }
    return first;
}

}  // namespace

int hgt_apply_batches(hgt_batch* bs, uint32_t n, void* stream) { return apply_batches(bs, n, stream, 0); }

int hgt_apply_batches_ex(hgt_batch* bs, uint32_t n, void* stream, uint32_t flags) {
    return apply_batches(bs, n, stream, flags);
}

int hgt_tune_flush(uint32_t* n_settled) {
    Tuner& T = tuner();
    std::lock_guard<std::mutex> lk(T.mu);
    tune_load(T);
    tune_harvest(T, true);
    if (n_settled) {
        uint32_t k = 0;
        for (auto& kv : T.tab) k += kv.second.pick >= 0;
        *n_settled = k;
    }
    return HGT_OK;
}

int hgt_sync(hgt_graph* g, int* status) {
    if (!g) return HGT_EINVAL;
    if (hipStreamSynchronize(g->last_stream) != hipSuccess) {
        (void)hipGetLastError();
        if (status) *status = HGT_EDEVICE;
        return HGT_EDEVICE;
    }
    if (status) *status = g->poisoned ? HGT_EPOISONED : g->sticky;
    return HGT_OK;
}

int hgt_triad_counts(hgt_graph* g, int type, int64_t window, uint64_t* out_host, uint32_t n_out) {
    if (!g || !out_host) return HGT_EINVAL;
    if (g->poisoned) return HGT_EPOISONED;
    int off, n;
    switch (type) {
        case HGT_TRIAD_HYPEREDGE: off = CNT_HE; n = 30; break;
        case HGT_TRIAD_INCIDENT_VERTEX: off = CNT_IV; n = 3; break;
        case HGT_TRIAD_TEMPORAL: off = CNT_TMP; n = 96; break;
        default: return HGT_EINVAL;
    }
    if (n_out < (uint32_t)n) return HGT_EINVAL;
    if (!(g->track_mask & (1u << type))) return HGT_ENOTTRACKED;
    if (type == HGT_TRIAD_TEMPORAL ? window != g->window : window != 0) return HGT_ENOTTRACKED;
    HIP_OK(hipMemcpyAsync(out_host, g->counts.as<uint64_t>() + off, n * 8, hipMemcpyDeviceToHost, g->last_stream));
    HIP_OK(hipStreamSynchronize(g->last_stream));
    return HGT_OK;
}

int hgt_destroy(hgt_graph* g) {
    if (!g) return HGT_EINVAL;
    (void)hipStreamSynchronize(g->last_stream);
    destroy_graph(g);
    return HGT_OK;
}

int hgt_compact(hgt_graph* g, void* stream) {
    if (!g) return HGT_EINVAL;
    if (g->poisoned) return HGT_EPOISONED;
    hipStream_t s = (hipStream_t)stream;
    int rc = compact_pools(g, s);
    if (!rc) g->last_stream = s;
    return rc;
}

int hgt_get_info(hgt_graph* g, hgt_info* o) {
    if (!g || !o) return HGT_EINVAL;
    HIP_OK(hipStreamSynchronize(g->last_stream));
    o->n_vertices = g->st.n_vertices;
    o->track_mask = g->track_mask;
    o->next_id = g->next_id;
    o->n_live = g->n_live;
    o->n_incidences = g->n_inc;
    o->edge_capacity = g->st.id_cap;
    o->h2v_pool_words = g->h2v.bytes / 4;
    o->h2v_used_words = g->h_bump;
    o->v2h_pool_words = g->v2h.bytes / 4;
    o->v2h_used_words = g->v_bump;
    o->temporal_window = g->window;
    o->batches = g->batches;
    o->compactions = g->compactions;
    o->graph_launches = g->graph_launches;
    return HGT_OK;
}

int hgt_profile(hgt_graph* g, int enable) {
    if (!g) return HGT_EINVAL;
    HIP_OK(hipStreamSynchronize(g->last_stream));
    if (ensure(g->stats, ST_N * 8)) return HGT_ENOMEM;
    HIP_OK(hipMemset(g->stats.p, 0, ST_N * 8));
    g->recs.clear();
    g->ev_used = 0;
    g->store_bytes = 0;
    g->prof = enable != 0;
    g->prof_phases = enable >= 2;
    return HGT_OK;
}

int hgt_profile_read(hgt_graph* g, hgt_kernel_time* out, uint32_t n_max, uint32_t* n_out) {
    if (!g || (!out && n_max)) return HGT_EINVAL;
    HIP_OK(hipStreamSynchronize(g->last_stream));
    uint64_t st[ST_N] = {0};
    if (g->stats.p) HIP_OK(hipMemcpy(st, g->stats.p, ST_N * 8, hipMemcpyDeviceToHost));
    hgt_kernel_time rows[PK_N];
    static_assert(PK_N <= 16, "profile rows");
    std::memset(rows, 0, sizeof rows);
    for (int k = 0; k < PK_N; k++) std::snprintf(rows[k].name, sizeof rows[k].name, "%s", kProfNames[k]);
    for (auto& r : g->recs) {
        float ms = 0;
        HIP_OK(hipEventElapsedTime(&ms, r.a, r.b));
        rows[r.kind].launches++;
        rows[r.kind].total_ms += ms;
    }
    rows[PK_DELTA_BIG].algo_bytes = st[ST_BYTES_BIG];
    rows[PK_TMP].algo_bytes = st[ST_TMP0 + ST_BYTES_SMALL] + st[ST_TMP0 + ST_BYTES_BIG];
    rows[PK_TMP].events = st[ST_TMP0 + ST_EXPANDED];
    rows[PK_TMP].aux = st[ST_TMP0 + ST_DEFERRED];
    rows[PK_IV_PAIRS].algo_bytes = st[ST_IV_BYTES];
    rows[PK_COMMIT].algo_bytes = g->store_bytes;
    rows[PK_DELTA_BIG].events = st[ST_DEFER0 + 2];
    rows[PK_DELTA_SMALL].algo_bytes = st[ST_HEB0];
    rows[PK_DELTA_MED].algo_bytes = st[ST_HEB0 + 1];
    rows[PK_DELTA_GLOBAL].algo_bytes = st[ST_HEB0 + 2];
    rows[PK_DELTA_SMALL].events = st[ST_DEFER0];
    rows[PK_DELTA_SMALL].aux = st[ST_DEFER0 + 1];
    uint32_t n = std::min<uint32_t>(n_max, PK_N);
    for (uint32_t i = 0; i < n; i++) out[i] = rows[i];
    if (n_out) *n_out = PK_N;
    return HGT_OK;
}

int hgt_profile_counters(hgt_graph* g, uint64_t* out, uint32_t n_max, uint32_t* n_out) {
    if (!g || (!out && n_max)) return HGT_EINVAL;
    HIP_OK(hipStreamSynchronize(g->last_stream));
    uint64_t st[ST_N] = {0};
    if (g->stats.p) HIP_OK(hipMemcpy(st, g->stats.p, ST_N * 8, hipMemcpyDeviceToHost));
    uint32_t n = std::min<uint32_t>(n_max, ST_N);
    for (uint32_t i = 0; i < n; i++) out[i] = st[i];
    if (n_out) *n_out = ST_N;
    return HGT_OK;
}

int hgt_export_h2v(hgt_graph* g, uint64_t* offsets_host, uint32_t* members_host, uint8_t* live_host) {
    if (!g || !offsets_host || !members_host || !live_host) return HGT_EINVAL;
    if (g->poisoned) return HGT_EPOISONED;
    hipStream_t s = g->last_stream;
    HIP_OK(hipStreamSynchronize(s));
    uint64_t n = g->next_id;
    std::vector<uint64_t> off(n), bm((n + 63) / 64 + 1);
    std::vector<uint32_t> len(n), pool(g->h_bump);
    if (n) {
        HIP_OK(hipMemcpy(off.data(), g->h_off.p, n * 8, hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(len.data(), g->h_len.p, n * 4, hipMemcpyDeviceToHost));
        HIP_OK(hipMemcpy(bm.data(), g->free_bm.p, ((n + 63) / 64) * 8, hipMemcpyDeviceToHost));
    }
    if (g->h_bump) HIP_OK(hipMemcpy(pool.data(), g->h2v.p, g->h_bump * 4, hipMemcpyDeviceToHost));
    uint64_t k = 0;
    for (uint64_t i = 0; i < n; i++) {
        bool free_ = (bm[i >> 6] >> (i & 63)) & 1;
        live_host[i] = free_ ? 0 : 1;
        offsets_host[i] = k;
        if (!free_) {
            if (off[i] + len[i] > g->h_bump) return HGT_EDEVICE;
            std::memcpy(members_host + k, pool.data() + off[i], len[i] * 4);
            k += len[i];
        }
    }
    offsets_host[n] = k;
    return HGT_OK;
}

int hgt_export_v2h(hgt_graph* g, uint64_t* offsets_host, uint32_t* members_host) {
    if (!g || !offsets_host || !members_host) return HGT_EINVAL;
    if (g->poisoned) return HGT_EPOISONED;
    HIP_OK(hipStreamSynchronize(g->last_stream));
    uint64_t V = g->st.n_vertices;
    std::vector<uint64_t> off(V);
    std::vector<uint32_t> len(V), pool(g->v_bump);
    HIP_OK(hipMemcpy(off.data(), g->v_off.p, V * 8, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(len.data(), g->v_len.p, V * 4, hipMemcpyDeviceToHost));
    if (g->v_bump) HIP_OK(hipMemcpy(pool.data(), g->v2h.p, g->v_bump * 4, hipMemcpyDeviceToHost));
    uint64_t k = 0;
    for (uint64_t v = 0; v < V; v++) {
        offsets_host[v] = k;
        if (len[v]) {
            if (off[v] + len[v] > g->v_bump) return HGT_EDEVICE;
            std::memcpy(members_host + k, pool.data() + off[v], len[v] * 4);
            k += len[v];
        }
    }
    offsets_host[V] = k;
    return HGT_OK;
}

}  // extern "C"

// ===========================================================================
// Snapshot and restore: a host copy of a graph's whole state, in the byte
// form that include/hgt.h documents, and the way back into a graph.
// ===========================================================================
struct hgt_snap {
    std::vector<uint64_t> words;  // header and sections, 8-byte aligned
};

namespace {

constexpr char kSnapMagic[8] = {'H', 'G', 'T', 'S', 'N', 'A', 'P', '1'};
constexpr uint32_t kSnapVersion = 1;

struct SnapHeader {
    char magic[8];
    uint32_t version, track_mask, n_vertices, n_counts;
    int64_t window;
    uint64_t next_id, h_bump, v_bump, next_seq, n_live, n_inc;
    int64_t last_ts;
    uint64_t payload_bytes, checksum;
    uint8_t pad[24];
};
static_assert(sizeof(SnapHeader) == 128, "the snapshot header is 128 bytes");

enum SnapSec { SS_COUNTS, SS_H_OFF, SS_H_LEN, SS_H_CAP, SS_H_SEQ, SS_H_TS, SS_FREE_BM, SS_H2V, SS_HIST, SS_V_OFF,
               SS_V_LEN, SS_V_CAP, SS_V2H, SS_V2H_TS, SS_N };

// Byte offset (from the start of the payload) and unpadded size of each section.
struct SnapLayout {
    uint64_t off[SS_N], bytes[SS_N], total;
};

SnapLayout snap_layout(uint32_t track, uint64_t V, uint64_t next_id, uint64_t hb, uint64_t vb) {
    const bool tmp = track & (1u << HGT_TRIAD_TEMPORAL), he = track & (1u << HGT_TRIAD_HYPEREDGE);
    const uint64_t b[SS_N] = {CNT_N * 8ull, next_id * 8, next_id * 4, next_id * 4, next_id * 8, tmp ? next_id * 8 : 0,
                              (next_id + 63) / 64 * 8, hb * 4, he ? hb * 8 : 0, V * 8, V * 4, V * 4, vb * 4,
                              tmp ? vb * 8 : 0};
    SnapLayout L;
    uint64_t o = 0;
    for (int i = 0; i < SS_N; i++) {
        L.off[i] = o;
        L.bytes[i] = b[i];
        o += (b[i] + 7) & ~7ull;
    }
    L.total = o;
    return L;
}

// FNV-1a applied to 64-bit words
uint64_t snap_checksum(const uint64_t* w, uint64_t n) {
    uint64_t h = 0xcbf29ce484222325ull;
    for (uint64_t i = 0; i < n; i++) h = (h ^ w[i]) * 0x100000001b3ull;
    return h;
}

template <class T> const T* snap_sec(const hgt_snap* s, const SnapLayout& L, int sec) {
    return (const T*)((const char*)s->words.data() + sizeof(SnapHeader) + L.off[sec]);
}

// The structural checks of a snapshot read from bytes (see hgt_snap_load).
bool snap_consistent(const hgt_snap* s) {
    const SnapHeader& H = *(const SnapHeader*)s->words.data();
    const SnapLayout L = snap_layout(H.track_mask, H.n_vertices, H.next_id, H.h_bump, H.v_bump);
    const bool tmp = H.track_mask & (1u << HGT_TRIAD_TEMPORAL);
    const uint64_t n = H.next_id, V = H.n_vertices;
    const uint64_t* h_off = snap_sec<uint64_t>(s, L, SS_H_OFF);
    const uint32_t* h_len = snap_sec<uint32_t>(s, L, SS_H_LEN);
    const uint32_t* h_cap = snap_sec<uint32_t>(s, L, SS_H_CAP);
    const uint64_t* h_seq = snap_sec<uint64_t>(s, L, SS_H_SEQ);
    const int64_t* h_ts = tmp ? snap_sec<int64_t>(s, L, SS_H_TS) : nullptr;
    const uint64_t* bm = snap_sec<uint64_t>(s, L, SS_FREE_BM);
    const uint32_t* h2v = snap_sec<uint32_t>(s, L, SS_H2V);
    const uint64_t* v_off = snap_sec<uint64_t>(s, L, SS_V_OFF);
    const uint32_t* v_len = snap_sec<uint32_t>(s, L, SS_V_LEN);
    const uint32_t* v_cap = snap_sec<uint32_t>(s, L, SS_V_CAP);
    const uint32_t* v2h = snap_sec<uint32_t>(s, L, SS_V2H);
    const int64_t* v2h_ts = tmp ? snap_sec<int64_t>(s, L, SS_V2H_TS) : nullptr;
    auto is_free = [&](uint64_t id) { return (bm[id >> 6] >> (id & 63)) & 1ull; };
    if (n & 63)
        if (bm[n >> 6] >> (n & 63)) return false;  // IDs at or above next_id are not free
    uint64_t live = 0, inc = 0;
    for (uint64_t id = 0; id < n; id++) {
        if (h_cap[id] && (h_off[id] > H.h_bump || h_cap[id] > H.h_bump - h_off[id])) return false;
        if (is_free(id)) continue;
        const uint32_t len = h_len[id];
        if (len < 1 || len > HGT_MAX_CARD || len > h_cap[id] || h_seq[id] >= H.next_seq) return false;
        if (tmp && h_ts[id] > H.last_ts) return false;
        const uint32_t* row = h2v + h_off[id];
        for (uint32_t k = 0; k < len; k++)
            if (row[k] >= V || (k && row[k] <= row[k - 1])) return false;
        live++;
        inc += len;
    }
    if (live != H.n_live || inc != H.n_inc) return false;
    uint64_t inc_v = 0;
    for (uint64_t v = 0; v < V; v++) {
        const uint32_t len = v_len[v];
        if (v_cap[v] && (v_off[v] > H.v_bump || v_cap[v] > H.v_bump - v_off[v])) return false;
        if (len > v_cap[v]) return false;
        for (uint32_t k = 0; k < len; k++) {
            const uint64_t w = v_off[v] + k;
            const uint32_t id = v2h[w];
            if (id >= n || is_free(id) || (k && id <= v2h[w - 1])) return false;
            if (tmp && v2h_ts[w] != h_ts[id]) return false;
        }
        inc_v += len;
    }
    if (inc_v != inc) return false;
    // every incidence of the h2v map is in the v2h map (equal totals and
    // duplicate-free lists make the two maps equal)
    for (uint64_t id = 0; id < n; id++) {
        if (is_free(id)) continue;
        const uint32_t* row = h2v + h_off[id];
        for (uint32_t k = 0; k < h_len[id]; k++) {
            if (!v_len[row[k]]) return false;
            const uint32_t* a = v2h + v_off[row[k]];
            const uint32_t* e = a + v_len[row[k]];
            const uint32_t* f = std::lower_bound(a, e, (uint32_t)id);
            if (f == e || *f != id) return false;
        }
    }
    return true;
}

}  // namespace

extern "C" {

int hgt_snapshot(hgt_graph* g, hgt_snap** out, void* stream) {
    if (!g || !out) return HGT_EINVAL;
    *out = nullptr;
    if (g->poisoned) return HGT_EPOISONED;
    hipStream_t s = (hipStream_t)stream;
    HIP_OK(hipStreamSynchronize(g->last_stream));
    DevScalars sc{};
    HIP_OK(hipMemcpyAsync(&sc, g->scal.p, sizeof sc, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (sc.next_id != g->next_id || sc.h_bump != g->h_bump || sc.v_bump != g->v_bump || sc.n_live != g->n_live ||
        sc.n_inc != g->n_inc || sc.next_seq != g->next_seq)
        return HGT_EDEVICE;  // device scalars and host mirrors disagree
    const uint64_t n = g->next_id, V = g->st.n_vertices;
    const SnapLayout L = snap_layout(g->track_mask, V, n, g->h_bump, g->v_bump);
    hgt_snap* snap = new (std::nothrow) hgt_snap();
    if (!snap) return HGT_ENOMEM;
    try {
        snap->words.assign((sizeof(SnapHeader) + L.total) / 8, 0);
    } catch (...) {
        delete snap;
        return HGT_ENOMEM;
    }
    SnapHeader& H = *(SnapHeader*)snap->words.data();
    std::memcpy(H.magic, kSnapMagic, 8);
    H.version = kSnapVersion;
    H.track_mask = g->track_mask;
    H.n_vertices = (uint32_t)V;
    H.n_counts = CNT_N;
    H.window = g->window;
    H.next_id = n;
    H.h_bump = g->h_bump;
    H.v_bump = g->v_bump;
    H.next_seq = g->next_seq;
    H.n_live = g->n_live;
    H.n_inc = g->n_inc;
    H.last_ts = sc.last_ts;
    H.payload_bytes = L.total;
    const void* src[SS_N] = {g->counts.p, g->h_off.p, g->h_len.p, g->h_cap.p, g->h_seq.p, g->h_ts.p, g->free_bm.p,
                             g->h2v.p, g->hpool.p, g->v_off.p, g->v_len.p, g->v_cap.p, g->v2h.p, g->v2h_ts.p};
    char* pay = (char*)snap->words.data() + sizeof(SnapHeader);
    int rc = HGT_OK;
    for (int i = 0; i < SS_N && rc == HGT_OK; i++)
        if (L.bytes[i] && hip_failed(hipMemcpyAsync(pay + L.off[i], src[i], L.bytes[i], hipMemcpyDeviceToHost, s),
                                     "snapshot copy", __LINE__))
            rc = HGT_EDEVICE;
    if (hip_failed(hipStreamSynchronize(s), "snapshot sync", __LINE__)) rc = HGT_EDEVICE;
    if (rc) {
        delete snap;
        return rc;
    }
    H.checksum = snap_checksum((const uint64_t*)pay, L.total / 8);
    *out = snap;
    return HGT_OK;
}

int hgt_restore(hgt_graph* g, const hgt_snap* snap, void* stream) {
    if (!g || !snap || snap->words.size() < sizeof(SnapHeader) / 8) return HGT_EINVAL;
    const SnapHeader& H = *(const SnapHeader*)snap->words.data();
    if (H.n_vertices != g->st.n_vertices || H.track_mask != g->track_mask || H.window != g->window)
        return HGT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const bool tmp = g->track_mask & (1u << HGT_TRIAD_TEMPORAL), he = g->track_mask & (1u << HGT_TRIAD_HYPEREDGE);
    const uint64_t n = H.next_id, V = H.n_vertices;
    const SnapLayout L = snap_layout(H.track_mask, V, n, H.h_bump, H.v_bump);
    if (hip_failed(hipStreamSynchronize(g->last_stream), "restore wait", __LINE__)) return HGT_EDEVICE;
    // room first (the ID arrays keep their contents when they grow; the pools
    // are replaced only once every new one has been allocated)
    int rc = ensure_id_cap(g, n, s);
    if (rc) return rc;
    const uint64_t h2v_b = std::max<uint64_t>(H.h_bump * 4, g->h2v.bytes);
    const uint64_t v2h_b = std::max<uint64_t>(H.v_bump * 4, g->v2h.bytes);
    DevBuf nb[4];  // h2v, histograms, v2h, v2h timestamps
    DevBuf* cur[4] = {&g->h2v, &g->hpool, &g->v2h, &g->v2h_ts};
    const uint64_t want[4] = {h2v_b, he ? 2 * h2v_b : 0, v2h_b, tmp ? 2 * v2h_b : 0};
    for (int i = 0; i < 4 && rc == HGT_OK; i++)
        if (want[i] > cur[i]->bytes) rc = dev_alloc(nb[i], (want[i] + 4095) & ~(size_t)4095);
    if (rc) {
        for (DevBuf& b : nb) dev_free(b);
        return rc;
    }
    for (int i = 0; i < 4; i++)
        if (nb[i].p) {
            dev_free(*cur[i]);
            *cur[i] = nb[i];
        }
    refresh_view(g);
    // from here a failure leaves the graph part-way
    g->poisoned = true;
    g->sticky = HGT_EPOISONED;
    void* dst[SS_N] = {g->counts.p, g->h_off.p, g->h_len.p, g->h_cap.p, g->h_seq.p, g->h_ts.p, g->free_bm.p,
                       g->h2v.p, g->hpool.p, g->v_off.p, g->v_len.p, g->v_cap.p, g->v2h.p, g->v2h_ts.p};
    const char* pay = (const char*)snap->words.data() + sizeof(SnapHeader);
    for (int i = 0; i < SS_N; i++)
        if (L.bytes[i]) HIP_OK(hipMemcpyAsync(dst[i], pay + L.off[i], L.bytes[i], hipMemcpyHostToDevice, s));
    // IDs from next_id up are fresh: length and capacity 0, not free
    const uint64_t cap = g->st.id_cap, bm_words = (n + 63) / 64;
    HIP_OK(hipMemsetAsync(g->h_len.as<uint32_t>() + n, 0, (cap - n) * 4, s));
    HIP_OK(hipMemsetAsync(g->h_cap.as<uint32_t>() + n, 0, (cap - n) * 4, s));
    HIP_OK(hipMemsetAsync(g->free_bm.as<uint64_t>() + bm_words, 0, (cap / 64 - bm_words) * 8, s));
    HIP_OK(hipMemsetAsync(g->counts.as<uint64_t>() + CNT_N, 0, (ACC_N - CNT_N) * 8, s));
    DevScalars sc{};
    sc.status = HGT_OK;
    sc.next_id = n;
    sc.h_bump = H.h_bump;
    sc.v_bump = H.v_bump;
    sc.next_seq = H.next_seq;
    sc.last_ts = H.last_ts;
    sc.n_live = H.n_live;
    sc.n_inc = H.n_inc;
    HIP_OK(hipMemcpyAsync(g->scal.p, &sc, sizeof sc, hipMemcpyHostToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
    g->next_id = n;
    g->h_bump = H.h_bump;
    g->v_bump = H.v_bump;
    g->next_seq = H.next_seq;
    g->n_live = H.n_live;
    g->n_inc = H.n_inc;
    g->last_stream = s;
    g->poisoned = false;
    g->sticky = HGT_OK;
    return HGT_OK;
}

int hgt_snap_bytes(const hgt_snap* snap, void* out_host, uint64_t cap, uint64_t* n_bytes) {
    if (!snap || !n_bytes) return HGT_EINVAL;
    const uint64_t nb = snap->words.size() * 8;
    *n_bytes = nb;
    if (out_host) {
        if (cap < nb) return HGT_EINVAL;
        std::memcpy(out_host, snap->words.data(), nb);
    }
    return HGT_OK;
}

int hgt_snap_load(const void* bytes, uint64_t n_bytes, hgt_snap** out) {
    if (!bytes || !out) return HGT_EINVAL;
    *out = nullptr;
    if (n_bytes < sizeof(SnapHeader) || n_bytes % 8) return HGT_EINVAL;
    SnapHeader H;
    std::memcpy(&H, bytes, sizeof H);
    if (std::memcmp(H.magic, kSnapMagic, 8) || H.version != kSnapVersion || (H.track_mask & ~7u) ||
        H.n_vertices == 0 || H.n_vertices > 0x7fffffffu || H.n_counts != CNT_N || H.window < 0 ||
        H.next_id > 0xfffffff0ull || H.h_bump > (1ull << 40) || H.v_bump > (1ull << 40))
        return HGT_EINVAL;
    const SnapLayout L = snap_layout(H.track_mask, H.n_vertices, H.next_id, H.h_bump, H.v_bump);
    if (H.payload_bytes != L.total || n_bytes != sizeof(SnapHeader) + L.total) return HGT_EINVAL;
    hgt_snap* snap = new (std::nothrow) hgt_snap();
    if (!snap) return HGT_ENOMEM;
    try {
        snap->words.resize(n_bytes / 8);
    } catch (...) {
        delete snap;
        return HGT_ENOMEM;
    }
    std::memcpy(snap->words.data(), bytes, n_bytes);
    if (snap_checksum(snap->words.data() + sizeof(SnapHeader) / 8, L.total / 8) != H.checksum ||
        !snap_consistent(snap)) {
        delete snap;
        return HGT_EINVAL;
    }
    *out = snap;
    return HGT_OK;
}

int hgt_snap_free(hgt_snap* snap) {
    if (!snap) return HGT_EINVAL;
    delete snap;
    return HGT_OK;
}

}  // extern "C"
