// server.hip -- the served form: a request loop over many resident hypergraphs
// (tenants) with footprint-based admission and continuous batching.
//
// Clients submit host batches.  A server thread takes the queued requests in
// arrival order, admits those whose tenant is idle and whose buffers and
// footprint fit, stages their inputs into a device arena, and applies them as
// one round through hgt_apply_batches (one planning wait for the whole round,
// shared triad launches).  Up to four rounds are in flight, each on a stream
// of its own with its own triad-phase scratch, so a round is planned and its
// triad phases run while earlier rounds are still on the GPU; completion is
// observed through an event per round, in any order.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace {

uint64_t now_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

constexpr uint64_t kAlign = 256;
inline uint64_t align_up(uint64_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// First-fit allocator over [0, cap) with coalescing frees (host bookkeeping of
// the device arena and its pinned mirror).
struct RangeAlloc {
    std::map<uint64_t, uint64_t> free_;  // offset -> size
    uint64_t cap = 0, used = 0;
    void init(uint64_t c) {
        cap = c;
        used = 0;
        free_.clear();
        free_[0] = c;
    }
    bool alloc(uint64_t n, uint64_t* off) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            uint64_t rest = it->second - n;
            uint64_t at = it->first + n;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used += n;
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t n) {
        used -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct Request {
    uint64_t ticket = 0;
    uint32_t tenant = 0;
    hgt_graph* graph = nullptr;  // the tenant's graph, copied at admission under the lock
    std::vector<uint32_t> del, mem;
    std::vector<uint64_t> off;
    std::vector<int64_t> ts;
    uint64_t n_ins = 0;
    uint32_t* out_ids_host = nullptr;
    uint64_t footprint = 0;
    // arena range: del | off | mem | ts | ids | counts (256-byte aligned parts)
    uint64_t a_off = 0, a_len = 0;
    uint64_t o_del = 0, o_off = 0, o_mem = 0, o_ts = 0, o_ids = 0, o_cnt = 0;
    bool done = false;
    hgt_result res{};
};

struct Round {
    std::vector<Request*> reqs;
    hipEvent_t ev = nullptr;
    int stream = 0;
    uint64_t id = 0;
};

}  // namespace

struct hgt_server {
    hgt_server_desc desc{};
    int device = 0;
    static constexpr int kStreams = 4;      // most rounds in flight
    hipStream_t streams[kStreams] = {};
    PhaseCtx* ctx[kStreams] = {};           // phase scratch of the round on each stream
    bool stream_busy[kStreams] = {};
    void* d_arena = nullptr;   // device
    char* h_arena = nullptr;   // pinned mirror
    RangeAlloc arena;
    std::vector<hgt_graph*> tenants;
    std::vector<uint8_t> busy;             // a request of the tenant is in a round
    std::vector<std::deque<Request*>> per_tenant;  // queued, FIFO per tenant
    std::deque<Request*> queue;            // queued, arrival order
    std::unordered_map<uint64_t, Request*> by_ticket;
    std::vector<Round*> inflight;
    std::vector<hipEvent_t> ev_pool;
    uint64_t next_ticket = 1, footprint_in_use = 0, rounds = 0, done_count = 0, running = 0;
    uint64_t max_round_seen = 0, max_inflight_seen = 0;
    bool stop = false;
    int fatal = HGT_OK;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
};

namespace {

// Footprint estimate of a request: its arena bytes plus the batch scratch the
// library sizes from the batch (pair keys of the store update, incident-vertex
// pair keys, batch-neighbour entries), from the request sizes and the tenant's
// mean cardinality and degree.
uint64_t footprint_of(const Request& r, const HgtSizes& z) {
    const double card = z.n_live ? (double)z.n_inc / (double)z.n_live : 1.0;
    const double deg = z.n_vertices ? (double)z.n_inc / (double)z.n_vertices : 1.0;
    const double n_del = (double)r.del.size();
    double pairs = (double)r.mem.size() + n_del * card;                 // (v, h) pairs
    double iv = 0;
    if (z.track_mask & (1u << HGT_TRIAD_INCIDENT_VERTEX)) {
        for (uint64_t j = 0; j < r.n_ins; j++) {
            double d = (double)(r.off[j + 1] - r.off[j]);
            iv += d * (d - 1) / 2;
        }
        iv += n_del * card * (card - 1) / 2;
    }
    double entries = (double)(r.n_ins + r.del.size()) * card * deg;   // neighbour entries
    double scratch = 110.0 * pairs + 40.0 * iv + 24.0 * entries + 64.0 * (double)(r.n_ins + r.del.size());
    return r.a_len + (uint64_t)scratch;
}

void fail_all_locked(hgt_server* s, int code);

// Stages the round's inputs, applies it, queues the read-back of IDs and
// counts and records the round's event.  Called without the lock: it reads
// only the round's requests (their graph pointers were copied at admission),
// never the tenant table, which hgt_server_add_tenant may grow meanwhile.
int launch_round(hgt_server* s, Round* R) {
    hipStream_t st = s->streams[R->stream];
    std::vector<hgt_batch> bs(R->reqs.size());
    char* H = s->h_arena;
    char* D = (char*)s->d_arena;
    for (size_t i = 0; i < R->reqs.size(); i++) {
        Request* q = R->reqs[i];
        // host copies -> pinned mirror -> device arena
        if (!q->del.empty()) std::memcpy(H + q->o_del, q->del.data(), q->del.size() * 4);
        if (q->n_ins) {
            std::memcpy(H + q->o_off, q->off.data(), (q->n_ins + 1) * 8);
            if (!q->mem.empty()) std::memcpy(H + q->o_mem, q->mem.data(), q->mem.size() * 4);
            if (!q->ts.empty()) std::memcpy(H + q->o_ts, q->ts.data(), q->ts.size() * 8);
        }
        uint64_t in_len = q->o_ids - q->o_del;
        if (in_len && hipMemcpyAsync(D + q->o_del, H + q->o_del, in_len, hipMemcpyHostToDevice, st) != hipSuccess)
            return HGT_EDEVICE;
        hgt_batch& b = bs[i];
        std::memset(&b, 0, sizeof b);
        b.graph = q->graph;
        b.del_ids = q->del.empty() ? nullptr : (const uint32_t*)(D + q->o_del);
        b.n_del = q->del.size();
        b.ins_offsets = q->n_ins ? (const uint64_t*)(D + q->o_off) : nullptr;
        b.ins_members = q->mem.empty() ? nullptr : (const uint32_t*)(D + q->o_mem);
        b.n_ins_members = q->mem.size();
        b.ins_ts = q->ts.empty() ? nullptr : (const int64_t*)(D + q->o_ts);
        b.n_ins = q->n_ins;
        b.out_ins_ids = q->n_ins ? (uint32_t*)(D + q->o_ids) : nullptr;
    }
    // the round's own phase scratch: rounds on the two streams overlap on the device
    hgt_use_phase_ctx(s->ctx[R->stream]);
    (void)hgt_apply_batches_ex(bs.data(), (uint32_t)bs.size(), st, s->desc.launch_flags);
    hgt_use_phase_ctx(nullptr);
    for (size_t i = 0; i < R->reqs.size(); i++) {
        Request* q = R->reqs[i];
        q->res.status = bs[i].status;
        if (q->n_ins && bs[i].status == HGT_OK &&
            hipMemcpyAsync(H + q->o_ids, D + q->o_ids, q->n_ins * 4, hipMemcpyDeviceToHost, st) != hipSuccess)
            return HGT_EDEVICE;
        int rc = hgt_counts_async(q->graph, (uint64_t*)(H + q->o_cnt), st);
        if (rc) return rc;
    }
    if (hipEventRecord(R->ev, st) != hipSuccess) return HGT_EDEVICE;
    return HGT_OK;
}

// Under the lock: results of a completed round, then its resources.
void complete_round_locked(hgt_server* s, Round* R) {
    const uint64_t t = now_ns();
    for (Request* q : R->reqs) {
        const uint64_t* c = (const uint64_t*)(s->h_arena + q->o_cnt);
        std::memcpy(q->res.he, c, 30 * 8);
        std::memcpy(q->res.iv, c + 30, 3 * 8);
        std::memcpy(q->res.temporal, c + 33, 96 * 8);
        if (q->out_ids_host && q->n_ins && q->res.status == HGT_OK)
            std::memcpy(q->out_ids_host, s->h_arena + q->o_ids, q->n_ins * 4);
        q->res.t_done_ns = t;
        q->res.round = R->id;
        q->res.round_size = (uint32_t)R->reqs.size();
        q->done = true;
        s->arena.release(q->a_off, q->a_len);
        s->footprint_in_use -= q->footprint;
        s->busy[q->tenant] = 0;
        s->running--;
        s->done_count++;
        // drop host copies of the inputs
        std::vector<uint32_t>().swap(q->del);
        std::vector<uint32_t>().swap(q->mem);
        std::vector<uint64_t>().swap(q->off);
        std::vector<int64_t>().swap(q->ts);
    }
    s->ev_pool.push_back(R->ev);
    delete R;
}

// Under the lock: the next round's requests (idle tenants, per-tenant FIFO,
// arrival order across tenants, arena and footprint limits).
Round* admit_locked(hgt_server* s) {
    if (s->queue.empty()) return nullptr;
    Round* R = nullptr;
    std::vector<uint8_t> taken(s->tenants.size(), 0);
    const uint64_t t = now_ns();
    for (auto it = s->queue.begin(); it != s->queue.end();) {
        Request* q = *it;
        const uint32_t tn = q->tenant;
        if (s->busy[tn] || taken[tn] || s->per_tenant[tn].front() != q) {
            taken[tn] = 1;  // later requests of this tenant wait for this one
            ++it;
            continue;
        }
        // the tenant is idle, so its size mirrors are those the request will see
        if (!q->footprint) q->footprint = footprint_of(*q, hgt_sizes(s->tenants[tn]));
        const bool alone = s->footprint_in_use == 0 && (!R || R->reqs.empty());
        if (!alone && s->footprint_in_use + q->footprint > s->desc.hbm_budget_bytes) {
            taken[tn] = 1;
            ++it;
            continue;
        }
        uint64_t off;
        if (!s->arena.alloc(q->a_len, &off)) {
            taken[tn] = 1;
            ++it;
            continue;
        }
        q->a_off = off;
        q->graph = s->tenants[tn];  // launch_round runs without the lock and must not index tenants
        q->o_del += off;
        q->o_off += off;
        q->o_mem += off;
        q->o_ts += off;
        q->o_ids += off;
        q->o_cnt += off;
        if (!R) R = new Round();
        R->reqs.push_back(q);
        q->res.t_admit_ns = t;
        s->footprint_in_use += q->footprint;
        s->busy[tn] = 1;
        taken[tn] = 1;
        s->per_tenant[tn].pop_front();
        it = s->queue.erase(it);
        s->running++;
        if (R->reqs.size() >= s->desc.max_round) break;
        if (s->footprint_in_use > s->desc.hbm_budget_bytes) break;  // a heavy request runs alone
    }
    return R;
}

void fail_all_locked(hgt_server* s, int code) {
    s->fatal = code;
    for (Request* q : s->queue) {
        q->res.status = code;
        q->done = true;
    }
    s->queue.clear();
    for (auto& d : s->per_tenant) d.clear();
}

void worker_main(hgt_server* s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // completed rounds, in any order (their tenants are distinct)
        for (size_t i = 0; i < s->inflight.size();) {
            Round* R = s->inflight[i];
            if (hipEventQuery(R->ev) != hipSuccess) { ++i; continue; }
            s->inflight.erase(s->inflight.begin() + i);
            s->stream_busy[R->stream] = false;
            complete_round_locked(s, R);
            s->cv_done.notify_all();
        }
        if (s->stop && s->queue.empty() && s->inflight.empty()) break;
        Round* R = nullptr;
        if (!s->fatal && s->inflight.size() < s->desc.max_inflight) R = admit_locked(s);
        if (R) {
            if (s->ev_pool.empty()) {
                hipEvent_t e;
                if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                    fail_all_locked(s, HGT_EDEVICE);
                    s->cv_done.notify_all();
                    continue;
                }
                s->ev_pool.push_back(e);
            }
            R->ev = s->ev_pool.back();
            s->ev_pool.pop_back();
            R->stream = 0;  // a stream with no round in flight (there is one: inflight < max_inflight)
            while (s->stream_busy[R->stream]) R->stream++;
            s->stream_busy[R->stream] = true;
            R->id = s->rounds++;
            s->max_round_seen = std::max<uint64_t>(s->max_round_seen, R->reqs.size());
            s->inflight.push_back(R);
            s->max_inflight_seen = std::max<uint64_t>(s->max_inflight_seen, s->inflight.size());
            lk.unlock();
            int rc = launch_round(s, R);
            lk.lock();
            if (rc) {
                // the device state is unknown: fail this round and everything queued
                for (Request* q : R->reqs) q->res.status = rc;
                (void)hipStreamSynchronize(s->streams[R->stream]);
                fail_all_locked(s, rc);
            }
            continue;
        }
        if (!s->inflight.empty()) {
            // wait without the lock until a round completes or 200 us pass; new
            // submissions are taken after that
            std::vector<hipEvent_t> evs;
            for (Round* R : s->inflight) evs.push_back(R->ev);
            lk.unlock();
            auto t_end = std::chrono::steady_clock::now() + std::chrono::microseconds(200);
            bool any = false;
            while (!any && std::chrono::steady_clock::now() < t_end) {
                for (hipEvent_t e : evs)
                    if (hipEventQuery(e) != hipErrorNotReady) any = true;
                if (!any) std::this_thread::yield();
            }
            lk.lock();
            continue;
        }
        s->cv_work.wait(lk);
    }
}

}  // namespace

extern "C" {

int hgt_server_create(const hgt_server_desc* d, hgt_server** out) {
    if (!d || !out) return HGT_EINVAL;
    *out = nullptr;
    if (d->launch_flags & ~(uint32_t)(HGT_BATCHES_GRAPH | HGT_BATCHES_AUTOTUNE)) return HGT_EINVAL;
    hgt_server* s = new (std::nothrow) hgt_server();
    if (!s) return HGT_ENOMEM;
    s->desc = *d;
    if (!s->desc.arena_bytes) s->desc.arena_bytes = 256ull << 20;
    if (!s->desc.max_round) s->desc.max_round = 256;
    if (!s->desc.max_inflight) s->desc.max_inflight = hgt_server::kStreams;
    s->desc.max_inflight = std::min<uint32_t>(s->desc.max_inflight, hgt_server::kStreams);
    s->desc.arena_bytes = align_up(s->desc.arena_bytes);
    int rc = HGT_OK;
    do {
        if (hipGetDevice(&s->device) != hipSuccess) { rc = HGT_EDEVICE; break; }
        for (uint32_t i = 0; i < s->desc.max_inflight && !rc; i++) {
            if (hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking) != hipSuccess) rc = HGT_EDEVICE;
            else if (!(s->ctx[i] = hgt_phase_ctx_create(s->device))) rc = HGT_ENOMEM;
        }
        if (rc) break;
        if (hipMalloc(&s->d_arena, s->desc.arena_bytes) != hipSuccess ||
            hipHostMalloc((void**)&s->h_arena, s->desc.arena_bytes, hipHostMallocDefault) != hipSuccess) {
            rc = HGT_ENOMEM;
            break;
        }
    } while (0);
    if (rc) {
        (void)hipGetLastError();
        if (s->d_arena) (void)hipFree(s->d_arena);
        if (s->h_arena) (void)hipHostFree(s->h_arena);
        for (PhaseCtx* c : s->ctx) hgt_phase_ctx_destroy(c);
        for (hipStream_t st : s->streams)
            if (st) (void)hipStreamDestroy(st);
        delete s;
        return rc;
    }
    s->arena.init(s->desc.arena_bytes);
    s->worker = std::thread(worker_main, s);
    *out = s;
    return HGT_OK;
}

int hgt_server_add_tenant(hgt_server* s, const hgt_build_desc* d, uint32_t* tenant) {
    if (!s || !d || !tenant) return HGT_EINVAL;
    hgt_build_desc b = *d;
    b.stream = s->streams[0];  // queued behind stream 0's rounds (other tenants)
    hgt_graph* g = nullptr;
    int rc = hgt_build(&b, &g);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(s->mu);
    s->tenants.push_back(g);
    s->busy.push_back(0);
    s->per_tenant.emplace_back();
    *tenant = (uint32_t)(s->tenants.size() - 1);
    return HGT_OK;
}

int hgt_server_tenant_graph(hgt_server* s, uint32_t tenant, hgt_graph** out) {
    if (!s || !out) return HGT_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (tenant >= s->tenants.size()) return HGT_EINVAL;
    *out = s->tenants[tenant];
    return HGT_OK;
}

int hgt_server_submit(hgt_server* s, uint32_t tenant, const hgt_request* r, uint64_t* ticket) {
    if (!s || !r || !ticket) return HGT_EINVAL;
    const uint64_t t0 = now_ns();
    if ((r->n_del && !r->del_ids) || (r->n_ins && !r->ins_offsets) || (r->n_ins_members && !r->ins_members))
        return HGT_EINVAL;
    Request* q = new (std::nothrow) Request();
    if (!q) return HGT_ENOMEM;
    q->tenant = tenant;
    q->n_ins = r->n_ins;
    q->out_ids_host = r->out_ins_ids_host;
    q->res.t_submit_ns = t0;
    q->res.tenant = tenant;
    try {
        q->del.assign(r->del_ids, r->del_ids + r->n_del);
        if (r->n_ins) {
            q->off.assign(r->ins_offsets, r->ins_offsets + r->n_ins + 1);
            uint64_t base = q->off[0];
            for (auto& o : q->off) o -= base;  // rows relative to the member buffer
            if (q->off.back() != r->n_ins_members) {
                delete q;
                return HGT_EINVAL;
            }
            q->mem.assign(r->ins_members, r->ins_members + r->n_ins_members);
            if (r->ins_ts) q->ts.assign(r->ins_ts, r->ins_ts + r->n_ins);
        }
    } catch (...) {
        delete q;
        return HGT_ENOMEM;
    }
    // arena layout
    uint64_t o = 0;
    q->o_del = o; o = align_up(o + q->del.size() * 4);
    q->o_off = o; o = align_up(o + (q->n_ins ? (q->n_ins + 1) * 8 : 0));
    q->o_mem = o; o = align_up(o + q->mem.size() * 4);
    q->o_ts = o;  o = align_up(o + q->ts.size() * 8);
    q->o_ids = o; o = align_up(o + q->n_ins * 4);
    q->o_cnt = o; o = align_up(o + HGT_COUNT_WORDS * 8);
    q->a_len = o;
    std::unique_lock<std::mutex> lk(s->mu);
    if (tenant >= s->tenants.size()) {
        delete q;
        return HGT_EINVAL;
    }
    if (q->a_len > s->arena.cap) {
        delete q;
        return HGT_ENOMEM;
    }
    if (s->fatal || s->stop) {
        int rc = s->fatal ? s->fatal : HGT_EINVAL;
        delete q;
        return rc;
    }
    q->ticket = s->next_ticket++;
    s->by_ticket[q->ticket] = q;
    s->queue.push_back(q);
    s->per_tenant[tenant].push_back(q);
    *ticket = q->ticket;
    lk.unlock();
    s->cv_work.notify_one();
    return HGT_OK;
}

int hgt_server_query(hgt_server* s, uint64_t ticket, int* done) {
    if (!s || !done) return HGT_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->by_ticket.find(ticket);
    if (it == s->by_ticket.end()) return HGT_EINVAL;
    *done = it->second->done ? 1 : 0;
    return HGT_OK;
}

int hgt_server_wait(hgt_server* s, uint64_t ticket, hgt_result* out) {
    if (!s) return HGT_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->by_ticket.find(ticket);
    if (it == s->by_ticket.end()) return HGT_EINVAL;
    Request* q = it->second;
    s->cv_done.wait(lk, [&] { return q->done; });
    int rc = q->res.status;
    if (out) *out = q->res;
    s->by_ticket.erase(it);
    delete q;
    return rc;
}

int hgt_server_get_info(hgt_server* s, hgt_server_info* o) {
    if (!s || !o) return HGT_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    o->rounds = s->rounds;
    o->requests_done = s->done_count;
    o->requests_pending = s->queue.size();
    o->requests_running = s->running;
    o->footprint_in_use = s->footprint_in_use;
    o->arena_in_use = s->arena.used;
    o->max_round_size = s->max_round_seen;
    o->max_inflight_seen = s->max_inflight_seen;
    return HGT_OK;
}

int hgt_server_destroy(hgt_server* s) {
    if (!s) return HGT_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (hipStream_t st : s->streams)
        if (st) (void)hipStreamSynchronize(st);
    for (auto& kv : s->by_ticket) delete kv.second;
    for (hgt_graph* g : s->tenants) hgt_destroy(g);
    for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
    for (PhaseCtx* c : s->ctx) hgt_phase_ctx_destroy(c);
    (void)hipFree(s->d_arena);
    (void)hipHostFree(s->h_arena);
    for (hipStream_t st : s->streams)
        if (st) (void)hipStreamDestroy(st);
    delete s;
    return HGT_OK;
}

}  // extern "C"
