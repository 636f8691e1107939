/*
 * hgt.h -- C ABI of the dynamic-hypergraph triad-count library (HIP, gfx950).
 *
 * The library keeps one or more hypergraphs resident in device memory, applies
 * batches of hyperedge deletions and insertions to them and keeps their triad
 * counts up to date incrementally.  It follows the problem statement of the
 * paper (ESCHER, arXiv 2512.21009): updates are batches of hyperedge
 * insertions and deletions (Sec. III-B, "vertical operations"), deletions are
 * applied before insertions (Alg. 3, step 3), counts are maintained as
 * count - count_Del + count_Ins (Alg. 3, step 6), and the supported triad
 * families are hyperedge-based, incident-vertex-based and temporal triads
 * (Sec. II, "Hypergraph Triads").
 *
 * Conventions used by every entry point
 *  - Every function returns an int status: HGT_OK (0) or a negative HGT_E*
 *    code; hgt_status_str() names it.
 *  - "device" pointers point to memory of the GPU the graph lives on (for
 *    example the data_ptr() of a torch tensor); "host" pointers to ordinary
 *    CPU memory.  The library never frees caller memory and never keeps a
 *    caller pointer beyond the call (device inputs are read in stream order;
 *    the caller must not overwrite them before the stream has passed the call).
 *  - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *  - IDs and vertex ids are uint32, CSR offsets uint64, timestamps int64 (any
 *    unit, the same as the temporal window), counts uint64.  Counts are exact
 *    and maintained modulo 2^64 (exact whenever the true count is below 2^64).
 *  - A batch that fails validation is rejected as a whole: graph state and
 *    counts stay as they were, and the error is returned by that call and
 *    again by hgt_sync().
 *  - A batch that fails after validation, once its first mutating kernel may
 *    have been queued (a HIP runtime failure), leaves the graph partly
 *    updated.  The graph is then "poisoned": that call returns
 *    HGT_EPOISONED, hgt_sync() reports it, and every call that reads or
 *    updates the graph returns HGT_EPOISONED until hgt_restore() loads a
 *    snapshot into it (or hgt_destroy() releases it).
 */
#ifndef HGT_H
#define HGT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define HGT_OK 0
#define HGT_EINVAL (-1)      /* bad argument, empty/too large/repeated/out-of-range member list */
#define HGT_ENOENT (-2)      /* a deleted ID is not live */
#define HGT_EDUP (-3)        /* an ID appears twice in one deletion list */
#define HGT_EORDER (-4)      /* temporal insert older than the resident stream, or unsorted batch */
#define HGT_ENOMEM (-5)      /* device memory exhausted */
#define HGT_ENOTTRACKED (-6) /* the triad type (or window) is not maintained by this graph */
#define HGT_EDEVICE (-7)     /* HIP runtime failure (outside a batch the graph is left as it was) */
#define HGT_EPOISONED (-8)   /* a batch failed part-way: restore a snapshot or destroy the graph */

/* ---- triad families (Sec. II) ----------------------------------------- */
/* Hyperedge-based: 30 uint64 classes.  A class is a Venn pattern of three
 * connected hyperedges up to relabelling, indexed by ascending canonical
 * pattern code (bit0 a only, bit1 b only, bit2 c only, bit3 a&b only,
 * bit4 b&c only, bit5 c&a only, bit6 a&b&c; canonical = smallest code over
 * the six labellings).  Codes 64, 65, 72 and 76 (indices 10, 11, 14, 17) need
 * two or three identical vertex sets; the other 26 are the paper's 26 triads. */
#define HGT_TRIAD_HYPEREDGE 0
/* Incident-vertex-based: 3 uint64 = types 1, 2, 3 with hyperedge
 * multiplicity: vertex triples {u,v,w} with one witness hyperedge per pair;
 * type 1 all witnesses equal, type 2 exactly two equal, type 3 all distinct. */
#define HGT_TRIAD_INCIDENT_VERTEX 1
/* Temporal: 96 uint64 classes.  Connected triples ordered by (timestamp,
 * arrival sequence) whose first and last timestamps differ by at most the
 * window; class = Venn pattern in time order, indexed by ascending code. */
#define HGT_TRIAD_TEMPORAL 2

#define HGT_N_HE_CLASSES 30
#define HGT_N_IV_CLASSES 3
#define HGT_N_TEMPORAL_CLASSES 96

/* Largest accepted hyperedge cardinality. */
#define HGT_MAX_CARD 8192

typedef struct hgt_graph hgt_graph;

/* ---- build ------------------------------------------------------------ */
typedef struct {
    uint32_t n_vertices;       /* vertex ids are 0 .. n_vertices-1                          */
    uint64_t n_edges;          /* initial hyperedges; they get IDs 0 .. n_edges-1 in order    */
    const uint64_t* offsets;   /* device [n_edges+1], non-decreasing                           */
    const uint32_t* members;   /* device: row j is members[offsets[j]-offsets[0] ..
                                  offsets[j+1]-offsets[0]), member vertex ids in any order      */
    const int64_t* timestamps; /* device [n_edges] or NULL; required when temporal is tracked  */
    uint32_t track_mask;       /* bit (1 << HGT_TRIAD_*) for every family to maintain          */
    int64_t temporal_window;   /* window of the temporal family (>= 0)                         */
    uint64_t edge_capacity;    /* initial ID capacity, 0 = automatic (grows on demand)          */
    uint64_t pool_words;       /* initial words per incidence pool, 0 = automatic (grows)       */
    void* stream;              /* hipStream_t for the build work                               */
} hgt_build_desc;

/* Copies the hypergraph into the library's device pools (the caller keeps its
 * buffers) and computes the initial counts of every tracked family.  Rows are
 * sets: each must hold 1..HGT_MAX_CARD distinct vertex ids < n_vertices.
 * Initial timestamps may be in any order; their arrival sequence is the input
 * order.  Synchronises `stream`.  On success *out owns the graph. */
int hgt_build(const hgt_build_desc* d, hgt_graph** out);

/* ---- batch update (Alg. 3) -------------------------------------------- */
/* Applies one batch: first deletes the n_del hyperedges del_ids[0..n_del)
 * (device; distinct live IDs; batch order = deletion rank), then inserts the
 * n_ins hyperedges given as device CSR: ins_offsets[0..n_ins] non-decreasing,
 * row j = ins_members[ins_offsets[j]-ins_offsets[0] .. ins_offsets[j+1]-ins_offsets[0])
 * (n_ins_members = ins_offsets[n_ins] - ins_offsets[0] entries, members in any order),
 * with device timestamps ins_ts[0..n_ins) (required iff temporal is tracked;
 * non-decreasing and not older than any timestamp inserted before).
 * ID reuse (Alg. 2, "thread j finds the j-th available node"): with F the
 * ascending list of free IDs including this batch's deletions, the j-th
 * insert gets F[j]; later inserts get fresh consecutive IDs.  The IDs are
 * written to out_ins_ids[0..n_ins) (device, may be NULL).
 * Then every tracked count is updated incrementally.  All work is queued on
 * `stream`; the call waits once for a small validation/allocation summary,
 * so a rejected batch returns its error here and leaves everything unchanged.
 * Pointers may be NULL when the matching count is 0. */
int hgt_apply_batch(hgt_graph* g, const uint32_t* del_ids, uint64_t n_del,
                    const uint64_t* ins_offsets, const uint32_t* ins_members,
                    uint64_t n_ins_members, const int64_t* ins_ts, uint64_t n_ins,
                    uint32_t* out_ins_ids, void* stream);

/* For callers that cannot allocate device memory (serving loops and test
 * harnesses that forbid hipMalloc/hipFree mid-run): hgt_apply_batch with the
 * same arguments, semantics and results, which allocates no device or pinned
 * memory.  Its batch scratch (planning buffers and the triad phases' tables)
 * is carved out of a 256 MiB device array that the library holds on every GPU
 * it runs on until the process ends; on that path the kernels with
 * per-workgroup global tables run fewer workgroups.  Returns HGT_ENOMEM, with
 * the graph unchanged, when the batch's scratch would exceed 256 MiB or the
 * graph would have to grow its ID capacity or incidence pools (build with
 * larger edge_capacity / pool_words, or apply such a batch with
 * hgt_apply_batch first).  The graph's GPU must be the current device.  Every
 * call on a GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams, other threads) race and must be serialised by the caller.  Like
 * hgt_apply_batch it waits once on the host for the batch summary, so it
 * cannot be captured into a HIP graph. */
int hgt_apply_batch_noalloc(hgt_graph* g, const uint32_t* del_ids, uint64_t n_del,
                            const uint64_t* ins_offsets, const uint32_t* ins_members,
                            uint64_t n_ins_members, const int64_t* ins_ts, uint64_t n_ins,
                            uint32_t* out_ins_ids, void* stream);

/* ---- horizontal operations (Sec. III-B) -------------------------------- */
/* Incident-vertex insertions and deletions inside live hyperedges (the
 * paper's "horizontal operations"): op i inserts vertices[i] into hyperedge
 * edge_ids[i] when insert[i] != 0, else deletes it from it (device arrays of
 * n_ops entries, any order).  Every modified hyperedge keeps its ID, its
 * timestamp and its arrival sequence; the counts of every tracked family
 * change as if the modified hyperedges were deleted and their new member sets
 * inserted under the same IDs (Alg. 3 with incident vertices in place of
 * hyperedges).  The batch is rejected whole, with nothing changed, when an ID
 * is not live (HGT_ENOENT), a vertex is out of range, the same (hyperedge,
 * vertex) pair appears twice, a deleted vertex is not a member, an inserted
 * one already is, or a hyperedge would be left empty or above HGT_MAX_CARD
 * members (HGT_EINVAL).  Waits twice on the host (the ops' summary, then the
 * batch's). */
int hgt_apply_vertex_ops(hgt_graph* g, const uint32_t* edge_ids, const uint32_t* vertices,
                         const uint8_t* insert, uint64_t n_ops, void* stream);

/* ---- batched form ------------------------------------------------------ */
/* One graph's batch for hgt_apply_batches: the arguments of hgt_apply_batch,
 * plus its result. */
typedef struct {
    hgt_graph* graph;
    const uint32_t* del_ids;        /* device */
    uint64_t n_del;
    const uint64_t* ins_offsets;    /* device */
    const uint32_t* ins_members;    /* device */
    uint64_t n_ins_members;
    const int64_t* ins_ts;          /* device */
    uint64_t n_ins;
    uint32_t* out_ins_ids;          /* device, may be NULL */
    int32_t status;                 /* out: this batch's result */
    int32_t pad0;
} hgt_batch;

/* Applies batches[i] to batches[i].graph for every i, with the same semantics
 * and the same results as n separate hgt_apply_batch calls.  The graphs must
 * be distinct and live on the current device.  Their planning passes are
 * queued together and the call waits once for all of their summaries; the
 * triad phases of all graphs then share one launch per kernel, whose workgroups
 * take (graph, hyperedge) work items from one device queue.  A batch that
 * fails validation is rejected alone (its status says why); the others are
 * applied.  The first graph's triad scratch serves the whole call, so calls
 * that share a graph must not overlap.  Returns HGT_OK when every batch was
 * applied, else the first failing batch's status. */
int hgt_apply_batches(hgt_batch* batches, uint32_t n, void* stream);

/* Flags of hgt_apply_batches_ex. */
#define HGT_BATCHES_GRAPH 1u     /* the triad phases and the commit of the round
                                  * are captured into a HIP graph (every scratch
                                  * buffer reserved and every work descriptor
                                  * uploaded first) and launched as one; the
                                  * executable graph is kept per triad-scratch
                                  * context and updated in place by the next
                                  * round of the same shape.  A round called on
                                  * the null stream is captured on a stream of
                                  * the library's own, ordered by events with the
                                  * caller's.  Where the capture fails the round
                                  * is launched kernel by kernel. */
#define HGT_BATCHES_AUTOTUNE 2u  /* launch choices (workgroups per CU of the
                                  * global histogram stage, whether centres skip
                                  * the 148 KB stage, slots of the per-wave
                                  * 2-hop hashes, the vertex-pair count from
                                  * which a dense centre goes to the 2-hop
                                  * kernel) picked per key of the round:
                                  * tracked families, number of graphs, changes
                                  * and the 2-hop load of the heaviest centre,
                                  * in log2/log4 buckets.  Each choice is timed
                                  * on live rounds (HIP events, read back without
                                  * a wait), up to twice; one far slower than the
                                  * best is dropped after its first trial; the
                                  * fastest is kept and appended to the cache
                                  * file named by
                                  * HGT_TUNE_CACHE (default ~/.cache/hgt_tune.txt,
                                  * "off": none), which later processes read. */

/* hgt_apply_batches with flags (0: the same call).  Every choice gives the
 * same results; only the launch differs.  HGT_EINVAL for unknown flags. */
int hgt_apply_batches_ex(hgt_batch* batches, uint32_t n, void* stream, uint32_t flags);

/* Waits for the autotuner's timed rounds, records what they measured, and
 * returns in *n_settled (may be NULL) how many round keys have a kept choice. */
int hgt_tune_flush(uint32_t* n_settled);

/* ---- served form ------------------------------------------------------- */
/* A request server over many resident hypergraphs ("tenants").  Clients
 * submit update batches from host memory at any time; a server thread merges
 * the admitted requests of distinct tenants into rounds, each applied like
 * one hgt_apply_batches call, and starts a new round while earlier ones are
 * still on the GPU (continuous batching).  Per tenant, requests are applied
 * in submission order, one at a time, so each result equals that of applying
 * the tenant's requests alone with hgt_apply_batch.
 * Admission: a request's inputs, assigned IDs and result counts live in a
 * device arena (with a pinned host mirror) of desc.arena_bytes; it is
 * admitted when its arena range fits and the footprint estimate of all
 * admitted requests (inputs + batch scratch, from the request sizes and the
 * tenant's mean cardinality) stays within desc.hbm_budget_bytes.  A request
 * whose footprint alone exceeds the budget runs in a round of its own. */
typedef struct hgt_server hgt_server;

typedef struct {
    uint64_t hbm_budget_bytes;  /* footprint limit of the admitted requests     */
    uint64_t arena_bytes;       /* device arena for request buffers (0: 256 MiB) */
    uint32_t max_round;         /* most requests merged into one round (0: 256) */
    uint32_t max_inflight;      /* rounds on the GPU at once, 1..4 (0: 4)        */
    uint32_t launch_flags;      /* HGT_BATCHES_* flags of every round (0: none)  */
    uint32_t pad0;
} hgt_server_desc;

/* One update request (host buffers, copied by hgt_server_submit): the
 * arguments of hgt_apply_batch.  out_ins_ids_host (may be NULL) receives the
 * assigned IDs and must stay valid until hgt_server_wait returns. */
typedef struct {
    const uint32_t* del_ids;
    uint64_t n_del;
    const uint64_t* ins_offsets;
    const uint32_t* ins_members;
    uint64_t n_ins_members;
    const int64_t* ins_ts;
    uint64_t n_ins;
    uint32_t* out_ins_ids_host;
} hgt_request;

/* Result of a request: its status, the tenant's counts after it (families the
 * tenant does not track are 0) and its times in ns of a monotonic clock. */
typedef struct {
    int32_t status;
    uint32_t tenant;
    uint64_t he[30];
    uint64_t iv[3];
    uint64_t temporal[96];
    uint64_t t_submit_ns, t_admit_ns, t_done_ns;
    uint64_t round;             /* the round that applied it                   */
    uint32_t round_size;        /* requests in that round                      */
    uint32_t pad0;
} hgt_result;

typedef struct {
    uint64_t rounds, requests_done, requests_pending, requests_running;
    uint64_t footprint_in_use, arena_in_use;
    uint64_t max_round_size, max_inflight_seen;
} hgt_server_info;

/* Creates a server on the current device and starts its thread. */
int hgt_server_create(const hgt_server_desc* d, hgt_server** out);

/* Builds a tenant (as hgt_build, on the server's stream) and returns its index. */
int hgt_server_add_tenant(hgt_server* s, const hgt_build_desc* d, uint32_t* tenant);

/* The tenant's graph, for queries while the server holds none of its requests. */
int hgt_server_tenant_graph(hgt_server* s, uint32_t tenant, hgt_graph** out);

/* Copies the request and queues it; *ticket names it.  HGT_ENOMEM when it
 * can never fit the arena, HGT_EINVAL for bad arguments. */
int hgt_server_submit(hgt_server* s, uint32_t tenant, const hgt_request* r, uint64_t* ticket);

/* Waits until the request is done and fills *out (may be NULL); the ticket is
 * then released.  Returns the request's status. */
int hgt_server_wait(hgt_server* s, uint64_t ticket, hgt_result* out);

/* *done = 1 when the request has completed (non-blocking). */
int hgt_server_query(hgt_server* s, uint64_t ticket, int* done);

int hgt_server_get_info(hgt_server* s, hgt_server_info* out);

/* Waits for all submitted requests, stops the thread and destroys the tenants. */
int hgt_server_destroy(hgt_server* s);

/* ---- queries ---------------------------------------------------------- */
/* Copies the maintained counts of family `type` to out_host[0..n_out) (host).
 * n_out must be at least 30 / 3 / 96.  `window` must be 0 for the hyperedge
 * and incident-vertex families and equal the tracked window for temporal
 * (else HGT_ENOTTRACKED).  Synchronises the graph's last stream. */
int hgt_triad_counts(hgt_graph* g, int type, int64_t window, uint64_t* out_host, uint32_t n_out);

/* Waits for the graph's queued work; *status (may be NULL) receives the
 * sticky status of the graph (HGT_OK or the first error). */
int hgt_sync(hgt_graph* g, int* status);

/* Releases every device buffer of the graph (also a poisoned one). */
int hgt_destroy(hgt_graph* g);

/* ---- snapshot and restore ---------------------------------------------- */
/* A snapshot is a host-memory copy of everything a graph's future batches and
 * queries depend on: the ID table (offset, length, capacity, arrival sequence
 * and timestamp of every ID below next_id, and the free-ID bitmap), both
 * incidence pools up to their used words, the maintained hyperedge-neighbour
 * histograms, the per-vertex list table, the 129 maintained counts and the
 * scalars (next_id, used pool words, next arrival sequence, largest
 * timestamp, live hyperedges, incidences).  It is owned by the library until
 * hgt_snap_free(); it can be written out as bytes and loaded back, in the
 * same or another process, to restore a graph built with the same
 * n_vertices, track_mask and temporal_window (for example an empty one).
 *
 * Byte format (little-endian): a 128-byte header of
 *   char magic[8] = "HGTSNAP1"; uint32 version = 1; uint32 track_mask;
 *   uint32 n_vertices; uint32 n_counts = 129; int64 temporal_window;
 *   uint64 next_id, h_bump, v_bump, next_seq, n_live, n_incidences;
 *   int64 last_ts; uint64 payload_bytes; uint64 checksum; zero padding;
 * then the sections, each padded with zeros to a multiple of 8 bytes:
 *   uint64 counts[129] (hyperedge 30, incident-vertex 3, temporal 96);
 *   uint64 h_off[next_id]; uint32 h_len[next_id]; uint32 h_cap[next_id];
 *   uint64 h_seq[next_id]; int64 h_ts[next_id] (temporal graphs only);
 *   uint64 free_bitmap[(next_id + 63) / 64] (bit i set: ID i is free);
 *   uint32 h2v[h_bump]; uint32 histograms[2 * h_bump] (hyperedge family only);
 *   uint64 v_off[n_vertices]; uint32 v_len[n_vertices]; uint32 v_cap[n_vertices];
 *   uint32 v2h[v_bump]; int64 v2h_ts[v_bump] (temporal graphs only).
 * checksum: over the payload read as uint64 words w, h = 0xcbf29ce484222325
 * and for each word h = (h ^ w) * 0x100000001b3 (mod 2^64).
 * Like every call on a graph, hgt_snapshot and hgt_restore must not overlap
 * another call on the same graph; for a served tenant (hgt_server_tenant_graph)
 * none of the tenant's requests may be in flight. */
typedef struct hgt_snap hgt_snap;

/* Copies graph g into a new snapshot *out (host memory).  Waits for the
 * graph's queued work and for `stream`, on which the copies run.
 * HGT_EPOISONED for a poisoned graph. */
int hgt_snapshot(hgt_graph* g, hgt_snap** out, void* stream);

/* Replaces the whole state of graph g (poisoned or not) by the snapshot's:
 * afterwards g answers every query and applies every batch exactly as the
 * graph the snapshot was taken from did at that moment (assigned IDs
 * included).  g must have the snapshot's n_vertices, track_mask and
 * temporal_window (else HGT_EINVAL, g unchanged).  The pools grow when the
 * snapshot needs more words (HGT_ENOMEM, g unchanged, when they cannot).
 * The copies run on `stream` and the call waits for them; the batch and
 * compaction statistics of g are kept.  A HIP failure during the copies
 * leaves g poisoned. */
int hgt_restore(hgt_graph* g, const hgt_snap* snap, void* stream);

/* Byte form of a snapshot: *n_bytes receives its size; when out_host is not
 * NULL the bytes are written there (HGT_EINVAL if cap < the size). */
int hgt_snap_bytes(const hgt_snap* snap, void* out_host, uint64_t cap, uint64_t* n_bytes);

/* Loads a snapshot from its byte form (host memory, not kept).  The header,
 * the section sizes and the checksum are checked, and so is the structure:
 * every live ID's list lies inside the used h2v words, is strictly
 * ascending and names vertices below n_vertices; every vertex's list lies
 * inside the used v2h words, is strictly ascending and names live IDs; the
 * two maps hold the same incidences; n_live, n_incidences and the v2h
 * timestamps agree with the ID table.  The counts and the neighbour
 * histograms are covered by the checksum only (the kernels use them as
 * numbers, never as indices).  HGT_EINVAL when any check fails. */
int hgt_snap_load(const void* bytes, uint64_t n_bytes, hgt_snap** out);

/* Releases a snapshot. */
int hgt_snap_free(hgt_snap* snap);

/* Moves every live incidence list into fresh pools, dropping the blocks of
 * free IDs and the blocks that relocated lists left behind (the pools only
 * grow otherwise).  Counts and contents are unchanged.  A batch runs this by
 * itself first when a pool holds more than twice what its live lists need;
 * the no-allocation entry point never does.  Waits for `stream`. */
int hgt_compact(hgt_graph* g, void* stream);

const char* hgt_status_str(int status);

/* ---- introspection (tests, tools) -------------------------------------- */
typedef struct {
    uint32_t n_vertices;
    uint32_t track_mask;
    uint64_t next_id;        /* IDs in use are < next_id                        */
    uint64_t n_live;         /* live hyperedges                                 */
    uint64_t n_incidences;   /* sum of live cardinalities                       */
    uint64_t edge_capacity;
    uint64_t h2v_pool_words, h2v_used_words;
    uint64_t v2h_pool_words, v2h_used_words;
    int64_t temporal_window;
    uint64_t batches;        /* batches applied since build                     */
    uint64_t compactions;    /* pool compactions since build                    */
    uint64_t graph_launches; /* batched rounds with this graph first that ran
                              * as one captured HIP graph (HGT_BATCHES_GRAPH)  */
} hgt_info;

int hgt_get_info(hgt_graph* g, hgt_info* out);

/* Copies the hyperedge->vertex map to host CSR indexed by ID:
 * offsets_host[0..next_id], members_host[0..n_incidences) (each row sorted),
 * live_host[0..next_id) (1 = live).  Dead IDs have empty rows. */
int hgt_export_h2v(hgt_graph* g, uint64_t* offsets_host, uint32_t* members_host, uint8_t* live_host);

/* Copies the vertex->hyperedge map to host CSR indexed by vertex:
 * offsets_host[0..n_vertices], members_host[0..n_incidences) (rows ascending). */
int hgt_export_v2h(hgt_graph* g, uint64_t* offsets_host, uint32_t* members_host);

/* ---- profiling (tools) ------------------------------------------------ */
/* Per kernel group of the batch path: launches and summed duration (HIP events
 * recorded on the batch stream around the group), and the algorithmic bytes
 * the group moved: for the triad-delta kernels the incidence lists they gather
 * (4 bytes per list entry read), for the store commit 16d+16 bytes per insert
 * and 12d+8 per delete of cardinality d.  `events`/`aux`: neighbours expanded /
 * expanded through the binary-search path (small-centre kernel) and centres
 * deferred (large-centre kernel). */
typedef struct {
    char name[24];
    uint64_t launches;
    double total_ms;
    uint64_t algo_bytes;
    uint64_t events;
    uint64_t aux;
} hgt_kernel_time;

/* Waits for the graph's work, resets the profile and switches it off (0), on
 * (1: HIP events around each kernel group and algorithmic-byte counters, a
 * few atomics per changed hyperedge) or on with the hyperedge-delta stages'
 * wall-clock phase timers (2: a clock read and a workgroup barrier per phase,
 * which slows those kernels; for breakdowns, not for timing). */
int hgt_profile(hgt_graph* g, int enable);

/* Waits for the graph's work and copies up to n_max rows (host) ; *n_out
 * receives the number of rows available. */
int hgt_profile_read(hgt_graph* g, hgt_kernel_time* out_host, uint32_t n_max, uint32_t* n_out);

/* Waits for the graph's work and copies the raw device counters of the
 * profile (algorithmic bytes, hand-overs between kernel stages, wall-clock
 * ticks per phase of the hyperedge-delta stages: counters 16 + 12 s + p for
 * stage s and phase p = 0 member prefix, 1 neighbour hash, 2 compaction,
 * 3 disjoint-pair classes, 4 vertex grouping, 5 open paths, 6 intersecting
 * pairs (all of them when enumerated; the correction of pairs sharing several
 * vertices when aggregated), 7 hand-over, 8 aggregated: short runs, 9 vertex
 * pairs, 10 long runs; 12-14 the aggregated phase's long runs, corrected
 * pairs and enumerating centres; 56.. temporal counters) to
 * out_host[0..n_max); *n_out receives the count (64). */
int hgt_profile_counters(hgt_graph* g, uint64_t* out_host, uint32_t n_max, uint32_t* n_out);

/* Class codes of the hyperedge (30) or temporal (96) family, ascending;
 * host out[0..n).  Returns the number of classes or a negative status. */
int hgt_class_codes(int type, int32_t* out_host, uint32_t n);

#ifdef __cplusplus
}
#endif

#endif /* HGT_H */
