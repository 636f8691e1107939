/*
 * hgt_oracle.c -- plain, slow CPU reference for hypergraph triad counts.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the GPU library; every table below is built
 * here from the definitions in the paper.
 *
 * Input hypergraphs are CSR over ID slots 0..n_slots-1: slot i is live when
 * live[i] != 0 and then holds the sorted, duplicate-free vertex list
 * members[offsets[i] .. offsets[i+1]).  The Python side canonicalises rows.
 *
 * Definitions followed (paper, Sec. II "Hypergraph Triads"):
 *  - hyperedge triad: an unordered triple of distinct hyperedges that is
 *    connected in the line graph (at least two of the three pairs share a
 *    vertex).  Its pattern is the emptiness of the 7 Venn regions of the
 *    three vertex sets; patterns equal up to relabelling form one class
 *    (26 classes for distinct vertex sets, plus 4 classes that need two or
 *    three identical vertex sets, reported separately).
 *  - temporal triad: a connected triple ordered by arrival time
 *    (timestamp, then arrival sequence for equal timestamps) whose first and
 *    last timestamps differ by at most the window; the class is the Venn
 *    pattern in time order, no relabelling (96 classes).
 *  - incident-vertex triads (types 1-3, with hyperedge multiplicity): a
 *    vertex triple {u,v,w} together with a witness hyperedge for each of its
 *    three pairs; type 1 = the three witnesses are one hyperedge, type 2 =
 *    exactly two witnesses coincide, type 3 = three distinct witnesses.
 *
 * Region bits of an ordered triple (a, b, c):
 *   bit0 a only, bit1 b only, bit2 c only, bit3 a&b not c, bit4 b&c not a,
 *   bit5 c&a not b, bit6 a&b&c.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define N_HE_CLASSES 30
#define N_TMP_CLASSES 96

/* ------------------------------------------------------------------ */
/* pattern tables                                                      */
/* ------------------------------------------------------------------ */
/* Members of each region, as a 3-bit set over {a=1, b=2, c=4}. */
static const int region_set[7] = {1, 2, 4, 3, 6, 5, 7};

static int tables_built = 0;
static int he_class[128];  /* canonical-pattern class index, -1 if not a triad */
static int tmp_class[128]; /* ordered-pattern class index, -1 if not a triad   */
static int he_codes[N_HE_CLASSES];
static int tmp_codes[N_TMP_CLASSES];
static int n_he = 0, n_tmp = 0;

static int pattern_is_triad(int code) {
    int has[3] = {0, 0, 0};
    for (int r = 0; r < 7; r++)
        if (code >> r & 1)
            for (int s = 0; s < 3; s++)
                if (region_set[r] >> s & 1) has[s] = 1;
    if (!has[0] || !has[1] || !has[2]) return 0; /* some hyperedge empty */
    /* pair (s,t) intersects when a non-empty region contains both */
    int pairs = 0;
    const int pr[3] = {3, 6, 5};
    for (int p = 0; p < 3; p++) {
        int meet = 0;
        for (int r = 0; r < 7; r++)
            if ((code >> r & 1) && (region_set[r] & pr[p]) == pr[p]) meet = 1;
        pairs += meet;
    }
    return pairs >= 2;
}

/* Pattern of the relabelled triple: new label k is old label perm[k]. */
static int relabel(int code, const int perm[3]) {
    int out = 0;
    for (int r = 0; r < 7; r++) {
        if (!(code >> r & 1)) continue;
        int s = region_set[r], ns = 0;
        for (int k = 0; k < 3; k++)
            if (s >> perm[k] & 1) ns |= 1 << k;
        for (int q = 0; q < 7; q++)
            if (region_set[q] == ns) out |= 1 << q;
    }
    return out;
}

static void build_tables(void) {
    if (tables_built) return;
    static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int canon[128];
    for (int c = 0; c < 128; c++) {
        canon[c] = -1;
        if (!pattern_is_triad(c)) continue;
        int m = 1000;
        for (int p = 0; p < 6; p++) {
            int r = relabel(c, perms[p]);
            if (r < m) m = r;
        }
        canon[c] = m;
    }
    n_he = 0;
    n_tmp = 0;
    for (int c = 0; c < 128; c++) {
        if (canon[c] == c) he_codes[n_he++] = c;
        if (canon[c] >= 0) tmp_codes[n_tmp++] = c;
    }
    for (int c = 0; c < 128; c++) {
        he_class[c] = -1;
        tmp_class[c] = -1;
        if (canon[c] < 0) continue;
        for (int i = 0; i < n_he; i++)
            if (he_codes[i] == canon[c]) he_class[c] = i;
        for (int i = 0; i < n_tmp; i++)
            if (tmp_codes[i] == c) tmp_class[c] = i;
    }
    tables_built = 1;
}

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int orc_n_he_classes(void) { build_tables(); return n_he; }
int orc_n_tmp_classes(void) { build_tables(); return n_tmp; }
void orc_he_class_codes(int32_t* out) { build_tables(); for (int i = 0; i < n_he; i++) out[i] = he_codes[i]; }
void orc_tmp_class_codes(int32_t* out) { build_tables(); for (int i = 0; i < n_tmp; i++) out[i] = tmp_codes[i]; }
int orc_he_class_of_code(int code) { build_tables(); return (code >= 0 && code < 128) ? he_class[code] : -1; }
int orc_tmp_class_of_code(int code) { build_tables(); return (code >= 0 && code < 128) ? tmp_class[code] : -1; }

/* ------------------------------------------------------------------ */
/* set helpers on sorted lists                                         */
/* ------------------------------------------------------------------ */
typedef struct {
    uint64_t n_slots;
    const uint64_t* off;
    const uint32_t* mem;
    const uint8_t* live;
    uint32_t n_vertices;
    /* vertex -> incident live slots (ascending) */
    uint64_t* voff;
    uint32_t* vmem;
} graph_t;

static uint64_t glen(const graph_t* g, uint64_t i) { return g->off[i + 1] - g->off[i]; }
static const uint32_t* grow(const graph_t* g, uint64_t i) { return g->mem + g->off[i]; }

static uint64_t inter2(const uint32_t* a, uint64_t na, const uint32_t* b, uint64_t nb) {
    uint64_t i = 0, j = 0, k = 0;
    while (i < na && j < nb) {
        if (a[i] < b[j]) i++;
        else if (a[i] > b[j]) j++;
        else { k++; i++; j++; }
    }
    return k;
}

static uint64_t inter3(const uint32_t* a, uint64_t na, const uint32_t* b, uint64_t nb,
                       const uint32_t* c, uint64_t nc) {
    uint64_t i = 0, j = 0, l = 0, k = 0;
    while (i < na && j < nb && l < nc) {
        uint32_t m = a[i];
        if (b[j] > m) m = b[j];
        if (c[l] > m) m = c[l];
        if (a[i] < m) { i++; continue; }
        if (b[j] < m) { j++; continue; }
        if (c[l] < m) { l++; continue; }
        k++; i++; j++; l++;
    }
    return k;
}

/* Venn pattern of the ordered triple (a, b, c). */
static int pattern3(const graph_t* g, uint64_t a, uint64_t b, uint64_t c) {
    const uint32_t *A = grow(g, a), *B = grow(g, b), *C = grow(g, c);
    uint64_t na = glen(g, a), nb = glen(g, b), nc = glen(g, c);
    int64_t ab = (int64_t)inter2(A, na, B, nb);
    int64_t bc = (int64_t)inter2(B, nb, C, nc);
    int64_t ca = (int64_t)inter2(C, nc, A, na);
    int64_t abc = (int64_t)inter3(A, na, B, nb, C, nc);
    int64_t r[7];
    r[0] = (int64_t)na - ab - ca + abc;
    r[1] = (int64_t)nb - ab - bc + abc;
    r[2] = (int64_t)nc - bc - ca + abc;
    r[3] = ab - abc;
    r[4] = bc - abc;
    r[5] = ca - abc;
    r[6] = abc;
    int code = 0;
    for (int i = 0; i < 7; i++)
        if (r[i] > 0) code |= 1 << i;
    return code;
}

static int build_v2h(graph_t* g) {
    uint32_t nv = g->n_vertices;
    g->voff = (uint64_t*)calloc((size_t)nv + 1, sizeof(uint64_t));
    if (!g->voff) return -1;
    for (uint64_t i = 0; i < g->n_slots; i++) {
        if (!g->live[i]) continue;
        for (uint64_t k = g->off[i]; k < g->off[i + 1]; k++) g->voff[g->mem[k] + 1]++;
    }
    for (uint32_t v = 0; v < nv; v++) g->voff[v + 1] += g->voff[v];
    g->vmem = (uint32_t*)malloc((size_t)(g->voff[nv] ? g->voff[nv] : 1) * sizeof(uint32_t));
    uint64_t* fill = (uint64_t*)malloc(((size_t)nv + 1) * sizeof(uint64_t));
    if (!g->vmem || !fill) { free(fill); return -1; }
    memcpy(fill, g->voff, ((size_t)nv + 1) * sizeof(uint64_t));
    /* ascending slot order gives ascending incidence lists */
    for (uint64_t i = 0; i < g->n_slots; i++) {
        if (!g->live[i]) continue;
        for (uint64_t k = g->off[i]; k < g->off[i + 1]; k++) g->vmem[fill[g->mem[k]]++] = (uint32_t)i;
    }
    free(fill);
    return 0;
}

static void free_graph(graph_t* g) {
    free(g->voff);
    free(g->vmem);
}

static int init_graph(graph_t* g, uint64_t n_slots, const uint64_t* off, const uint32_t* mem,
                      const uint8_t* live, uint32_t n_vertices) {
    g->n_slots = n_slots;
    g->off = off;
    g->mem = mem;
    g->live = live;
    g->n_vertices = n_vertices;
    g->voff = NULL;
    g->vmem = NULL;
    return build_v2h(g);
}

/* Line-graph neighbours of slot b (live slots sharing a vertex, excluding b),
   written into nb[]; stamp[] marks membership with the value tag. */
static uint64_t neighbours(const graph_t* g, uint64_t b, uint64_t* stamp, uint64_t tag, uint32_t* nb) {
    uint64_t k = 0;
    for (uint64_t p = g->off[b]; p < g->off[b + 1]; p++) {
        uint32_t v = g->mem[p];
        for (uint64_t q = g->voff[v]; q < g->voff[v + 1]; q++) {
            uint32_t x = g->vmem[q];
            if (x == b || stamp[x] == tag) continue;
            stamp[x] = tag;
            nb[k++] = x;
        }
    }
    return k;
}

/* ------------------------------------------------------------------ */
/* full counts                                                         */
/* ------------------------------------------------------------------ */
typedef struct {
    const int64_t* ts;
    const uint64_t* seq;
    int64_t window;
} tinfo_t;

static int earlier(const tinfo_t* t, uint64_t x, uint64_t y) {
    if (t->ts[x] != t->ts[y]) return t->ts[x] < t->ts[y];
    return t->seq[x] < t->seq[y];
}

/* Add the triad {a,b,c} to the hyperedge and/or temporal histograms. */
static void add_triad(const graph_t* g, uint64_t a, uint64_t b, uint64_t c, uint64_t* he,
                      uint64_t* tmp, const tinfo_t* ti, int64_t sign) {
    if (he) {
        int cl = he_class[pattern3(g, a, b, c)];
        he[cl] += (uint64_t)sign;
    }
    if (tmp) {
        uint64_t o[3] = {a, b, c};
        /* sort the three by arrival key */
        for (int i = 0; i < 3; i++)
            for (int j = 0; j + 1 < 3 - i; j++)
                if (earlier(ti, o[j + 1], o[j])) { uint64_t t = o[j]; o[j] = o[j + 1]; o[j + 1] = t; }
        if (ti->ts[o[2]] - ti->ts[o[0]] <= ti->window) {
            int cl = tmp_class[pattern3(g, o[0], o[1], o[2])];
            tmp[cl] += (uint64_t)sign;
        }
    }
}

/*
 * Full recount by line-graph wedges: every connected triple has at least one
 * hyperedge adjacent to the other two (a centre).  For each centre b and each
 * unordered pair {a,c} of its neighbours: if a and c also intersect the triple
 * is closed and has three centres, so it is counted only at its smallest ID;
 * otherwise b is its only centre.
 * he: u64[30] or NULL; tmp: u64[96] or NULL (needs ts, seq).
 */
int orc_count_full(uint64_t n_slots, const uint64_t* off, const uint32_t* mem, const uint8_t* live,
                   uint32_t n_vertices, const int64_t* ts, const uint64_t* seq, int64_t window,
                   uint64_t* he, uint64_t* tmp) {
    build_tables();
    graph_t g;
    if (init_graph(&g, n_slots, off, mem, live, n_vertices)) { free_graph(&g); return -1; }
    tinfo_t ti = {ts, seq, window};
    if (he) memset(he, 0, N_HE_CLASSES * sizeof(uint64_t));
    if (tmp) memset(tmp, 0, N_TMP_CLASSES * sizeof(uint64_t));
    int err = 0;
    /* temporal-only: a triple whose timestamps span more than the window is
       never counted, so such neighbours and pairs are skipped early */
    int tmp_only = (he == NULL && tmp != NULL);
#pragma omp parallel
    {
        uint64_t* stamp = (uint64_t*)malloc((n_slots ? n_slots : 1) * sizeof(uint64_t));
        uint32_t* nb = (uint32_t*)malloc((n_slots ? n_slots : 1) * sizeof(uint32_t));
        uint64_t lhe[N_HE_CLASSES], ltmp[N_TMP_CLASSES];
        memset(lhe, 0, sizeof lhe);
        memset(ltmp, 0, sizeof ltmp);
        if (!stamp || !nb) {
#pragma omp atomic write
            err = 1;
        } else {
            for (uint64_t i = 0; i < n_slots; i++) stamp[i] = UINT64_MAX;
#pragma omp for schedule(dynamic, 16)
            for (uint64_t b = 0; b < n_slots; b++) {
                if (!live[b]) continue;
                uint64_t k = neighbours(&g, b, stamp, b, nb);
                if (tmp_only) {
                    uint64_t kk = 0;
                    for (uint64_t i = 0; i < k; i++) {
                        int64_t d = ts[nb[i]] - ts[b];
                        if (d <= window && -d <= window) nb[kk++] = nb[i];
                    }
                    k = kk;
                }
                for (uint64_t i = 0; i < k; i++) {
                    for (uint64_t j = i + 1; j < k; j++) {
                        uint64_t a = nb[i], c = nb[j];
                        if (tmp_only) {
                            int64_t d = ts[a] - ts[c];
                            if (d > window || -d > window) continue;
                        }
                        int closed = inter2(grow(&g, a), glen(&g, a), grow(&g, c), glen(&g, c)) > 0;
                        if (closed && !(b < a && b < c)) continue;
                        add_triad(&g, a, b, c, he ? lhe : NULL, tmp ? ltmp : NULL, &ti, 1);
                    }
                }
            }
        }
#pragma omp critical
        {
            if (he) for (int i = 0; i < N_HE_CLASSES; i++) he[i] += lhe[i];
            if (tmp) for (int i = 0; i < N_TMP_CLASSES; i++) tmp[i] += ltmp[i];
        }
        free(stamp);
        free(nb);
    }
    free_graph(&g);
    return err ? -1 : 0;
}

/*
 * Triads (of the given graph) that contain at least one marked slot, each
 * counted once: at its smallest-ID marked member h.  The connected triples
 * containing h are {h,x,y} with x,y both neighbours of h, and {h,x,y} with x
 * a neighbour of h and y a neighbour of x that neither is h nor meets h.
 */
int orc_count_containing(uint64_t n_slots, const uint64_t* off, const uint32_t* mem,
                         const uint8_t* live, uint32_t n_vertices, const int64_t* ts,
                         const uint64_t* seq, int64_t window, const uint8_t* marked,
                         uint64_t* he, uint64_t* tmp) {
    build_tables();
    graph_t g;
    if (init_graph(&g, n_slots, off, mem, live, n_vertices)) { free_graph(&g); return -1; }
    tinfo_t ti = {ts, seq, window};
    if (he) memset(he, 0, N_HE_CLASSES * sizeof(uint64_t));
    if (tmp) memset(tmp, 0, N_TMP_CLASSES * sizeof(uint64_t));
    int err = 0;
    const int tmp_only = (he == NULL && tmp != NULL);
#pragma omp parallel
    {
        uint64_t* stamp = (uint64_t*)malloc((n_slots ? n_slots : 1) * sizeof(uint64_t));
        uint64_t* stamp2 = (uint64_t*)malloc((n_slots ? n_slots : 1) * sizeof(uint64_t));
        uint32_t* nb = (uint32_t*)malloc((n_slots ? n_slots : 1) * sizeof(uint32_t));
        uint32_t* nb2 = (uint32_t*)malloc((n_slots ? n_slots : 1) * sizeof(uint32_t));
        uint64_t lhe[N_HE_CLASSES], ltmp[N_TMP_CLASSES];
        memset(lhe, 0, sizeof lhe);
        memset(ltmp, 0, sizeof ltmp);
        if (!stamp || !stamp2 || !nb || !nb2) {
#pragma omp atomic write
            err = 1;
        } else {
            for (uint64_t i = 0; i < n_slots; i++) stamp[i] = stamp2[i] = UINT64_MAX;
            uint64_t tag2 = 0;
#pragma omp for schedule(dynamic, 4)
            for (uint64_t h = 0; h < n_slots; h++) {
                if (!live[h] || !marked[h]) continue;
                uint64_t k = neighbours(&g, h, stamp, h, nb);
                /* temporal only: a triple whose timestamps span more than the window
                   is never counted, so its members are skipped early (the closed
                   neighbourhood of h keeps all of N(h) for the test below) */
                uint64_t kw = k;
                if (tmp_only) {
                    kw = 0;
                    for (uint64_t i = 0; i < k; i++) {
                        int64_t d = ts[nb[i]] - ts[h];
                        if (d <= window && -d <= window) { uint32_t t = nb[kw]; nb[kw++] = nb[i]; nb[i] = t; }
                    }
                }
                /* both others adjacent to h */
                for (uint64_t i = 0; i < kw; i++) {
                    for (uint64_t j = i + 1; j < kw; j++) {
                        uint64_t x = nb[i], y = nb[j];
                        if ((marked[x] && x < h) || (marked[y] && y < h)) continue;
                        if (tmp_only) {
                            int64_t d = ts[x] - ts[y];
                            if (d > window || -d > window) continue;
                        }
                        add_triad(&g, h, x, y, he ? lhe : NULL, tmp ? ltmp : NULL, &ti, 1);
                    }
                }
                /* path h - x - y with y outside the closed neighbourhood of h */
                for (uint64_t i = 0; i < kw; i++) {
                    uint64_t x = nb[i];
                    if (marked[x] && x < h) continue;
                    uint64_t k2 = neighbours(&g, x, stamp2, tag2++, nb2);
                    for (uint64_t j = 0; j < k2; j++) {
                        uint64_t y = nb2[j];
                        if (y == h || stamp[y] == h) continue;
                        if (marked[y] && y < h) continue;
                        if (tmp_only) {
                            int64_t d1 = ts[y] - ts[h], d2 = ts[y] - ts[x];
                            if (d1 > window || -d1 > window || d2 > window || -d2 > window) continue;
                        }
                        add_triad(&g, h, x, y, he ? lhe : NULL, tmp ? ltmp : NULL, &ti, 1);
                    }
                }
            }
        }
#pragma omp critical
        {
            if (he) for (int i = 0; i < N_HE_CLASSES; i++) he[i] += lhe[i];
            if (tmp) for (int i = 0; i < N_TMP_CLASSES; i++) tmp[i] += ltmp[i];
        }
        free(stamp); free(stamp2); free(nb); free(nb2);
    }
    free_graph(&g);
    return err ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* incident-vertex triads                                              */
/* ------------------------------------------------------------------ */
typedef struct {
    uint64_t key;  /* u << 32 | v, u < v */
    uint64_t m;    /* hyperedges containing both */
    uint64_t w;    /* sum over those hyperedges of (|h| - 2) */
} pair_t;

static int cmp_pair(const void* a, const void* b) {
    uint64_t x = ((const pair_t*)a)->key, y = ((const pair_t*)b)->key;
    return x < y ? -1 : x > y;
}

static uint64_t choose3(uint64_t n) { return n < 3 ? 0 : n * (n - 1) * (n - 2) / 6; }

/*
 * out[0] = type 1 = sum_h C(|h|,3)                       (all witnesses equal)
 * out[1] = type 2 = sum_h (|h|-2) * sum_{pairs p in h} m_p  - 3 * type 1
 *          (a triple inside h, one of its three pairs re-witnessed by another
 *           hyperedge containing that pair)
 * out[2] = type 3 = sum_{u<v<w} m_uv m_vw m_uw - type 1 - type 2
 * where m_p is the number of live hyperedges containing the vertex pair p.
 * The triple-product sum runs over triangles of the weighted clique expansion.
 */
int orc_count_iv(uint64_t n_slots, const uint64_t* off, const uint32_t* mem, const uint8_t* live,
                 uint32_t n_vertices, uint64_t* out) {
    (void)n_vertices;
    uint64_t t1 = 0, npairs = 0;
    for (uint64_t i = 0; i < n_slots; i++) {
        if (!live[i]) continue;
        uint64_t d = off[i + 1] - off[i];
        t1 += choose3(d);
        npairs += d * (d - 1) / 2;
    }
    pair_t* P = (pair_t*)malloc((npairs ? npairs : 1) * sizeof(pair_t));
    if (!P) return -1;
    uint64_t k = 0;
    for (uint64_t i = 0; i < n_slots; i++) {
        if (!live[i]) continue;
        uint64_t d = off[i + 1] - off[i];
        for (uint64_t a = off[i]; a < off[i + 1]; a++)
            for (uint64_t b = a + 1; b < off[i + 1]; b++) {
                P[k].key = (uint64_t)mem[a] << 32 | mem[b];
                P[k].m = 1;
                P[k].w = d - 2;
                k++;
            }
    }
    qsort(P, npairs, sizeof(pair_t), cmp_pair);
    /* aggregate equal pairs */
    uint64_t u = 0;
    for (uint64_t i = 0; i < npairs; i++) {
        if (u > 0 && P[u - 1].key == P[i].key) {
            P[u - 1].m += P[i].m;
            P[u - 1].w += P[i].w;
        } else {
            P[u++] = P[i];
        }
    }
    uint64_t s2 = 0;
    for (uint64_t i = 0; i < u; i++) s2 += P[i].m * P[i].w;
    /* forward adjacency: for each vertex, its larger neighbours (sorted) */
    uint32_t nv = n_vertices;
    uint64_t* aoff = (uint64_t*)calloc((size_t)nv + 1, sizeof(uint64_t));
    if (!aoff) { free(P); return -1; }
    for (uint64_t i = 0; i < u; i++) aoff[(P[i].key >> 32) + 1]++;
    for (uint32_t v = 0; v < nv; v++) aoff[v + 1] += aoff[v];
    /* P is sorted by (u, v), so the rows are already contiguous and sorted */
    uint64_t tot = 0;
    for (uint64_t e = 0; e < u; e++) {
        uint32_t a = (uint32_t)(P[e].key >> 32), b = (uint32_t)P[e].key;
        /* common larger neighbours w > b of a and b */
        uint64_t i = aoff[a], ie = aoff[a + 1], j = aoff[b], je = aoff[b + 1];
        while (i < ie && j < je) {
            uint32_t wa = (uint32_t)P[i].key, wb = (uint32_t)P[j].key;
            if (wa <= b) { i++; continue; }
            if (wa < wb) i++;
            else if (wa > wb) j++;
            else { tot += P[e].m * P[i].m * P[j].m; i++; j++; }
        }
    }
    free(aoff);
    free(P);
    out[0] = t1;
    out[1] = s2 - 3 * t1;
    out[2] = tot - out[0] - out[1];
    return 0;
}

/* ------------------------------------------------------------------ */
/* incident-vertex terms restricted to a set of vertex pairs           */
/* ------------------------------------------------------------------ */
static int cmp_u64(const void* a, const void* b) {
    uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
    return x < y ? -1 : x > y;
}

static int has_key(const uint64_t* keys, uint64_t n, uint64_t key) {
    uint64_t lo = 0, hi = n;
    while (lo < hi) {
        uint64_t mid = (lo + hi) / 2;
        if (keys[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo < n && keys[lo] == key;
}

static uint64_t pair_key(uint32_t u, uint32_t v) { return u < v ? (uint64_t)u << 32 | v : (uint64_t)v << 32 | u; }

/*
 * The two sums of orc_count_iv's closed forms, restricted to the vertex pairs
 * keys[0..n_keys) (u << 32 | v, u < v, ascending, distinct):
 *   out[0] = sum over the listed pairs p of m_p * w_p;
 *   out[1] = sum over the vertex triangles {a,b,c} having at least one listed
 *            pair of m_ab * m_bc * m_ca (each triangle once).
 * Every pair inside a changed hyperedge is listed, and no other pair changes
 * m or w, so the changes of these two sums between the graphs before and
 * after a batch are the changes of the full sums (the incident-vertex delta
 * of the batch, counted by definition).
 */
int orc_iv_partial(uint64_t n_slots, const uint64_t* off, const uint32_t* mem, const uint8_t* live,
                   uint32_t n_vertices, const uint64_t* keys, uint64_t n_keys, uint64_t* out) {
    graph_t g;
    if (init_graph(&g, n_slots, off, mem, live, n_vertices)) { free_graph(&g); return -1; }
    uint64_t s_sum = 0, x_sum = 0;
    int err = 0;
    /* distinct first endpoints */
    uint64_t* starts = (uint64_t*)malloc((n_keys + 1) * sizeof(uint64_t));
    uint64_t n_a = 0;
    if (!starts) { free_graph(&g); return -1; }
    for (uint64_t i = 0; i < n_keys; i++)
        if (i == 0 || (keys[i] >> 32) != (keys[i - 1] >> 32)) starts[n_a++] = i;
    starts[n_a] = n_keys;
#pragma omp parallel reduction(+ : s_sum, x_sum)
    {
        /* weight[c] = m_ac of the current a, valid where stamp[c] == tag */
        uint64_t* weight = (uint64_t*)calloc((size_t)n_vertices + 1, sizeof(uint64_t));
        uint64_t* stamp = (uint64_t*)malloc(((size_t)n_vertices + 1) * sizeof(uint64_t));
        if (!weight || !stamp) {
#pragma omp atomic write
            err = 1;
        } else {
            for (uint32_t v = 0; v <= n_vertices; v++) stamp[v] = UINT64_MAX;
#pragma omp for schedule(dynamic, 8)
            for (uint64_t ia = 0; ia < n_a; ia++) {
                const uint32_t a = (uint32_t)(keys[starts[ia]] >> 32);
                /* weighted neighbourhood of a in the clique expansion */
                for (uint64_t q = g.voff[a]; q < g.voff[a + 1]; q++) {
                    uint32_t h = g.vmem[q];
                    for (uint64_t k = off[h]; k < off[h + 1]; k++) {
                        uint32_t c = mem[k];
                        if (c == a) continue;
                        if (stamp[c] != ia) { stamp[c] = ia; weight[c] = 0; }
                        weight[c]++;
                    }
                }
                for (uint64_t i = starts[ia]; i < starts[ia + 1]; i++) {
                    const uint32_t b = (uint32_t)keys[i];
                    const uint64_t m_ab = stamp[b] == ia ? weight[b] : 0;
                    if (m_ab == 0) continue;
                    /* w_ab: hyperedges holding both a and b */
                    uint64_t w_ab = 0;
                    uint64_t p = g.voff[a], pe = g.voff[a + 1], r = g.voff[b], re = g.voff[b + 1];
                    while (p < pe && r < re) {
                        if (g.vmem[p] < g.vmem[r]) p++;
                        else if (g.vmem[p] > g.vmem[r]) r++;
                        else { w_ab += glen(&g, g.vmem[p]) - 2; p++; r++; }
                    }
                    s_sum += m_ab * w_ab;
                    /* triangles {a,b,c}: each occurrence of c in a hyperedge of b adds
                       m_ab * m_ac once (summing to m_ab * m_ac * m_bc); a triangle is
                       taken at its smallest listed pair */
                    const uint64_t kab = keys[i];
                    for (uint64_t q = g.voff[b]; q < g.voff[b + 1]; q++) {
                        uint32_t h = g.vmem[q];
                        for (uint64_t k = off[h]; k < off[h + 1]; k++) {
                            uint32_t c = mem[k];
                            if (c == b || c == a || stamp[c] != ia) continue;
                            uint64_t kac = pair_key(a, c), kbc = pair_key(b, c);
                            if ((kac < kab && has_key(keys, n_keys, kac)) || (kbc < kab && has_key(keys, n_keys, kbc)))
                                continue;
                            x_sum += m_ab * weight[c];
                        }
                    }
                }
            }
        }
        free(weight);
        free(stamp);
    }
    free(starts);
    free_graph(&g);
    out[0] = s_sum;
    out[1] = x_sum;
    return err ? -1 : 0;
}

/* The distinct vertex pairs inside the listed live slots, ascending (u << 32 | v).
 * out must hold sum over the slots of C(|h|, 2) keys; returns the distinct count. */
uint64_t orc_pairs_of(const uint64_t* off, const uint32_t* mem, const uint64_t* slots, uint64_t n_slots_listed,
                      uint64_t* out) {
    uint64_t k = 0;
    for (uint64_t i = 0; i < n_slots_listed; i++) {
        uint64_t h = slots[i];
        for (uint64_t x = off[h]; x < off[h + 1]; x++)
            for (uint64_t y = x + 1; y < off[h + 1]; y++) out[k++] = pair_key(mem[x], mem[y]);
    }
    qsort(out, k, sizeof(uint64_t), cmp_u64);
    uint64_t u = 0;
    for (uint64_t i = 0; i < k; i++)
        if (u == 0 || out[u - 1] != out[i]) out[u++] = out[i];
    return u;
}

/* Threads of the oracle's parallel loops (timing of the single-thread mode). */
void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
