"""Seeded synthetic hypergraph workloads.

This module only produces inputs: hypergraphs in CSR form (row offsets + member
vertex ids + optional integer timestamps) and streams of update batches.  It
holds none of the triad arithmetic and none of the ID-assignment rule: batches
name the hyperedges they delete by *handle* (the position of the hyperedge in
the stream of every hyperedge ever created), and each consumer translates
handles to the IDs its own store handed out.

The shapes follow the paper's workloads (Sec. V, Table III: large hypergraphs,
skewed vertex popularity, heavy-tailed cardinality, 50/50 insert/delete
batches, Poisson arrival times for temporal hypergraphs).  The paper's datasets
are not available, so these generators stand in for them.

Distributions
-------------
* cardinality: uniform on [lo, hi] or a discrete power law P(k) ~ k^-alpha on
  [lo, hi], sampled by inverse CDF;
* members: i.i.d. rank draws with weights (rank + q)^-s (Zipf for q = 0,
  Zipf-Mandelbrot for q > 0, uniform for s = 0); a draw that repeats a vertex
  already in the hyperedge is redrawn, column by column, until the hyperedge
  has the requested number of distinct vertices; ranks map to vertex ids
  through a seeded permutation so the hubs are not at id 0;
* members are emitted in draw order (unsorted) so consumers exercise their own
  canonicalisation;
* timestamps: microseconds, cumulative floor(Exp(mean)) gaps (ties occur);
* deletions: uniform without replacement over the handles live at batch start.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

SEED_BASE = 20251221


# --------------------------------------------------------------------------- #
# samplers
# --------------------------------------------------------------------------- #
def uniform_cards(rng: np.random.Generator, n: int, lo: int, hi: int) -> np.ndarray:
    return rng.integers(lo, hi + 1, size=n, dtype=np.int64)


def power_law_cards(rng: np.random.Generator, n: int, alpha: float, lo: int, hi: int) -> np.ndarray:
    ks = np.arange(lo, hi + 1, dtype=np.float64)
    w = ks ** (-alpha)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = rng.random(n)
    idx = np.searchsorted(cdf, u, side="right")
    idx = np.minimum(idx, len(ks) - 1)
    return (lo + idx).astype(np.int64)


class Popularity:
    """Vertex popularity: weight (rank + q)^-s over ranks 1..n, ranks mapped
    to vertex ids by a seeded permutation."""

    def __init__(self, n_vertices: int, s: float, q: float, rng: np.random.Generator):
        self.n = int(n_vertices)
        self.s = float(s)
        self.q = float(q)
        if self.s == 0.0:
            self.cdf = None
        else:
            w = (np.arange(1, self.n + 1, dtype=np.float64) + self.q) ** (-self.s)
            cdf = np.cumsum(w)
            cdf /= cdf[-1]
            self.cdf = cdf
        self.perm = rng.permutation(self.n).astype(np.uint32)

    def draw(self, rng: np.random.Generator, size) -> np.ndarray:
        if self.cdf is None:
            ranks = rng.integers(0, self.n, size=size)
        else:
            ranks = np.searchsorted(self.cdf, rng.random(size), side="right")
            ranks = np.minimum(ranks, self.n - 1)
        return self.perm[ranks]


def draw_members(rng: np.random.Generator, cards: np.ndarray, pop: Popularity) -> np.ndarray:
    """Members of len(cards) hyperedges, row-major (CSR order), each row made of
    distinct vertices.  Column c of every row with card > c is drawn at once;
    draws that repeat a vertex of an earlier column of the same row are redrawn."""
    n = len(cards)
    if n == 0:
        return np.zeros(0, dtype=np.uint32)
    if int(cards.max()) > pop.n:
        raise ValueError("cardinality exceeds the number of vertices")
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(cards, out=offsets[1:])
    out = np.zeros(int(offsets[-1]), dtype=np.uint32)
    order = np.argsort(-cards, kind="stable")  # rows by decreasing card
    sorted_cards = cards[order]
    max_card = int(sorted_cards[0])
    for c in range(max_card):
        n_rows = int(np.searchsorted(-sorted_cards, -c, side="left"))  # rows with card > c
        rows = order[:n_rows]
        vals = pop.draw(rng, n_rows)
        pending = np.arange(n_rows)
        cols = np.arange(c, dtype=np.int64)
        while True:
            base = offsets[rows[pending]]
            if c == 0:
                bad = np.zeros(len(pending), dtype=bool)
            else:
                bad = np.zeros(len(pending), dtype=bool)
                step = max(1, (1 << 22) // c)  # bound the temporary (rows x columns) array
                for a in range(0, len(pending), step):
                    blk = slice(a, a + step)
                    bad[blk] = (out[base[blk, None] + cols] == vals[pending[blk], None]).any(axis=1)
            if not bad.any():
                out[base + c] = vals[pending]
                break
            good = ~bad
            out[base[good] + c] = vals[pending[good]]
            pending = pending[bad]
            vals[pending] = pop.draw(rng, len(pending))
    return out


def poisson_times(rng: np.random.Generator, n: int, mean_gap_us: float, t0: int = 0) -> np.ndarray:
    gaps = np.floor(rng.exponential(mean_gap_us, size=n)).astype(np.int64)
    return t0 + np.cumsum(gaps)


# --------------------------------------------------------------------------- #
# containers
# --------------------------------------------------------------------------- #
@dataclass
class CSR:
    offsets: np.ndarray            # uint64 [n + 1]
    members: np.ndarray            # uint32 [offsets[-1]]
    ts: Optional[np.ndarray] = None  # int64 [n] or None

    @property
    def n(self) -> int:
        return len(self.offsets) - 1

    def row(self, i: int) -> np.ndarray:
        return self.members[int(self.offsets[i]):int(self.offsets[i + 1])]

    def rows(self, idx: np.ndarray) -> "CSR":
        idx = np.asarray(idx, dtype=np.int64)
        lens = (self.offsets[idx + 1] - self.offsets[idx]).astype(np.int64)
        offs = np.zeros(len(idx) + 1, dtype=np.uint64)
        np.cumsum(lens, out=offs[1:])
        if len(idx) and lens.sum():
            starts = self.offsets[idx].astype(np.int64)
            rep = np.repeat(starts - offs[:-1].astype(np.int64), lens)
            src = np.arange(int(offs[-1]), dtype=np.int64) + rep
            mem = self.members[src]
        else:
            mem = np.zeros(0, dtype=np.uint32)
        ts = None if self.ts is None else self.ts[idx]
        return CSR(offs, mem.astype(np.uint32), ts)


def _csr(cards: np.ndarray, members: np.ndarray, ts=None) -> CSR:
    offs = np.zeros(len(cards) + 1, dtype=np.uint64)
    np.cumsum(cards, out=offs[1:])
    return CSR(offs, members.astype(np.uint32), ts)


@dataclass
class Batch:
    del_handles: np.ndarray   # int64, deletion order = batch rank
    ins: CSR                  # inserted hyperedges (ts set for temporal streams)
    ins_handles: np.ndarray   # int64, handles given to the inserts

    @property
    def n_updates(self) -> int:
        return len(self.del_handles) + self.ins.n


@dataclass
class Stream:
    name: str
    n_vertices: int
    initial: CSR
    batches: List[Batch] = field(default_factory=list)
    window: int = 0           # temporal triad window (same unit as ts), 0 if unused
    params: dict = field(default_factory=dict)


# --------------------------------------------------------------------------- #
# generators
# --------------------------------------------------------------------------- #
def plain_stream(name: str, n_vertices: int, n_edges: int, card: tuple, pop_s: float, pop_q: float,
                 n_batches: int, n_ins: int, n_del: int, seed: int) -> Stream:
    """Static-style stream: build n_edges hyperedges, then n_batches batches of
    n_del uniform deletions of live handles + n_ins fresh hyperedges from the
    same distribution.  card = ("uniform", lo, hi) or ("power", alpha, lo, hi)."""
    rng = np.random.default_rng(seed)
    pop = Popularity(n_vertices, pop_s, pop_q, rng)

    def cards_of(n):
        if card[0] == "uniform":
            return uniform_cards(rng, n, card[1], card[2])
        return power_law_cards(rng, n, card[1], card[2], card[3])

    c0 = cards_of(n_edges)
    initial = _csr(c0, draw_members(rng, c0, pop))
    st = Stream(name, n_vertices, initial,
                params=dict(n_edges=n_edges, card=card, pop_s=pop_s, pop_q=pop_q, seed=seed))
    live = np.arange(n_edges, dtype=np.int64)
    next_handle = n_edges
    for _ in range(n_batches):
        k = min(n_del, len(live))
        pick = rng.choice(len(live), size=k, replace=False)
        dels = live[pick]
        keep = np.ones(len(live), dtype=bool)
        keep[pick] = False
        ci = cards_of(n_ins)
        ins = _csr(ci, draw_members(rng, ci, pop))
        ih = np.arange(next_handle, next_handle + n_ins, dtype=np.int64)
        next_handle += n_ins
        live = np.concatenate([live[keep], ih])
        st.batches.append(Batch(dels.astype(np.int64), ins, ih))
    return st


def temporal_stream(name: str, n_vertices: int, n_build: int, batch_size: int, n_batches: int,
                    alpha: float, lo: int, hi: int, mean_gap_us: float, expire_us: int,
                    window_us: int, seed: int, pop_s: float = 0.0, pop_q: float = 0.0) -> Stream:
    """Arrival stream in timestamp order.  The first n_build arrivals form the
    initial hypergraph; each batch inserts the next batch_size arrivals and
    deletes every live hyperedge whose timestamp is older than
    (largest timestamp of the batch) - expire_us, oldest first."""
    rng = np.random.default_rng(seed)
    pop = Popularity(n_vertices, pop_s, pop_q, rng)
    n_total = n_build + batch_size * n_batches
    cards = power_law_cards(rng, n_total, alpha, lo, hi)
    members = draw_members(rng, cards, pop)
    ts = poisson_times(rng, n_total, mean_gap_us)
    full = _csr(cards, members, ts)
    initial = full.rows(np.arange(n_build))
    st = Stream(name, n_vertices, initial, window=int(window_us),
                params=dict(n_build=n_build, batch_size=batch_size, alpha=alpha, lo=lo, hi=hi,
                            mean_gap_us=mean_gap_us, expire_us=expire_us, seed=seed))
    oldest_live = 0  # handles are in timestamp order; live handles form a suffix range
    for b in range(n_batches):
        lo_h = n_build + b * batch_size
        hi_h = lo_h + batch_size
        cutoff = int(ts[hi_h - 1]) - int(expire_us)
        first_keep = int(np.searchsorted(ts[:lo_h], cutoff, side="left"))
        first_keep = max(first_keep, oldest_live)
        dels = np.arange(oldest_live, first_keep, dtype=np.int64)
        oldest_live = first_keep
        ih = np.arange(lo_h, hi_h, dtype=np.int64)
        st.batches.append(Batch(dels, full.rows(ih), ih))
    return st


# --------------------------------------------------------------------------- #
# the named workloads (full sizes) and scaled versions for tests
# --------------------------------------------------------------------------- #
def tiny(seed: int = SEED_BASE + 1) -> Stream:
    """2,000 vertices, 1,000 hyperedges, card U[2,8], Zipf(1.2) popularity;
    one batch of 100 inserts + 100 deletions."""
    return plain_stream("tiny", 2000, 1000, ("uniform", 2, 8), 1.2, 0.0, 1, 100, 100, seed)


def medium(seed: int = SEED_BASE + 2, q: float = 1.0e4, scale: float = 1.0, n_batches: int = 10) -> Stream:
    """1M vertices, 2M hyperedges, card power law 2.5 on [2,64], vertex
    popularity (rank + q)^-1.1; batches of 50k inserts + 50k deletions.
    q = 0 is the literal Zipf(1.1); the default q = 1e4 keeps the hub degree
    low enough for exact hyperedge-triad enumeration."""
    nv = max(64, int(round(1_000_000 * scale)))
    ne = max(16, int(round(2_000_000 * scale)))
    nb = max(1, int(round(50_000 * scale)))
    qq = q * scale if q > 0 else 0.0
    return plain_stream("medium", nv, ne, ("power", 2.5, 2, 64), 1.1, qq, n_batches, nb, nb, seed)


def temporal(seed: int = SEED_BASE + 3, scale: float = 1.0, n_batches: int = 10) -> Stream:
    """500k vertices (uniform popularity), 4M initial hyperedges, card power
    law 2.2 on [2,128], Poisson arrivals at 1e3/s (us timestamps); batches of
    200k arrivals with expiry of hyperedges older than 3600 s; window 600 s."""
    nv = max(256, int(round(500_000 * scale)))
    nbld = max(64, int(round(4_000_000 * scale)))
    bs = max(8, int(round(200_000 * scale)))
    gap = 1000.0 / scale  # keep the same number of hyperedges per window at any scale
    return temporal_stream("temporal", nv, nbld, bs, n_batches, 2.2, 2, 128, gap,
                           int(3_600_000_000), int(600_000_000), seed)


def dyadic(seed: int = SEED_BASE + 6, n_vertices: int = 1_000_000, n_edges: int = 8_000_000, pop_s: float = 0.8,
           pop_q: float = 1.0e3, n_batches: int = 10, n_changes: int = 100_000) -> Stream:
    """A graph (every hyperedge has cardinality 2, no edge twice): n_edges
    distinct edges between vertices of popularity (rank + q)^-s, then batches
    of n_changes / 2 deletions of uniform live edges and n_changes / 2 new
    edges absent from the graph at that point.  The graph special case of
    the incident-vertex family: its type-3 count is the triangle count."""
    rng = np.random.default_rng(seed)
    pop = Popularity(n_vertices, pop_s, pop_q, rng)

    def fresh(n, present_sorted):
        """n new distinct edges (lo, hi) whose keys lo * |V| + hi are absent from present_sorted."""
        got_lo, got_hi, got_keys = [], [], np.zeros(0, np.int64)
        need = n
        while need > 0:
            k = int(need * 1.3) + 16
            a = pop.draw(rng, k).astype(np.int64)
            b = pop.draw(rng, k).astype(np.int64)
            lo, hi = np.minimum(a, b), np.maximum(a, b)
            ok = lo != hi
            lo, hi = lo[ok], hi[ok]
            keys = lo * n_vertices + hi
            _, first = np.unique(keys, return_index=True)
            first = np.sort(first)  # first occurrences, in draw order
            lo, hi, keys = lo[first], hi[first], keys[first]
            new = ~np.isin(keys, present_sorted) & ~np.isin(keys, got_keys)
            lo, hi, keys = lo[new][:need], hi[new][:need], keys[new][:need]
            got_lo.append(lo)
            got_hi.append(hi)
            got_keys = np.concatenate([got_keys, keys])
            need -= len(keys)
        out = np.stack([np.concatenate(got_lo), np.concatenate(got_hi)], axis=1)
        # each edge's members in a random order
        flip = rng.random(len(out)) < 0.5
        out[flip] = out[flip][:, ::-1]
        return out, got_keys

    e0, k0 = fresh(n_edges, np.zeros(0, np.int64))
    initial = _csr(np.full(n_edges, 2, np.int64), e0.reshape(-1).astype(np.uint32))
    st = Stream("dyadic", n_vertices, initial, params=dict(n_edges=n_edges, pop_s=pop_s, pop_q=pop_q, seed=seed))
    live = np.arange(n_edges, dtype=np.int64)
    live_keys = k0
    next_handle = n_edges
    for _ in range(n_batches):
        k = min(n_changes // 2, len(live))
        pick = rng.choice(len(live), size=k, replace=False)
        dels = live[pick]
        keep = np.ones(len(live), dtype=bool)
        keep[pick] = False
        kept_keys = live_keys[keep]
        ne, nk = fresh(n_changes - k, np.sort(kept_keys))
        ih = np.arange(next_handle, next_handle + len(ne), dtype=np.int64)
        next_handle += len(ne)
        live = np.concatenate([live[keep], ih])
        live_keys = np.concatenate([kept_keys, nk])
        st.batches.append(Batch(dels.astype(np.int64), _csr(np.full(len(ne), 2, np.int64),
                                                             ne.reshape(-1).astype(np.uint32)), ih))
    return st


def _uniform_rows(rng: np.random.Generator, cards: np.ndarray, n_vertices: int):
    """Rows of uniform members: every incidence drawn at once, a vertex drawn
    twice in one row kept once (rows ascending); returns (cards, members)."""
    n = len(cards)
    rows = np.repeat(np.arange(n, dtype=np.int64), cards)
    keys = rows * n_vertices + rng.integers(0, n_vertices, size=len(rows), dtype=np.int64)
    keys.sort()
    keep = np.ones(len(keys), dtype=bool)
    keep[1:] = keys[1:] != keys[:-1]
    keys = keys[keep]
    r = keys // n_vertices
    return np.bincount(r, minlength=n).astype(np.int64), (keys - r * n_vertices).astype(np.uint32)


def random_hypergraph(n_edges: int, seed: int = SEED_BASE + 7, alpha: float = 2.5, card_hi: int = 8192,
                      n_batches: int = 4, n_changes: int = 50_000) -> Stream:
    """The paper's random-hypergraph scaling sweep shape: n_edges hyperedges on
    |V| = |E| / 3 vertices of uniform popularity, cardinality power law alpha on
    [2, card_hi] (a vertex drawn twice in a hyperedge is kept once), batches of
    n_changes / 2 uniform deletions + n_changes / 2 new hyperedges."""
    rng = np.random.default_rng(seed)
    nv = max(card_hi, n_edges // 3)
    cards, mem = _uniform_rows(rng, power_law_cards(rng, n_edges, alpha, 2, card_hi), nv)
    st = Stream(f"random[{n_edges}]", nv, _csr(cards, mem),
                params=dict(n_edges=n_edges, alpha=alpha, card_hi=card_hi, seed=seed))
    live = np.arange(n_edges, dtype=np.int64)
    next_handle = n_edges
    for _ in range(n_batches):
        k = min(n_changes // 2, len(live))
        pick = rng.choice(len(live), size=k, replace=False)
        dels = live[pick]
        keep = np.ones(len(live), dtype=bool)
        keep[pick] = False
        ci, mi = _uniform_rows(rng, power_law_cards(rng, n_changes - k, alpha, 2, card_hi), nv)
        ih = np.arange(next_handle, next_handle + len(ci), dtype=np.int64)
        next_handle += len(ci)
        live = np.concatenate([live[keep], ih])
        st.batches.append(Batch(dels.astype(np.int64), _csr(ci, mi), ih))
    return st


@dataclass
class VertexOps:
    edge_ids: np.ndarray   # int64 (hyperedge IDs; horizontal operations keep IDs)
    vertices: np.ndarray   # int64
    insert: np.ndarray     # bool


def vertex_op_batches(st: Stream, n_batches: int, n_ops: int, seed: int = SEED_BASE + 8,
                      pop_s: float = 1.1, pop_q: float = 1.0e4) -> List[VertexOps]:
    """Batches of incident-vertex modifications on the initial hyperedges of
    st (IDs 0..n-1): n_ops / 2 deletions of a member of a uniform hyperedge
    (never its last) and n_ops / 2 insertions of a non-member vertex drawn with
    popularity (rank + q)^-s into a uniform hyperedge; no (hyperedge, vertex)
    pair twice in a batch.  The rows are followed from batch to batch."""
    rng = np.random.default_rng(seed)
    pop = Popularity(st.n_vertices, pop_s, pop_q, rng)
    off = st.initial.offsets.astype(np.int64)
    mem = st.initial.members
    rows = {}

    def row(h):
        if h not in rows:
            rows[h] = set(mem[off[h]:off[h + 1]].tolist())
        return rows[h]

    n = st.initial.n
    out = []
    for _ in range(n_batches):
        used = set()
        e, v, ins = [], [], []
        hd = rng.integers(0, n, size=n_ops)  # candidates for deletions
        for h in hd.tolist():
            if len(e) >= n_ops // 2:
                break
            r = row(h)
            if len(r) < 2:
                continue
            x = int(rng.choice(sorted(r)))
            if (h, x) in used:
                continue
            used.add((h, x))
            r.remove(x)
            e.append(h); v.append(x); ins.append(False)
        hi = rng.integers(0, n, size=n_ops)
        vi = pop.draw(rng, n_ops)
        for h, x in zip(hi.tolist(), vi.tolist()):
            if len(e) >= n_ops:
                break
            r = row(h)
            if x in r or (h, x) in used:
                continue
            used.add((h, x))
            r.add(x)
            e.append(h); v.append(x); ins.append(True)
        order = rng.permutation(len(e))
        out.append(VertexOps(np.array(e, np.int64)[order], np.array(v, np.int64)[order], np.array(ins, bool)[order]))
    return out


def log_uniform_int(rng: np.random.Generator, lo: float, hi: float, size=None) -> np.ndarray:
    return np.round(np.exp(rng.uniform(np.log(lo), np.log(hi), size=size))).astype(np.int64)


def batched_sizes(seed: int = SEED_BASE + 4, n_graphs: int = 256, e_lo: float = 1e3, e_hi: float = 2e5,
                  b_lo: float = 10, b_hi: float = 5e4):
    """(|E_g|, batch size) of every graph of batched(...) with the same arguments."""
    rng = np.random.default_rng(seed)
    sizes = log_uniform_int(rng, e_lo, e_hi, n_graphs)
    bsz = log_uniform_int(rng, b_lo, b_hi, n_graphs)
    return sizes, bsz


def batched(seed: int = SEED_BASE + 4, n_graphs: int = 256, e_lo: float = 1e3, e_hi: float = 2e5,
            b_lo: float = 10, b_hi: float = 5e4, card_hi: int = 256, n_batches: int = 1,
            only: Optional[List[int]] = None) -> List[Stream]:
    """n_graphs independent hypergraphs, |E_g| log-uniform in [e_lo, e_hi],
    |V_g| = |E_g| / 2, card power law 2.5 on [2, card_hi], uniform popularity;
    each with batches of one log-uniform size in [b_lo, b_hi] (60% inserts).
    `only` (graph indices) generates just those graphs, identical to the same
    graphs of the full set."""
    sizes, bsz = batched_sizes(seed, n_graphs, e_lo, e_hi, b_lo, b_hi)
    out = []
    for g in (range(n_graphs) if only is None else only):
        ne = int(sizes[g])
        nv = max(card_hi, ne // 2)
        n_b = int(min(bsz[g], ne))
        n_i = int(round(0.6 * n_b))
        n_d = n_b - n_i
        out.append(plain_stream(f"batched[{g}]", nv, ne, ("power", 2.5, 2, card_hi), 0.0, 0.0,
                                n_batches, n_i, n_d, seed * 1000 + g))
    return out


@dataclass
class Served:
    """Tenants (one Stream each; its batches are the tenant's requests in
    order) and the arrival sequence: (arrival time in us, tenant, index of the
    request in the tenant's stream, reported family)."""
    tenants: List[Stream]
    arrivals: List[tuple]


FAMILIES = ("hyperedge", "incident_vertex", "temporal")


def tenant_stream(name: str, n_vertices: int, n_edges: int, alpha: float, card_hi: int, pop_s: float, pop_q: float,
                  sizes: List[tuple], mean_gap_us: float, window_us: int, seed: int) -> Stream:
    """A tenant: n_edges initial hyperedges with Poisson timestamps, then one
    batch per (n_ins, n_del) in `sizes`: n_del deletions uniform over the live
    hyperedges and n_ins new ones from the same distribution, stamped after
    every earlier hyperedge of the tenant."""
    rng = np.random.default_rng(seed)
    pop = Popularity(n_vertices, pop_s, pop_q, rng)
    hi = min(card_hi, n_vertices)
    c0 = power_law_cards(rng, n_edges, alpha, 2, hi)
    ts0 = poisson_times(rng, n_edges, mean_gap_us)
    initial = _csr(c0, draw_members(rng, c0, pop), ts0)
    st = Stream(name, n_vertices, initial, window=int(window_us),
                params=dict(n_edges=n_edges, alpha=alpha, card_hi=card_hi, pop_s=pop_s, pop_q=pop_q, seed=seed))
    live = np.arange(n_edges, dtype=np.int64)
    next_handle = n_edges
    t_last = int(ts0[-1]) if n_edges else 0
    for n_ins, n_del in sizes:
        k = min(int(n_del), len(live))
        pick = rng.choice(len(live), size=k, replace=False)
        dels = live[pick]
        keep = np.ones(len(live), dtype=bool)
        keep[pick] = False
        ci = power_law_cards(rng, int(n_ins), alpha, 2, hi)
        ts = poisson_times(rng, int(n_ins), mean_gap_us, t_last)
        if n_ins:
            t_last = int(ts[-1])
        ins = _csr(ci, draw_members(rng, ci, pop), ts)
        ih = np.arange(next_handle, next_handle + int(n_ins), dtype=np.int64)
        next_handle += int(n_ins)
        live = np.concatenate([live[keep], ih])
        st.batches.append(Batch(dels.astype(np.int64), ins, ih))
    return st


def _tenant_sizes(rng, n_tenants, total_edges, size_lo, size_hi) -> np.ndarray:
    w = np.exp(rng.uniform(np.log(size_lo), np.log(size_hi), n_tenants))
    return np.maximum(np.round(w / w.sum() * total_edges).astype(np.int64), 64)


def served_tenant_sizes(seed: int = SEED_BASE + 5, n_tenants: int = 64, total_edges: float = 20e6,
                        size_lo: float = 1e4, size_hi: float = 1e6) -> np.ndarray:
    """Initial hyperedges of every tenant of served(...) with the same arguments."""
    return _tenant_sizes(np.random.default_rng(seed), n_tenants, total_edges, size_lo, size_hi)


def served(seed: int = SEED_BASE + 5, n_tenants: int = 64, total_edges: float = 20e6, n_requests: int = 256,
           rate_per_s: float = 1000.0, req_lo: float = 1, req_hi: float = 1e5, card_hi: int = 4096,
           pop_q: float = 3.0e3, size_lo: float = 1e4, size_hi: float = 1e6,
           window_us: int = 600_000_000, only: Optional[List[int]] = None) -> Served:
    """64 tenants with sizes log-uniform in [size_lo, size_hi] rescaled to
    total_edges hyperedges, |V_t| = |E_t| / 2, cardinality power law 2.0 on
    [2, card_hi], popularity (rank + pop_q)^-1.3, Poisson timestamps (1e3/s,
    us) and window 600 s; n_requests requests with Poisson arrivals at
    rate_per_s, tenant uniform, size log-uniform in [req_lo, req_hi] (half
    inserts, half deletions), reported family uniform.  `only` (tenant
    indices) generates just those tenants' streams (the others are None),
    identical to the same tenants of the full set."""
    rng = np.random.default_rng(seed)
    n_e = _tenant_sizes(rng, n_tenants, total_edges, size_lo, size_hi)
    tenant_of = rng.integers(0, n_tenants, n_requests)
    sizes = log_uniform_int(rng, req_lo, req_hi, n_requests)
    fam = rng.integers(0, 3, n_requests)
    gaps = rng.exponential(1e6 / rate_per_s, n_requests)
    t_arr = np.cumsum(gaps)
    per = [[] for _ in range(n_tenants)]
    arrivals = []
    for r in range(n_requests):
        t = int(tenant_of[r])
        n = int(sizes[r])
        n_ins = (n + 1) // 2
        per[t].append((n_ins, n - n_ins))
        arrivals.append((float(t_arr[r]), t, len(per[t]) - 1, FAMILIES[int(fam[r])]))
    tenants = []
    for t in range(n_tenants):
        if only is not None and t not in only:
            tenants.append(None)
            continue
        ne = int(n_e[t])
        nv = max(64, ne // 2)
        tenants.append(tenant_stream(f"served[{t}]", nv, ne, 2.0, card_hi, 1.3, pop_q, per[t], 1000.0,
                                     window_us, seed * 1000 + t))
    return Served(tenants, arrivals)
