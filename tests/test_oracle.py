"""Pins of the CPU oracle against things other than itself.

* the numbers of classes the paper states (26 hyperedge triads, 96 temporal);
* hand-worked examples (tests/golden/hand_examples.json);
* brute force over all hyperedge triples / all witness assignments on tiny
  random hypergraphs, written straight from the definitions with Python sets;
* the graph special case of incident-vertex type 3 against the textbook
  triangle count trace(A^3) / 6 (numpy matrix product);
* invariants: incremental delta == recount difference, insert-then-delete
  restores every count, relabelling vertices or IDs changes nothing, a window
  covering every span makes the temporal counts collapse onto the hyperedge
  counts;
* the ID-reuse rule of the paper's Fig. 5 example.
"""
import itertools
import json
import os

import numpy as np
import pytest

from oracle import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")
REGION_SETS = [{0}, {1}, {2}, {0, 1}, {1, 2}, {0, 2}, {0, 1, 2}]  # bit i -> labels it lies in


def csr(rows):
    off = np.zeros(len(rows) + 1, np.uint64)
    off[1:] = np.cumsum([len(r) for r in rows])
    mem = np.array([v for r in rows for v in r], np.uint32)
    return off, mem


def graph(rows, nv=None, ts=None, window=0):
    nv = nv or (max((max(r) for r in rows if r), default=0) + 1)
    off, mem = csr(rows)
    return O.OracleGraph(nv, off, mem, ts=ts, window=window)


# ---------------------------------------------------------------- brute force
def pattern(A, B, C):
    sets = [set(A), set(B), set(C)]
    code = 0
    for i, labs in enumerate(REGION_SETS):
        inside = set.intersection(*[sets[l] for l in labs])
        outside = set().union(*[sets[l] for l in range(3) if l not in labs])
        if inside - outside:
            code |= 1 << i
    return code


def canonical(A, B, C):
    return min(pattern(*p) for p in itertools.permutations((A, B, C)))


def connected(A, B, C):
    return sum(bool(set(x) & set(y)) for x, y in ((A, B), (B, C), (A, C))) >= 2


def brute_he(rows):
    out = {}
    for a, b, c in itertools.combinations(range(len(rows)), 3):
        if connected(rows[a], rows[b], rows[c]):
            k = canonical(rows[a], rows[b], rows[c])
            out[k] = out.get(k, 0) + 1
    return out


def brute_tmp(rows, ts, window):
    out = {}
    for tri in itertools.combinations(range(len(rows)), 3):
        o = sorted(tri, key=lambda i: (ts[i], i))  # arrival sequence = row index here
        if ts[o[2]] - ts[o[0]] > window:
            continue
        if connected(*(rows[i] for i in o)):
            k = pattern(*(rows[i] for i in o))
            out[k] = out.get(k, 0) + 1
    return out


def brute_iv(rows):
    """Enumerate vertex triples and one witness hyperedge per pair."""
    verts = sorted({v for r in rows for v in r})
    t = [0, 0, 0]
    for u, v, w in itertools.combinations(verts, 3):
        wit = [[i for i, r in enumerate(rows) if x in r and y in r] for x, y in ((u, v), (v, w), (u, w))]
        for e in itertools.product(*wit):
            distinct = len(set(e))
            t[{1: 0, 2: 1, 3: 2}[distinct]] += 1
    return t


def as_dict(counts, codes):
    return {int(codes[i]): int(c) for i, c in enumerate(counts) if c}


def random_rows(rng, n, nv, lo, hi, dup_frac=0.1):
    rows = []
    for _ in range(n):
        if rows and rng.random() < dup_frac:
            rows.append(list(rows[rng.integers(len(rows))]))
            continue
        k = int(rng.integers(lo, hi + 1))
        p = np.arange(1, nv + 1, dtype=float) ** -1.0
        rows.append(sorted(rng.choice(nv, size=min(k, nv), replace=False, p=p / p.sum()).tolist()))
    return rows


# ---------------------------------------------------------------- class tables
def test_class_counts_match_paper():
    he = O.he_class_codes()
    assert len(he) == 30
    # identical-set patterns: some pair of labels with no region separating them
    def needs_identical(code):
        for s, t in ((0, 1), (1, 2), (0, 2)):
            if not any((code >> i & 1) and ((s in R) != (t in R)) for i, R in enumerate(REGION_SETS)):
                return True
        return False
    non_degenerate = [c for c in he if not needs_identical(int(c))]
    assert len(non_degenerate) == 26  # "26 unique hypergraph triads" (Sec. II)
    assert len(O.tmp_class_codes()) == 96  # "96 temporal hypergraph motifs" (Sec. VI)
    assert list(he) == sorted(he)


def test_hand_examples():
    gold = json.load(open(GOLD))
    he_codes = O.he_class_codes()
    tm_codes = O.tmp_class_codes()
    for ex in gold["hyperedge"]:
        g = graph(ex["rows"])
        assert as_dict(g.he_counts(), he_codes) == {int(k): v for k, v in ex["codes"].items()}, ex
    for ex in gold["incident_vertex"]:
        g = graph(ex["rows"])
        assert g.iv_counts().tolist() == ex["counts"], ex
    for ex in gold["temporal"]:
        g = graph(ex["rows"], ts=np.array(ex["ts"], np.int64), window=ex["window"])
        assert as_dict(g.temporal_counts(), tm_codes) == {int(k): v for k, v in ex["codes"].items()}, ex


# ---------------------------------------------------------------- brute force pins
@pytest.mark.parametrize("seed", range(6))
def test_he_matches_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    rows = random_rows(rng, 28, 14, 1, 5)
    g = graph(rows, nv=14)
    assert as_dict(g.he_counts(), O.he_class_codes()) == brute_he(rows)


@pytest.mark.parametrize("seed", range(6))
def test_temporal_matches_brute_force(seed):
    rng = np.random.default_rng(200 + seed)
    rows = random_rows(rng, 26, 12, 1, 5)
    ts = np.sort(rng.integers(0, 40, size=len(rows))).astype(np.int64)  # many ties
    window = int(rng.integers(0, 30))
    g = graph(rows, nv=12, ts=ts, window=window)
    assert as_dict(g.temporal_counts(), O.tmp_class_codes()) == brute_tmp(rows, ts, window)


@pytest.mark.parametrize("seed", range(6))
def test_iv_matches_witness_brute_force(seed):
    rng = np.random.default_rng(300 + seed)
    rows = random_rows(rng, 14, 9, 2, 5, dup_frac=0.2)
    g = graph(rows, nv=9)
    assert g.iv_counts().tolist() == brute_iv(rows)


def test_iv_graph_case_is_triangle_count():
    rng = np.random.default_rng(7)
    nv = 60
    pairs = set()
    while len(pairs) < 400:
        u, v = sorted(rng.choice(nv, 2, replace=False).tolist())
        pairs.add((u, v))
    rows = [list(p) for p in sorted(pairs)]
    A = np.zeros((nv, nv), dtype=np.int64)
    for u, v in rows:
        A[u, v] = A[v, u] = 1
    tri = int(np.trace(A @ A @ A)) // 6
    assert graph(rows, nv=nv).iv_counts().tolist() == [0, 0, tri]


def test_temporal_wide_window_collapses_to_hyperedge_counts():
    rng = np.random.default_rng(11)
    rows = random_rows(rng, 60, 25, 1, 6)
    ts = np.sort(rng.integers(0, 1000, size=len(rows))).astype(np.int64)
    g = graph(rows, nv=25, ts=ts, window=10**9)
    tm = g.temporal_counts()
    he = g.he_counts()
    tcodes, hcodes = O.tmp_class_codes(), O.he_class_codes()
    folded = np.zeros(30, np.uint64)
    for i, c in enumerate(tcodes):
        folded[O.he_class_of_code(int(c))] += tm[i]
    assert (folded == he).all()
    assert int(he.sum()) > 0


# ---------------------------------------------------------------- batch semantics
def test_id_reuse_follows_fig5():
    # Fig. 5: after deleting h1, h5, h6 and h10 the j-th inserting thread takes
    # the j-th available block; thread 2 lands on h5.
    rows = [[i, i + 1] for i in range(12)]
    g = graph(rows, nv=20)
    st, ids = g.apply_batch([10, 1, 6, 5], *csr([[0, 3], [1, 4]]))
    assert st == O.OK and ids.tolist() == [1, 5]
    st, ids = g.apply_batch([], *csr([[2, 7], [3, 9], [4, 11], [5, 8]]))
    assert st == O.OK and ids.tolist() == [6, 10, 12, 13]
    assert g.next_id == 14


def test_batch_errors_leave_state_unchanged():
    rows = [[0, 1], [1, 2], [2, 3]]
    g = graph(rows, nv=5, ts=np.array([1, 2, 3], np.int64), window=10)
    before = (g.off.copy(), g.mem.copy(), g.live.copy())
    assert g.apply_batch([7], *csr([]))[0] == O.ENOENT
    assert g.apply_batch([1, 1], *csr([]))[0] == O.EDUP
    assert g.apply_batch([], *csr([[1, 1]]), np.array([5]))[0] == O.EINVAL
    assert g.apply_batch([], *csr([[]]), np.array([5]))[0] == O.EINVAL
    assert g.apply_batch([], *csr([[9]]), np.array([5]))[0] == O.EINVAL
    assert g.apply_batch([], *csr([[1, 2]]), np.array([2]))[0] == O.EORDER
    assert g.apply_batch([], *csr([[1, 2], [2, 3]]), np.array([9, 8]))[0] == O.EORDER
    # every rejected batch above left the rows, members and live flags as they were
    assert (g.off == before[0]).all() and (g.mem == before[1]).all() and (g.live == before[2]).all()
    assert g.next_id == 3 and g.last_ts == 3
    st, _ = g.apply_batch([0], *csr([]))
    assert st == O.OK and g.live.tolist() == [0, 1, 1]
    assert g.apply_batch([0], *csr([]))[0] == O.ENOENT  # already deleted


def _batch(rng, g, n_del, n_ins, nv, card):
    live = g.live_ids()
    dels = rng.choice(live, size=min(n_del, len(live)), replace=False)
    rows = random_rows(rng, n_ins, nv, 1, card)
    return dels, rows


@pytest.mark.parametrize("seed", range(5))
def test_delta_by_definition_equals_recount(seed):
    rng = np.random.default_rng(400 + seed)
    nv = 40
    rows = random_rows(rng, 80, nv, 1, 5)
    ts = np.sort(rng.integers(0, 500, size=len(rows))).astype(np.int64)
    g = graph(rows, nv=nv, ts=ts, window=120)
    he, tm, iv = g.he_counts(), g.temporal_counts(), g.iv_counts()
    for _ in range(3):
        dels, ins = _batch(rng, g, 12, 15, nv, 5)
        t_ins = np.sort(rng.integers(g.last_ts, g.last_ts + 200, size=len(ins))).astype(np.int64)
        old = g.copy()
        st, ids = g.apply_batch(dels, *csr(ins), t_ins)
        assert st == O.OK
        dhe, dtm = O.delta_by_definition(old, g, dels, ids)
        he, tm = he + dhe, tm + dtm
        assert (he == g.he_counts()).all()
        assert (tm == g.temporal_counts()).all()
        iv = g.iv_counts()
    assert int(he.sum()) > 0 and int(tm.sum()) > 0 and int(iv.sum()) > 0


def test_insert_then_delete_restores_counts():
    rng = np.random.default_rng(5)
    nv = 30
    g = graph(random_rows(rng, 70, nv, 1, 5), nv=nv)
    he0, iv0 = g.he_counts(), g.iv_counts()
    st, ids = g.apply_batch([], *csr(random_rows(rng, 20, nv, 1, 6)))
    assert st == O.OK
    assert not (g.he_counts() == he0).all()
    st, _ = g.apply_batch(ids, *csr([]))
    assert st == O.OK
    assert (g.he_counts() == he0).all() and (g.iv_counts() == iv0).all()


def test_relabelling_invariance():
    rng = np.random.default_rng(9)
    nv = 35
    rows = random_rows(rng, 90, nv, 1, 6)
    ts = np.sort(rng.integers(0, 300, size=len(rows))).astype(np.int64)
    g = graph(rows, nv=nv, ts=ts, window=80)
    vp = rng.permutation(nv)
    order = rng.permutation(len(rows))
    # relabel vertices and re-number hyperedges (keeping arrival order by ts)
    rows2 = [sorted(int(vp[v]) for v in rows[i]) for i in order]
    ts2 = ts[order]
    srt = np.argsort(ts2, kind="stable")
    rows2 = [rows2[i] for i in srt]
    ts2 = ts2[srt]
    g2 = graph(rows2, nv=nv, ts=ts2, window=80)
    assert (g.he_counts() == g2.he_counts()).all()
    assert (g.iv_counts() == g2.iv_counts()).all()
    # temporal classes depend on tie order only through equal timestamps
    if len(np.unique(ts)) == len(ts):
        assert (g.temporal_counts() == g2.temporal_counts()).all()


# ------------------------------------------- incident-vertex delta by definition
def _iv_brute_sums(rows, keys):
    """The two restricted sums written straight from the definitions with Python
    sets: m_p and w_p per listed pair, and every vertex triangle with a listed pair."""
    listed = {(int(k) >> 32, int(k) & 0xffffffff) for k in keys}
    m, w = {}, {}
    for r in rows:
        for a, b in itertools.combinations(sorted(r), 2):
            m[(a, b)] = m.get((a, b), 0) + 1
            w[(a, b)] = w.get((a, b), 0) + len(r) - 2
    s = sum(m.get(p, 0) * w.get(p, 0) for p in listed)
    verts = sorted({v for r in rows for v in r})
    x = 0
    for a, b, c in itertools.combinations(verts, 3):
        if {(a, b), (b, c), (a, c)} & listed:
            x += m.get((a, b), 0) * m.get((b, c), 0) * m.get((a, c), 0)
    return s, x


@pytest.mark.parametrize("seed", range(4))
def test_iv_partial_sums_brute_force(seed):
    rng = np.random.default_rng(700 + seed)
    nv = 14
    rows = random_rows(rng, 25, nv, 1, 5)
    g = graph(rows, nv=nv)
    pick = rng.choice(len(rows), size=5, replace=False)
    keys = g.pairs_of(pick)
    want = {(a, b) for i in pick for a, b in itertools.combinations(sorted(rows[i]), 2)}
    assert {(int(k) >> 32, int(k) & 0xffffffff) for k in keys} == want
    assert list(keys) == sorted(keys)
    s, x = g.iv_partial(keys)
    assert (int(s), int(x)) == _iv_brute_sums(rows, keys)


def test_iv_partial_all_pairs_equals_closed_forms():
    # every pair listed: the sums are the full ones, T2 + 3 T1 and T1 + T2 + T3
    rng = np.random.default_rng(77)
    nv = 30
    rows = random_rows(rng, 60, nv, 1, 6)
    g = graph(rows, nv=nv)
    t1, t2, t3 = (int(v) for v in g.iv_counts())
    s, x = g.iv_partial(g.pairs_of(np.arange(len(rows))))
    assert int(s) == t2 + 3 * t1
    assert int(x) == t1 + t2 + t3


@pytest.mark.parametrize("seed", range(4))
def test_iv_delta_by_definition_equals_recount(seed):
    rng = np.random.default_rng(800 + seed)
    nv = 35
    g = graph(random_rows(rng, 90, nv, 1, 6), nv=nv)
    for _ in range(3):
        dels, ins = _batch(rng, g, 15, 12, nv, 6)
        old = g.copy()
        st, ids = g.apply_batch(dels, *csr(ins))
        assert st == O.OK
        d = O.iv_delta_by_definition(old, g, dels, ids)
        with np.errstate(over="ignore"):
            want = g.iv_counts() - old.iv_counts()
        assert (d == want).all(), (d, want)
    # a plain deletion batch and a plain insert batch
    old = g.copy()
    dels = g.live_ids()[:7]
    assert g.apply_batch(dels, *csr([]))[0] == O.OK
    with np.errstate(over="ignore"):
        assert (O.iv_delta_by_definition(old, g, dels, []) == g.iv_counts() - old.iv_counts()).all()


# ------------------------------------------------- horizontal (vertex) operations
def random_vertex_ops(rng, g, n_edges, nv, max_per_edge=3):
    """Valid ops on n_edges live hyperedges: some members deleted (one always
    kept), some non-members inserted."""
    eids, verts, ins = [], [], []
    for h in rng.choice(g.live_ids(), size=min(n_edges, len(g.live_ids())), replace=False).tolist():
        row = g.row(h).tolist()
        n_del = int(rng.integers(0, min(max_per_edge, len(row) - 1) + 1))
        for v in rng.choice(row, size=n_del, replace=False).tolist():
            eids.append(h); verts.append(v); ins.append(1 == 0)
        outside = [v for v in range(nv) if v not in row]
        n_ins = int(rng.integers(0 if n_del else 1, max_per_edge + 1))
        for v in rng.choice(outside, size=min(n_ins, len(outside)), replace=False).tolist():
            eids.append(h); verts.append(v); ins.append(True)
    order = rng.permutation(len(eids))
    return (np.array(eids, np.int64)[order], np.array(verts, np.int64)[order], np.array(ins, bool)[order])


def _rows_of(g):
    return [g.row(i).tolist() for i in range(g.n_slots) if g.live[i]]


@pytest.mark.parametrize("seed", range(4))
def test_vertex_ops_brute_force(seed):
    """Counts after a batch of vertex insertions/deletions equal brute force on
    the modified hyperedge sets (timestamps and arrival order kept)."""
    rng = np.random.default_rng(900 + seed)
    nv = 12
    rows = random_rows(rng, 14, nv, 1, 4)
    ts = np.sort(rng.integers(0, 60, size=len(rows))).astype(np.int64)
    g = graph(rows, nv=nv, ts=ts, window=25)
    e, v, ins = random_vertex_ops(rng, g, 5, nv)
    st, mod = g.apply_vertex_ops(e, v, ins)
    assert st == O.OK and sorted(set(e.tolist())) == mod.tolist()
    new_rows = _rows_of(g)
    for h in range(len(rows)):
        want = set(rows[h]) | {int(x) for x, i, y in zip(v, ins, e) if i and y == h}
        want -= {int(x) for x, i, y in zip(v, ins, e) if not i and y == h}
        assert new_rows[h] == sorted(want)
    assert as_dict(g.he_counts(), O.he_class_codes()) == brute_he(new_rows)
    assert as_dict(g.temporal_counts(), O.tmp_class_codes()) == brute_tmp(new_rows, ts, 25)
    assert g.iv_counts().tolist() == brute_iv(new_rows)


def test_vertex_ops_inverse_and_delete_reinsert():
    rng = np.random.default_rng(31)
    nv = 30
    rows = random_rows(rng, 60, nv, 1, 6)
    g = graph(rows, nv=nv)
    he0, iv0 = g.he_counts(), g.iv_counts()
    e, v, ins = random_vertex_ops(rng, g, 12, nv)
    old = g.copy()
    st, mod = g.apply_vertex_ops(e, v, ins)
    assert st == O.OK
    he1, iv1 = g.he_counts(), g.iv_counts()
    assert not (he1 == he0).all()
    # the same change as deleting the modified hyperedges and inserting their new rows
    g2 = old.copy()
    new = [g.row(h).tolist() for h in mod.tolist()]
    st2, _ = g2.apply_batch(mod, *csr(new))
    assert st2 == O.OK
    assert (g2.he_counts() == he1).all() and (g2.iv_counts() == iv1).all()
    # delta by definition over the modified IDs on both sides
    dhe, _ = O.delta_by_definition(old, g, mod, mod)
    with np.errstate(over="ignore"):
        assert (he0 + dhe == he1).all()
        assert (O.iv_delta_by_definition(old, g, mod, mod) == iv1 - iv0).all()
    # the inverse ops restore every count and row
    st, _ = g.apply_vertex_ops(e, v, ~ins)
    assert st == O.OK
    assert (g.he_counts() == he0).all() and (g.iv_counts() == iv0).all()
    assert _rows_of(g) == _rows_of(old)


def test_vertex_ops_errors_leave_state_unchanged():
    rows = [[0, 1], [1, 2], [2, 3, 4]]
    g = graph(rows, nv=6, ts=np.array([1, 2, 3], np.int64), window=10)
    assert g.apply_batch([1], *csr([]))[0] == O.OK  # ID 1 is dead now
    before = (g.off.copy(), g.mem.copy(), g.live.copy())
    cases = [
        (O.ENOENT, ([1], [0], [True])),           # hyperedge not live
        (O.ENOENT, ([7], [0], [True])),           # never used
        (O.EINVAL, ([0], [6], [True])),           # vertex out of range
        (O.EINVAL, ([0], [1], [True])),           # already a member
        (O.EINVAL, ([0], [3], [False])),          # not a member
        (O.EINVAL, ([0, 0], [0, 1], [False, False])),  # would leave it empty
        (O.EINVAL, ([2, 2], [5, 5], [True, True])),    # the same op twice
        (O.EINVAL, ([2, 2], [3, 3], [False, True])),   # the same pair twice
    ]
    for code, (e, v, i) in cases:
        assert g.apply_vertex_ops(e, v, i)[0] == code, (e, v, i)
        assert (g.off == before[0]).all() and (g.mem == before[1]).all() and (g.live == before[2]).all()
    st, mod = g.apply_vertex_ops([2, 0], [4, 5], [False, True])
    assert st == O.OK and mod.tolist() == [0, 2]
    assert g.row(0).tolist() == [0, 1, 5] and g.row(2).tolist() == [2, 3]
