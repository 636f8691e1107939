"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Counts are integers and must match exactly (tolerance 0); assigned IDs and the
exported incidence store must match the oracle's rebuilt maps.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2512_21009_amd import workloads as W

from .gpu_harness import Pair, compare_counts, compare_store, dev

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")
ALL = ("hyperedge", "incident_vertex", "temporal")


def _stream_from_rows(rows, ts=None, window=0, nv=None):
    nv = nv or (max(max(r) for r in rows) + 1)
    off = np.zeros(len(rows) + 1, np.uint64)
    off[1:] = np.cumsum([len(r) for r in rows])
    mem = np.array([v for r in rows for v in r], np.uint32)
    return W.Stream("rows", nv, W.CSR(off, mem, None if ts is None else np.asarray(ts, np.int64)), window=window)


def test_hand_examples(gpu_lib):
    gold = json.load(open(GOLD))
    for ex in gold["hyperedge"] + gold["incident_vertex"]:
        p = Pair(_stream_from_rows(ex["rows"]), track=("hyperedge", "incident_vertex"))
        compare_counts(p.g, p.o, p.track, f"hand {ex['rows']}")
        p.close()
    for ex in gold["temporal"]:
        p = Pair(_stream_from_rows(ex["rows"], ts=ex["ts"], window=ex["window"]), track=("temporal",))
        compare_counts(p.g, p.o, p.track, f"hand temporal {ex['rows']}")
        p.close()


def _random_stream(seed, n_edges=120, nv=50, n_batches=3, n_ins=25, n_del=20, temporal=True, card=(1, 6), s=1.0):
    if temporal:
        st = W.temporal_stream("rnd", nv, n_edges, n_ins, n_batches, 2.0, card[0], card[1], 7.0, 700, 150, seed,
                               pop_s=s)
        return st
    return W.plain_stream("rnd", nv, n_edges, ("uniform", card[0], card[1]), s, 0.0, n_batches, n_ins, n_del, seed)


@pytest.mark.parametrize("seed", range(4))
def test_random_small_all_families(gpu_lib, seed):
    st = _random_stream(1000 + seed)
    p = Pair(st, track=ALL)
    compare_counts(p.g, p.o, ALL, "build")
    compare_store(p.g, p.o, "build")
    for k, b in enumerate(st.batches):
        p.apply(b, f"batch {k}")
        compare_store(p.g, p.o, f"batch {k}")
        compare_counts(p.g, p.o, ALL, f"batch {k}")
    p.close()


@pytest.mark.parametrize("seed", range(3))
def test_random_plain_he_iv(gpu_lib, seed):
    st = _random_stream(2000 + seed, n_edges=300, nv=120, n_batches=3, n_ins=60, n_del=70, temporal=False, card=(1, 9))
    p = Pair(st, track=("hyperedge", "incident_vertex"))
    compare_counts(p.g, p.o, p.track, "build")
    for k, b in enumerate(st.batches):
        p.apply(b, f"batch {k}")
        compare_store(p.g, p.o, f"batch {k}")
        compare_counts(p.g, p.o, p.track, f"batch {k}")
    p.close()


def test_tiny_config(gpu_lib):
    """2,000 vertices, 1,000 hyperedges, card U[2,8], Zipf(1.2); 100 + 100 updates."""
    st = W.tiny()
    p = Pair(st, track=("hyperedge", "incident_vertex"))
    compare_counts(p.g, p.o, p.track, "tiny build")
    p.apply(st.batches[0], "tiny batch")
    compare_store(p.g, p.o, "tiny batch")
    compare_counts(p.g, p.o, p.track, "tiny batch")
    p.close()


def test_hub_heavy_large_centres(gpu_lib):
    """A strong hub forces centres into the large-neighbourhood kernel and
    neighbours into the binary-search 2-hop path; cards above 64 exercise the
    workgroup sort."""
    st = W.plain_stream("hub", 400, 700, ("power", 1.6, 2, 150), 1.3, 0.0, 2, 80, 90, W.SEED_BASE + 77)
    p = Pair(st, track=("hyperedge", "incident_vertex"))
    compare_counts(p.g, p.o, p.track, "hub build")
    for k, b in enumerate(st.batches):
        p.apply(b, f"hub batch {k}")
        compare_store(p.g, p.o, f"hub batch {k}")
        compare_counts(p.g, p.o, p.track, f"hub batch {k}")
    p.close()


def test_medium_scaled(gpu_lib):
    """Medium shape (power-law 2.5 cards on [2,64], Zipf-Mandelbrot popularity) at 1/1000 scale."""
    st = W.medium(scale=0.001, n_batches=3)
    p = Pair(st, track=("hyperedge", "incident_vertex"))
    compare_counts(p.g, p.o, p.track, "medium build")
    for k, b in enumerate(st.batches):
        p.apply(b, f"medium batch {k}")
        compare_counts(p.g, p.o, p.track, f"medium batch {k}")
    compare_store(p.g, p.o, "medium end")
    p.close()


def test_temporal_scaled(gpu_lib):
    """Temporal shape (power-law 2.2 cards on [2,128], Poisson arrivals, 3600 s
    expiry, 600 s window) at 1/500 scale."""
    st = W.temporal(scale=0.002, n_batches=3)
    p = Pair(st, track=("temporal",))
    compare_counts(p.g, p.o, p.track, "temporal build")
    for k, b in enumerate(st.batches):
        p.apply(b, f"temporal batch {k}")
        compare_counts(p.g, p.o, p.track, f"temporal batch {k}")
    compare_store(p.g, p.o, "temporal end")
    p.close()


def test_edge_cases(gpu_lib):
    rows = [[0, 1], [1, 2], [2, 3], [0, 2, 3], [4], [1, 4, 5]]
    st = _stream_from_rows(rows, nv=8)
    p = Pair(st, track=("hyperedge", "incident_vertex"))
    compare_counts(p.g, p.o, p.track, "edge build")
    empty = W.CSR(np.zeros(1, np.uint64), np.zeros(0, np.uint32))
    # deletions only, then everything, then inserts only (fresh + reused IDs)
    p.apply(W.Batch(np.array([1, 4]), empty, np.zeros(0, np.int64)), "del only")
    compare_counts(p.g, p.o, p.track, "del only")
    p.apply(W.Batch(np.array([0, 2, 3, 5]), empty, np.zeros(0, np.int64)), "del all")
    compare_counts(p.g, p.o, p.track, "del all")
    compare_store(p.g, p.o, "del all")
    ins = W.CSR(np.array([0, 3, 5, 6, 9], np.uint64), np.array([7, 1, 2, 0, 1, 6, 2, 1, 0], np.uint32))
    p.apply(W.Batch(np.zeros(0, np.int64), ins, np.arange(100, 104)), "ins only")
    compare_counts(p.g, p.o, p.track, "ins only")
    compare_store(p.g, p.o, "ins only")
    p.close()


def test_errors_leave_state_unchanged(gpu_lib):
    from paper_2512_21009_amd import hgt
    rows = [[0, 1], [1, 2], [2, 3], [0, 3]]
    st = _stream_from_rows(rows, ts=[1, 2, 3, 4], window=10, nv=5)
    p = Pair(st, track=("hyperedge", "temporal"))
    before = (p.g.triad_counts("hyperedge"), p.g.triad_counts("temporal"), p.g.export_h2v()[1].tolist())
    g = p.g
    cases = [
        (hgt.ENOENT, dict(del_ids=dev([9], np.int32))),
        (hgt.EDUP, dict(del_ids=dev([1, 1], np.int32))),
        (hgt.EINVAL, dict(ins_offsets=dev([0, 2], np.int64), ins_members=dev([1, 1], np.int32), ins_ts=dev([5], np.int64))),
        (hgt.EINVAL, dict(ins_offsets=dev([0, 1], np.int64), ins_members=dev([7], np.int32), ins_ts=dev([5], np.int64))),
        (hgt.EORDER, dict(ins_offsets=dev([0, 2], np.int64), ins_members=dev([1, 2], np.int32), ins_ts=dev([3], np.int64))),
        (hgt.EORDER, dict(ins_offsets=dev([0, 2, 4], np.int64), ins_members=dev([1, 2, 2, 3], np.int32),
                          ins_ts=dev([9, 8], np.int64))),
    ]
    for code, kw in cases:
        rc, _ = g.apply_batch(raise_on_error=False, **kw)
        assert rc == code, (rc, code, kw)
        after = (g.triad_counts("hyperedge"), g.triad_counts("temporal"), g.export_h2v()[1].tolist())
        assert after == before
    assert g.sync() != hgt.OK  # sticky status reports the first error
    p.close()


@pytest.mark.parametrize("stage", [1, 2, 3])
def test_every_kernel_path(gpu_lib, monkeypatch, stage):
    """Force every centre past the first `stage` stages of the histogram kernel
    (1: 148 KB LDS arena, 2: global-memory arena, 3: 2-hop kernel) and check
    the same results."""
    monkeypatch.setenv("HGT_FORCE_STAGE", str(stage))
    monkeypatch.setenv("HGT_SKIP_LDS148", "0")  # keep the 148 KB stage in the sequence
    st = _random_stream(3000 + stage, n_edges=250, nv=90, n_batches=2, n_ins=50, n_del=60, temporal=False,
                        card=(1, 9))
    p = Pair(st, track=("hyperedge",))
    compare_counts(p.g, p.o, p.track, f"stage {stage} build")
    for k, b in enumerate(st.batches):
        p.apply(b, f"stage {stage} batch {k}")
        compare_counts(p.g, p.o, p.track, f"stage {stage} batch {k}")
    p.close()
    st = W.medium(scale=0.0005, n_batches=2)
    p = Pair(st, track=("hyperedge",))
    compare_counts(p.g, p.o, p.track, f"stage {stage} medium build")
    for k, b in enumerate(st.batches):
        p.apply(b, f"stage {stage} medium batch {k}")
        compare_counts(p.g, p.o, p.track, f"stage {stage} medium batch {k}")
    p.close()


@pytest.mark.parametrize("agg", ["0", "1"])
def test_pair_phase_paths(gpu_lib, monkeypatch, agg):
    """Intersecting neighbour pairs aggregated per shared vertex (1, with long
    runs counted by histogram and pairs sharing several vertices corrected) or
    enumerated per run (0); the dense hub graph sends most centres to the
    enumerating path either way.  Same counts as the oracle."""
    monkeypatch.setenv("HGT_PAIR_AGG", agg)
    for st in (W.medium(scale=0.001, n_batches=2),
               W.plain_stream("hub", 400, 700, ("power", 1.6, 2, 150), 1.3, 0.0, 2, 80, 90, W.SEED_BASE + 79)):
        p = Pair(st, track=("hyperedge",))
        for k, b in enumerate(st.batches):
            p.apply(b, f"pair phase {agg} batch {k}")
            compare_counts(p.g, p.o, p.track, f"pair phase {agg} batch {k}")
        p.close()


def test_incident_vertex_without_maps(gpu_lib, monkeypatch):
    """Every incident-vertex owner evaluated pair by pair without a clique map
    (the path of owners too large for the global stage's arena): same counts."""
    monkeypatch.setenv("HGT_IV_DIRECT", "1")
    for st in (_random_stream(4100, n_edges=200, nv=70, n_batches=2, n_ins=40, n_del=40, temporal=False, card=(1, 7)),
               W.medium(scale=0.0005, n_batches=2)):
        p = Pair(st, track=("incident_vertex",))
        for k, b in enumerate(st.batches):
            p.apply(b, f"iv direct batch {k}")
            compare_counts(p.g, p.o, p.track, f"iv direct batch {k}")
        p.close()


def test_removed_knobs_change_nothing(gpu_lib, monkeypatch):
    """The run-table pair phase (with its pair hash) and time-ordered incidence
    lists were removed after GPU runs with them switched on ended in a fault.
    Their former environment switches must not bring any other path back: with
    them set, the results are those of the oracle, through the default paths."""
    monkeypatch.setenv("HGT_PAIR_RUNS", "1")
    monkeypatch.setenv("HGT_PAIR_CAP", "3")
    monkeypatch.setenv("HGT_TIME_ORDER", "1")
    for st, track in ((W.medium(scale=0.0005, n_batches=2), ("hyperedge",)),
                      (W.plain_stream("hub", 400, 700, ("power", 1.6, 2, 150), 1.3, 0.0, 2, 80, 90, W.SEED_BASE + 78),
                       ("hyperedge",)),
                      (_random_stream(4200, n_edges=150, nv=60, n_batches=2), ("temporal",))):
        p = Pair(st, track=track)
        compare_counts(p.g, p.o, p.track, "removed knobs build")
        for k, b in enumerate(st.batches):
            p.apply(b, f"removed knobs batch {k}")
            compare_counts(p.g, p.o, p.track, f"removed knobs batch {k}")
        compare_store(p.g, p.o, "removed knobs end")
        p.close()


@pytest.mark.parametrize("slots", ["64", "256"])
def test_two_hop_hash_in_passes(gpu_lib, monkeypatch, slots):
    """Per-wave 2-hop hashes of 64 / 256 slots: every neighbour with more than
    a few dozen 2-hop entries is hashed in several passes over parts of its
    neighbours, and passes that overflow are split; hyperedge centres are all
    sent to the 2-hop kernel, temporal centres use it anyway.  Same counts."""
    monkeypatch.setenv("HGT_WAVE_SLOTS", slots)
    monkeypatch.setenv("HGT_FORCE_STAGE", "3")
    st = W.plain_stream("hub", 400, 700, ("power", 1.6, 2, 150), 1.3, 0.0, 2, 80, 90, W.SEED_BASE + 81)
    p = Pair(st, track=("hyperedge",))
    compare_counts(p.g, p.o, p.track, f"passes {slots} hub build")
    for k, b in enumerate(st.batches):
        p.apply(b, f"passes {slots} hub batch {k}")
        compare_counts(p.g, p.o, p.track, f"passes {slots} hub batch {k}")
    p.close()
    st = W.temporal_stream("tpass", 300, 1500, 300, 2, 1.8, 2, 40, 50.0, 40_000, 20_000, W.SEED_BASE + 82, pop_s=1.1)
    p = Pair(st, track=("temporal",))
    compare_counts(p.g, p.o, p.track, f"passes {slots} temporal build")
    for k, b in enumerate(st.batches):
        p.apply(b, f"passes {slots} temporal batch {k}")
        compare_counts(p.g, p.o, p.track, f"passes {slots} temporal batch {k}")
    p.close()


def test_incident_vertex_large_owner_stage(gpu_lib, monkeypatch):
    """Every incident-vertex owner passed on to the stage with 16 MB maps (the
    stage of the largest owners): same counts."""
    monkeypatch.setenv("HGT_IV_FORCE_STAGE", "2")
    for st in (_random_stream(4300, n_edges=200, nv=70, n_batches=2, n_ins=40, n_del=40, temporal=False, card=(1, 7)),
               W.medium(scale=0.0005, n_batches=2)):
        p = Pair(st, track=("incident_vertex",))
        compare_counts(p.g, p.o, p.track, "iv stage 2 build")
        for k, b in enumerate(st.batches):
            p.apply(b, f"iv stage 2 batch {k}")
            compare_counts(p.g, p.o, p.track, f"iv stage 2 batch {k}")
        p.close()


def test_dyadic_graph_triangles(gpu_lib):
    """The graph special case: hyperedges of two vertices, no edge twice.  The
    incident-vertex counts are [0, 0, triangles] with the triangle count the
    textbook trace(A^3) / 6 of the adjacency matrix, after the build and after
    every batch; hyperedge counts equal the oracle's."""
    st = W.dyadic(n_vertices=600, n_edges=6000, n_batches=3, n_changes=1200, seed=W.SEED_BASE + 62)
    p = Pair(st, track=("hyperedge", "incident_vertex"))

    def triangles():
        off, mem, live = p.g.export_h2v()
        e = mem.reshape(-1, 2).astype(np.int64)
        a = np.zeros((st.n_vertices, st.n_vertices), np.int64)
        a[e[:, 0], e[:, 1]] = 1
        a[e[:, 1], e[:, 0]] = 1
        return int(np.trace(a @ a @ a)) // 6

    for k in range(len(st.batches) + 1):
        if k:
            p.apply(st.batches[k - 1], f"dyadic batch {k - 1}")
        compare_counts(p.g, p.o, p.track, f"dyadic step {k}")
        iv = p.g.triad_counts("incident_vertex")
        assert iv[0] == 0 and iv[1] == 0 and iv[2] == triangles() > 0, (k, iv)
    p.close()


def test_compaction_keeps_store_and_counts(gpu_lib):
    """Pool compaction (every live list moved into fresh pools) in the middle of
    a stream of batches: the used pool words shrink, and the exported store and
    every count still equal the oracle's, also after the following batches."""
    st = W.temporal_stream("compact", 80, 400, 120, 5, 2.0, 1, 9, 7.0, 2000, 400, seed=W.SEED_BASE + 600)
    p = Pair(st, track=ALL)
    for k, b in enumerate(st.batches):
        p.apply(b, f"compaction batch {k}")
        if k == 2:
            before = p.g.info()
            p.g.compact()
            after = p.g.info()
            assert after["compactions"] == before["compactions"] + 1
            assert after["h2v_used_words"] < before["h2v_used_words"]
            assert after["v2h_used_words"] < before["v2h_used_words"]
            compare_store(p.g, p.o, "after compaction")
            compare_counts(p.g, p.o, ALL, "after compaction")
    compare_store(p.g, p.o, "compaction end")
    compare_counts(p.g, p.o, ALL, "compaction end")
    p.close()


_ORACLE_CACHE = {}


@pytest.mark.parametrize("shape,slice_lh", [("entries", "0"), ("entries", "100000000"), ("vertex-pairs", "0")])
def test_dense_centres(gpu_lib, monkeypatch, shape, slice_lh):
    """Dense graphs, and a batch that deletes their largest hyperedges and
    inserts their rows again.  In the first (3,000 hyperedges with up to 400
    members on 900 vertices) those centres hold more than 65,536 neighbour-row
    entries; in the second (600 hyperedges with up to 120 members on 150
    vertices) fewer, but their neighbours share more than 65,536 vertex pairs.
    Either way they go to the 2-hop kernel, shared among several workgroups
    (or, with a slice size above every centre's lists, one workgroup each);
    the change of the counts equals the oracle's delta by definition."""
    from .test_gpu_fullsize import _gpu_delta, _oracle_delta
    if slice_lh != "0":
        monkeypatch.setenv("HGT_SLICE_LH", slice_lh)
    monkeypatch.delenv("HGT_FORCE_STAGE", raising=False)
    nv, ne, hi = (900, 3000, 400) if shape == "entries" else (150, 600, 120)
    st = W.plain_stream("dense", nv, ne, ("power", 1.4, 2, hi), 0.0, 0.0, 1, 1, 1, W.SEED_BASE + 91)
    ini = st.initial
    cards = np.diff(ini.offsets.astype(np.int64))
    big = np.argsort(-cards, kind="stable")[:2].astype(np.int64)
    neighbour_entries = 0
    rows = ini.rows(big)
    mem = set(ini.members[ini.offsets[big[0]]:ini.offsets[big[0] + 1]].tolist())
    for i in range(ini.n):  # the entries of the largest centre's neighbour rows
        r = ini.members[ini.offsets[i]:ini.offsets[i + 1]]
        if i != big[0] and mem.intersection(r.tolist()):
            neighbour_entries += len(r)
    if shape == "entries":
        assert neighbour_entries > 65536, neighbour_entries
    else:
        assert neighbour_entries < 65536, neighbour_entries
    p = Pair(W.Stream("dense", st.n_vertices, ini), track=("hyperedge",))
    before = np.array(p.g.triad_counts("hyperedge"), np.uint64)
    batch = W.Batch(del_handles=big, ins=rows, ins_handles=np.arange(ini.n, ini.n + len(big), dtype=np.int64))
    args, fin = p.prepare(batch, "dense")
    out = p.g.apply_batch(*args)
    ids = out.cpu().numpy().astype(np.int64)
    after = np.array(p.g.triad_counts("hyperedge"), np.uint64)
    if shape not in _ORACLE_CACHE:  # the same oracle delta serves both slice sizes
        _ORACLE_CACHE[shape] = _oracle_delta(p.o, big, rows, None, ("hyperedge",))
    _, oids, want = _ORACLE_CACHE[shape]
    assert ids.tolist() == [int(x) for x in oids]
    got = _gpu_delta({"hyperedge": before}, {"hyperedge": after})["hyperedge"]
    bad = np.nonzero(got != want["hyperedge"])[0]
    assert len(bad) == 0, f"classes {bad.tolist()[:8]}: gpu {got[bad][:8]} oracle {want['hyperedge'][bad][:8]}"
    p.close()


def test_sliced_two_hop_centres(gpu_lib, monkeypatch):
    """Centres of the 2-hop kernel shared by several workgroups (a tiny slice
    size makes nearly every centre sliced): hyperedge centres all sent there,
    temporal centres use it anyway.  Same counts as the oracle."""
    monkeypatch.setenv("HGT_SLICE_LH", "48")
    monkeypatch.setenv("HGT_FORCE_STAGE", "3")
    st = W.plain_stream("slices", 400, 700, ("power", 1.6, 2, 150), 1.3, 0.0, 2, 80, 90, W.SEED_BASE + 83)
    p = Pair(st, track=("hyperedge",))
    compare_counts(p.g, p.o, p.track, "sliced build")
    for k, b in enumerate(st.batches):
        p.apply(b, f"sliced batch {k}")
        compare_counts(p.g, p.o, p.track, f"sliced batch {k}")
    p.close()
    st = W.temporal_stream("tslices", 300, 1500, 300, 2, 1.8, 2, 40, 50.0, 40_000, 20_000, W.SEED_BASE + 84, pop_s=1.1)
    p = Pair(st, track=("temporal", "hyperedge"))
    compare_counts(p.g, p.o, p.track, "sliced temporal build")
    for k, b in enumerate(st.batches):
        p.apply(b, f"sliced temporal batch {k}")
        compare_counts(p.g, p.o, p.track, f"sliced temporal batch {k}")
    p.close()
