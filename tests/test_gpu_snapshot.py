"""GPU tests of snapshot / restore and of the poisoned state.

A fault is injected from the host (HGT_INJECT_FAULT=1: a batch that passed
validation stops right after its store update was queued, as if the next
launch had failed); every kernel that was queued runs to completion, so the
GPU itself never faults.  The graph must then refuse every call with
HGT_EPOISONED until a snapshot is restored, after which it must match the
oracle exactly, batch after batch.
"""
import os

import numpy as np
import pytest

from paper_2512_21009_amd import workloads as W

from .gpu_harness import Pair, apply_many, compare_counts, compare_store, dev

pytestmark = pytest.mark.gpu

ALL = ("hyperedge", "incident_vertex", "temporal")


def _temporal_stream(seed, n_batches=4):
    return W.temporal_stream("snap", 60, 160, 30, n_batches, 2.0, 1, 7, 7.0, 700, 150, seed)


def _plain_stream(seed, n_batches=3):
    return W.plain_stream("snap", 120, 300, ("uniform", 1, 9), 1.0, 0.0, n_batches, 60, 70, seed)


def _check(p, where, track=None):
    compare_store(p.g, p.o, where)
    compare_counts(p.g, p.o, track or p.track, where)


class _Injected:
    """HGT_INJECT_FAULT=1 while the block runs."""

    def __enter__(self):
        os.environ["HGT_INJECT_FAULT"] = "1"

    def __exit__(self, *exc):
        os.environ.pop("HGT_INJECT_FAULT", None)


def _assert_poisoned(hgt, g, st_batch_args):
    import torch
    assert g.sync() == hgt.EPOISONED
    rc, _ = g.apply_batch(*st_batch_args, raise_on_error=False)
    assert rc == hgt.EPOISONED
    calls = [lambda: g.triad_counts("hyperedge"), g.export_h2v, g.export_v2h, g.snapshot, g.compact,
             lambda: g.apply_vertex_ops(dev([0], np.int32), dev([0], np.int32), dev([1], np.uint8))]
    for call in calls:
        with pytest.raises(hgt.HgtError) as e:
            call()
        assert e.value.code == hgt.EPOISONED
    torch.cuda.synchronize()


def test_injected_fault_poisons_and_restore_recovers(gpu_lib):
    hgt = gpu_lib
    st = _temporal_stream(W.SEED_BASE + 501)
    p = Pair(st, track=ALL)
    p.apply(st.batches[0], "batch 0")
    snap = p.g.snapshot()
    args, _ = p.prepare(st.batches[1], "batch 1 (fault)")
    with _Injected():
        rc, _ = p.g.apply_batch(*args, raise_on_error=False)
    assert rc == hgt.EPOISONED
    _assert_poisoned(hgt, p.g, args)
    p.g.restore(snap)
    assert p.g.sync() == hgt.OK
    _check(p, "restored after the fault")
    for k in range(1, len(st.batches)):
        p.apply(st.batches[k], f"batch {k} after restore")
        _check(p, f"batch {k} after restore")
    snap.close()
    p.close()


def test_restore_rolls_back_across_compaction(gpu_lib):
    """Snapshot, apply two batches and compact (the pools shrink to what the
    live lists need), then restore: the graph is back at the snapshot and
    replays the same batches with the same IDs and counts."""
    st = _plain_stream(W.SEED_BASE + 502)
    p = Pair(st, track=("hyperedge", "incident_vertex"))
    p.apply(st.batches[0], "batch 0")
    snap = p.g.snapshot()
    o0, gid0, oid0 = p.o.copy(), dict(p.gid), dict(p.oid)
    for k in (1, 2):
        p.apply(st.batches[k], f"batch {k}")
    p.g.compact()
    _check(p, "compacted")
    p.g.restore(snap)
    p.o, p.gid, p.oid = o0, gid0, oid0
    _check(p, "rolled back")
    for k in (1, 2):
        p.apply(st.batches[k], f"batch {k} replayed")
        _check(p, f"batch {k} replayed")
    p.close()


def test_snapshot_bytes_restore_into_fresh_graph(gpu_lib):
    """The byte form, loaded back (with its structural checks), restores into
    an empty graph built with the same vertex count, families and window; the
    two graphs then take the same batches to the same state."""
    hgt = gpu_lib
    import torch
    st = _temporal_stream(W.SEED_BASE + 503)
    p = Pair(st, track=ALL)
    p.apply(st.batches[0], "batch 0")
    data = p.g.snapshot().to_bytes()
    assert data[:8] == b"HGTSNAP1"
    snap = hgt.Snapshot.from_bytes(data)
    assert snap.to_bytes() == data
    empty = (dev([0], np.int64), dev(np.zeros(0), np.int32), dev(np.zeros(0), np.int64))
    g2 = hgt.Graph.build(st.n_vertices, *empty, track=ALL, window=st.window)
    g2.restore(snap)
    q = Pair.__new__(Pair)
    q.__dict__.update(p.__dict__)
    q.g = g2
    _check(q, "fresh graph restored")
    for k in range(1, len(st.batches)):
        args, finish = p.prepare(st.batches[k], f"batch {k}")
        out1 = p.g.apply_batch(*args)
        out2 = g2.apply_batch(*args)
        torch.cuda.synchronize()
        assert out1.cpu().tolist() == out2.cpu().tolist(), f"batch {k}: assigned IDs differ"
        finish(out1)
        _check(p, f"batch {k} original")
        _check(q, f"batch {k} restored copy")
    g2.close()
    p.close()


def test_restore_rejects_another_shape(gpu_lib):
    hgt = gpu_lib
    st = _plain_stream(W.SEED_BASE + 504, n_batches=1)
    p = Pair(st, track=("hyperedge", "incident_vertex"))
    snap = p.g.snapshot()
    empty = (dev([0], np.int64), dev(np.zeros(0), np.int32))
    for nv, track in ((st.n_vertices + 1, ("hyperedge", "incident_vertex")), (st.n_vertices, ("hyperedge",))):
        g2 = hgt.Graph.build(nv, *empty, track=track)
        with pytest.raises(hgt.HgtError) as e:
            g2.restore(snap)
        assert e.value.code == hgt.EINVAL
        assert g2.sync() == hgt.OK
        g2.close()
    p.apply(st.batches[0], "batch 0")
    _check(p, "batch 0")
    p.close()


def test_batched_round_with_a_poisoned_graph(gpu_lib):
    """A fault inside a batched round poisons every graph of the round (also
    when the round would be launched as a captured HIP graph); a poisoned
    graph's batch is refused alone in later rounds; restoring brings each
    back."""
    hgt = gpu_lib
    pairs = [Pair(_plain_stream(W.SEED_BASE + 510 + i), track=("hyperedge", "incident_vertex")) for i in range(2)]
    snaps = [p.g.snapshot() for p in pairs]
    items = [(p.g,) + p.prepare(p.st.batches[0])[0] for p in pairs]
    for graph in (False, True):
        with _Injected():
            rc, st, _ = hgt.apply_batches(items, raise_on_error=False, graph=graph)
        assert rc == hgt.EPOISONED and st == [hgt.EPOISONED] * 2, (graph, rc, st)
        for p, s in zip(pairs, snaps):
            assert p.g.sync() == hgt.EPOISONED
            p.g.restore(s)
            _check(p, f"restored (graph={graph})")
    # poison the first graph alone, then run a round over both
    a, b = pairs
    args_a, _ = a.prepare(a.st.batches[0])
    with _Injected():
        rc, _ = a.g.apply_batch(*args_a, raise_on_error=False)
    assert rc == hgt.EPOISONED
    args_b, fin_b = b.prepare(b.st.batches[0], "b batch 0")
    rc, st, outs = hgt.apply_batches([(a.g,) + args_a, (b.g,) + args_b], raise_on_error=False)
    assert rc == hgt.EPOISONED and st == [hgt.EPOISONED, hgt.OK], (rc, st)
    import torch
    torch.cuda.synchronize()
    fin_b(outs[1])
    _check(b, "b after the mixed round")
    a.g.restore(snaps[0])
    apply_many([a, b], [a.st.batches[0], b.st.batches[1]], "both after restore", graph=True)
    _check(a, "a after restore")
    _check(b, "b second batch")
    for p in pairs:
        p.close()
