"""The no-allocation entry point, hgt_apply_batch_noalloc, against
hgt_apply_batch on identical copies of a graph: the same assigned IDs,
incidence store and counts of every family (tolerance 0) on two calls in a
row, the second with a smaller batch; and batches that would need more than
the fixed scratch array, or a larger graph, are rejected with the graph
unchanged."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2512_21009_amd import workloads as W

from .gpu_harness import compare_counts, dev

pytestmark = pytest.mark.gpu

ALL = ("hyperedge", "incident_vertex", "temporal")


def _build(hgt, st, track, **kw):
    ini = st.initial
    ts = dev(ini.ts, np.int64) if "temporal" in track else None
    return hgt.Graph.build(st.n_vertices, dev(ini.offsets, np.int64), dev(ini.members, np.int32), ts, track=track,
                           window=st.window, **kw)


def _state(g, track):
    off, mem, live = g.export_h2v()
    voff, vmem = g.export_v2h()
    return ([g.triad_counts(k) for k in track], off.tolist(), mem.tolist(), live.tolist(), voff.tolist(),
            vmem.tolist())


def _args(batch, ids_of, temporal, n_del=None, n_ins=None):
    dels = batch.del_handles if n_del is None else batch.del_handles[:n_del]
    ins = batch.ins if n_ins is None else batch.ins.rows(np.arange(n_ins))
    d = np.array([ids_of[int(h)] for h in dels], np.int64)
    handles = batch.ins_handles if n_ins is None else batch.ins_handles[:n_ins]
    args = dict(del_ids=dev(d, np.int32) if len(d) else None,
                ins_offsets=dev(ins.offsets, np.int64) if ins.n else None,
                ins_members=dev(ins.members, np.int32) if ins.n else None,
                ins_ts=dev(ins.ts, np.int64) if (temporal and ins.n) else None)
    return args, dels, handles, ins


def test_noalloc_matches_apply_batch_twice(gpu_lib):
    import torch
    hgt = gpu_lib
    st = W.temporal_stream("noalloc", 3000, 6000, 900, 2, 2.2, 2, 40, 50.0, 200_000, 60_000, seed=W.SEED_BASE + 123)
    a = _build(hgt, st, ALL, edge_capacity=20000, pool_words=1 << 20)
    b = _build(hgt, st, ALL, edge_capacity=20000, pool_words=1 << 20)
    o = orc.OracleGraph(st.n_vertices, st.initial.offsets, st.initial.members, ts=st.initial.ts, window=st.window)
    ids_of = {h: h for h in range(st.initial.n)}
    # first call: a whole batch; second call: a smaller part of the next batch
    for k, (n_del, n_ins) in enumerate(((None, None), (120, 250))):
        args, dels, handles, ins = _args(st.batches[k], ids_of, True, n_del, n_ins)
        out_a = a.apply_batch(noalloc=True, **args)
        out_b = b.apply_batch(**args)
        torch.cuda.synchronize()
        ga, gb = out_a.cpu().numpy().tolist(), out_b.cpu().numpy().tolist()
        assert ga == gb, f"call {k}: assigned IDs differ"
        assert _state(a, ALL) == _state(b, ALL), f"call {k}: counts or store differ"
        stt, oids = o.apply_batch(np.array([ids_of[int(h)] for h in dels], np.int64), ins.offsets, ins.members,
                                  ins.ts)
        assert stt == orc.OK and oids.tolist() == ga
        compare_counts(a, o, ALL, f"no-allocation call {k}")
        for h, i in zip(handles, ga):
            ids_of[int(h)] = int(i)
        for h in dels:
            ids_of.pop(int(h))
    assert a.sync() == hgt.OK and b.sync() == hgt.OK
    a.close()
    b.close()


def test_noalloc_rejects_growth_and_oversize(gpu_lib):
    import torch
    hgt = gpu_lib
    # the graph would have to grow its ID capacity: rejected, unchanged; the same
    # batch through hgt_apply_batch then grows it, after which the entry point works
    st = W.plain_stream("noalloc-grow", 500, 400, ("uniform", 2, 6), 0.8, 0.0, 2, 700, 50, W.SEED_BASE + 124)
    track = ("hyperedge", "incident_vertex")
    g = _build(hgt, st, track)
    ids_of = {h: h for h in range(st.initial.n)}
    before = _state(g, track)
    args, dels, handles, _ = _args(st.batches[0], ids_of, False)
    rc, _ = g.apply_batch(noalloc=True, raise_on_error=False, **args)
    assert rc == hgt.ENOMEM
    assert _state(g, track) == before
    out = g.apply_batch(**args)
    torch.cuda.synchronize()
    for h, i in zip(handles, out.cpu().numpy().tolist()):
        ids_of[int(h)] = int(i)
    for h in dels:
        ids_of.pop(int(h))
    args, _, _, _ = _args(st.batches[1], ids_of, False, 20, 30)
    g.apply_batch(noalloc=True, **args)
    g.close()
    # a graph whose batch scratch exceeds the fixed array: rejected, unchanged
    big = W.medium(scale=0.3, n_batches=1)
    gb = _build(hgt, big, ("hyperedge",))
    before = _state(gb, ("hyperedge",))
    args, _, _, _ = _args(big.batches[0], {h: h for h in range(big.initial.n)}, False, 50, 50)
    rc, _ = gb.apply_batch(noalloc=True, raise_on_error=False, **args)
    assert rc == hgt.ENOMEM
    assert _state(gb, ("hyperedge",)) == before
    gb.close()
