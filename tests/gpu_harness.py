"""Drive the HIP library and the CPU oracle side by side on one input stream.

Each side translates the stream's deletion handles to the IDs it handed out
itself; the IDs, the incidence store (exported from the device) and every
tracked count are compared after the build and after every batch.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as orc


def dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(dtype))).to("cuda:0")


def oracle_v2h(o: orc.OracleGraph):
    """vertex -> ascending live IDs, from the oracle's rows."""
    lens = o.lens()
    ids = np.repeat(np.arange(o.n_slots, dtype=np.int64), lens)
    live = np.repeat(o.live.astype(bool), lens)
    v = o.mem.astype(np.int64)[live]
    h = ids[live]
    order = np.lexsort((h, v))
    v, h = v[order], h[order]
    off = np.zeros(o.n_vertices + 1, np.int64)
    np.add.at(off, v + 1, 1)
    return np.cumsum(off), h.astype(np.uint32)


def compare_store(g, o: orc.OracleGraph, where: str):
    off, mem, live = g.export_h2v()
    n = len(live)
    assert n == o.next_id, f"{where}: next_id {n} vs {o.next_id}"
    assert (live == o.live[:n]).all(), f"{where}: live flags differ"
    olens = o.lens()[:n] * o.live[:n]
    glens = np.diff(off.astype(np.int64))
    assert (glens == olens).all(), f"{where}: h2v lengths differ"
    oo = np.concatenate([o.row(i) for i in range(n) if o.live[i]]) if olens.sum() else np.zeros(0, np.uint32)
    assert (mem == oo).all(), f"{where}: h2v members differ"
    voff, vmem = g.export_v2h()
    ooff, omem = oracle_v2h(o)
    assert (voff.astype(np.int64) == ooff).all(), f"{where}: v2h lengths differ"
    assert (vmem == omem).all(), f"{where}: v2h lists differ"


def compare_counts(g, o: orc.OracleGraph, track, where: str, full=True, expect=None):
    """Compare device counts with the oracle's recount (full=True) or with
    `expect` (a dict of kind -> np.ndarray, e.g. accumulated deltas)."""
    for kind in track:
        got = np.array(g.triad_counts(kind), dtype=np.uint64)
        if expect is not None and kind in expect:
            want = expect[kind]
        elif kind == "hyperedge":
            want = o.he_counts()
        elif kind == "incident_vertex":
            want = o.iv_counts()
        else:
            want = o.temporal_counts()
        bad = np.nonzero(got != want)[0]
        assert len(bad) == 0, f"{where}: {kind} differs at classes {bad.tolist()[:8]}: gpu {got[bad][:8]} oracle {want[bad][:8]}"


class Pair:
    """A device graph and an oracle graph fed the same stream."""

    def __init__(self, stream, track=("hyperedge",), edge_capacity=0, pool_words=0):
        from paper_2512_21009_amd import hgt
        self.st = stream
        self.track = tuple(track)
        ini = stream.initial
        temporal = "temporal" in self.track
        ts = ini.ts if temporal else None
        self.g = hgt.Graph.build(stream.n_vertices, dev(ini.offsets, np.int64), dev(ini.members, np.int32),
                                 dev(ts, np.int64) if ts is not None else None, track=self.track,
                                 window=stream.window, edge_capacity=edge_capacity, pool_words=pool_words)
        self.o = orc.OracleGraph(stream.n_vertices, ini.offsets, ini.members, ts=ts, window=stream.window)
        n0 = ini.n
        self.gid = {h: h for h in range(n0)}  # handle -> device ID
        self.oid = {h: h for h in range(n0)}  # handle -> oracle ID

    def prepare(self, batch, where=""):
        """Device arguments of `batch` (del_ids, ins_offsets, ins_members, ins_ts)
        and a function that takes the assigned-ID tensor, applies the batch to
        the oracle and checks the IDs."""
        temporal = "temporal" in self.track
        gd = np.array([self.gid[h] for h in batch.del_handles], dtype=np.int64)
        ins = batch.ins
        ts = ins.ts if temporal else None
        args = (dev(gd, np.int32) if len(gd) else None,
                dev(ins.offsets, np.int64) if ins.n else None,
                dev(ins.members, np.int32) if ins.n else None,
                dev(ts, np.int64) if (ts is not None and ins.n) else None)

        def finish(out):
            od = np.array([self.oid[h] for h in batch.del_handles], dtype=np.int64)
            st, oids = self.o.apply_batch(od, ins.offsets, ins.members, ts)
            assert st == orc.OK, f"{where}: oracle rejected the batch ({st})"
            gids = out.cpu().numpy().astype(np.uint32) if out is not None else np.zeros(0, np.uint32)
            assert gids.tolist() == oids.tolist(), f"{where}: assigned IDs differ"
            for h, a, b in zip(batch.ins_handles, gids, oids):
                self.gid[int(h)] = int(a)
                self.oid[int(h)] = int(b)
            for h in batch.del_handles:
                self.gid.pop(int(h), None)
                self.oid.pop(int(h), None)
            return gids
        return args, finish

    def apply(self, batch, where=""):
        import torch
        args, finish = self.prepare(batch, where)
        out = self.g.apply_batch(*args)
        torch.cuda.synchronize()
        return finish(out)

    def close(self):
        self.g.close()


def apply_many(pairs, batches, where="", **kw):
    """Applies batches[i] to pairs[i] through the batched entry point (one call,
    keyword arguments passed on) and to each oracle; checks the assigned IDs."""
    import torch
    from paper_2512_21009_amd import hgt
    items, fins = [], []
    for k, (p, b) in enumerate(zip(pairs, batches)):
        args, fin = p.prepare(b, f"{where} graph {k}")
        items.append((p.g,) + args)
        fins.append(fin)
    outs = hgt.apply_batches(items, **kw)
    torch.cuda.synchronize()
    for fin, out in zip(fins, outs):
        fin(out)
