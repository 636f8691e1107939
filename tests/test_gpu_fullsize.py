"""The Medium workload at its full size (1M vertices, 2M hyperedges, one batch
of 50k deletions and 50k inserts), where the oracle is too slow to compare
with: properties that hold at any size.

* The counts maintained incrementally through the batch equal the counts of a
  fresh build of the resulting hyperedge set.
* The batch's inverse (deleting its inserts, re-inserting its deletions)
  restores every count.
"""
import numpy as np
import pytest

from paper_2512_21009_amd import workloads as W

from .gpu_harness import dev

pytestmark = pytest.mark.gpu

FAMS = ("hyperedge", "incident_vertex")


def _gather_rows(off, mem, rows):
    """CSR (offsets, members) of the given rows of (off, mem)."""
    off = off.astype(np.int64)
    lens = off[rows + 1] - off[rows]
    out_off = np.zeros(len(rows) + 1, np.int64)
    out_off[1:] = np.cumsum(lens)
    shift = np.repeat(off[rows] - out_off[:-1], lens)
    return out_off, mem[np.arange(out_off[-1], dtype=np.int64) + shift]


def test_medium_full_size_rebuild_and_inverse(gpu_lib):
    hgt = gpu_lib
    st = W.medium(n_batches=1)
    ini, b = st.initial, st.batches[0]
    g = hgt.Graph.build(st.n_vertices, dev(ini.offsets, np.int64), dev(ini.members, np.int32), track=FAMS)
    before = {f: g.triad_counts(f) for f in FAMS}
    dels = b.del_handles.astype(np.int64)  # the first batch deletes initial hyperedges: handle = ID
    ids = g.apply_batch(del_ids=dev(dels, np.int32), ins_offsets=dev(b.ins.offsets, np.int64),
                        ins_members=dev(b.ins.members, np.int32))
    after = {f: g.triad_counts(f) for f in FAMS}
    assert after != before

    # incremental == fresh build of the live hyperedges
    off, mem, live = g.export_h2v()
    rows = np.nonzero(live)[0].astype(np.int64)
    assert len(rows) == ini.n
    r_off, r_mem = _gather_rows(off, mem, rows)
    g2 = hgt.Graph.build(st.n_vertices, dev(r_off, np.int64), dev(r_mem, np.int32), track=FAMS)
    rebuilt = {f: g2.triad_counts(f) for f in FAMS}
    g2.close()
    assert rebuilt == after, ("full-size rebuild", rebuilt, after)

    # the inverse batch restores every count
    d_off, d_mem = _gather_rows(ini.offsets, ini.members, dels)
    ins_ids = ids.cpu().numpy().astype(np.int64)
    g.apply_batch(del_ids=dev(ins_ids, np.int32), ins_offsets=dev(d_off, np.int64), ins_members=dev(d_mem, np.int32))
    restored = {f: g.triad_counts(f) for f in FAMS}
    g.close()
    assert restored == before, ("inverse batch", restored, before)
