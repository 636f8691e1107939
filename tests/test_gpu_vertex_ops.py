"""GPU parity of the horizontal operations (incident-vertex insertions and
deletions inside live hyperedges) through hgt_apply_vertex_ops against the
oracle: exported store and every tracked count after each batch of ops,
mixed with ordinary batches; rejected batches leave the graph unchanged."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2512_21009_amd import workloads as W

from .gpu_harness import Pair, compare_counts, compare_store, dev
from .test_oracle import random_vertex_ops

pytestmark = pytest.mark.gpu

ALL = ("hyperedge", "incident_vertex", "temporal")


def _ops(p, e, v, ins, where):
    import torch
    rc = p.g.apply_vertex_ops(dev(e, np.int32), dev(v, np.int32), dev(ins.astype(np.uint8), np.uint8),
                              raise_on_error=False)
    torch.cuda.synchronize()
    st, _ = p.o.apply_vertex_ops(e, v, ins)
    assert st == orc.OK and rc == 0, (where, st, rc)


@pytest.mark.parametrize("seed", range(3))
def test_vertex_ops_random_all_families(gpu_lib, seed):
    rng = np.random.default_rng(5000 + seed)
    st = W.temporal_stream("vops", 60, 150, 30, 2, 2.0, 1, 7, 7.0, 700, 150, seed=W.SEED_BASE + 500 + seed)
    p = Pair(st, track=ALL)
    for k in range(3):
        e, v, ins = random_vertex_ops(rng, p.o, 25, st.n_vertices)
        _ops(p, e, v, ins, f"ops {k}")
        compare_store(p.g, p.o, f"ops {k}")
        compare_counts(p.g, p.o, ALL, f"ops {k}")
        if k < len(st.batches):  # an ordinary batch in between (IDs freed and reused)
            p.apply(st.batches[k], f"batch {k}")
            compare_store(p.g, p.o, f"batch {k}")
            compare_counts(p.g, p.o, ALL, f"batch {k}")
    p.close()


def test_vertex_ops_medium_shape(gpu_lib):
    """Medium's shape at 1/1000 scale: 300 hyperedges modified per batch of ops."""
    rng = np.random.default_rng(5100)
    st = W.medium(scale=0.001, n_batches=1)
    p = Pair(st, track=("hyperedge", "incident_vertex"))
    for k in range(2):
        e, v, ins = random_vertex_ops(rng, p.o, 300, st.n_vertices, max_per_edge=4)
        _ops(p, e, v, ins, f"medium ops {k}")
        compare_counts(p.g, p.o, p.track, f"medium ops {k}")
    compare_store(p.g, p.o, "medium ops end")
    p.close()


def test_vertex_ops_errors_leave_state_unchanged(gpu_lib):
    hgt = gpu_lib
    rows = [[0, 1], [1, 2], [2, 3, 4], [0, 4]]
    off = np.zeros(len(rows) + 1, np.uint64)
    off[1:] = np.cumsum([len(r) for r in rows])
    mem = np.array([x for r in rows for x in r], np.uint32)
    st = W.Stream("rows", 6, W.CSR(off, mem, np.array([1, 2, 3, 4], np.int64)), window=10)
    p = Pair(st, track=ALL)
    p.apply(W.Batch(np.array([1]), W.CSR(np.zeros(1, np.uint64), np.zeros(0, np.uint32)), np.zeros(0, np.int64)),
            "delete 1")
    g = p.g
    before = ([g.triad_counts(f) for f in ALL], g.export_h2v()[1].tolist(), g.export_v2h()[1].tolist())
    cases = [
        (hgt.ENOENT, [1], [0], [1]),            # not live
        (hgt.ENOENT, [9], [0], [1]),            # never used
        (hgt.EINVAL, [0], [6], [1]),            # vertex out of range
        (hgt.EINVAL, [0], [1], [1]),            # already a member
        (hgt.EINVAL, [0], [3], [0]),            # not a member
        (hgt.EINVAL, [0, 0], [0, 1], [0, 0]),   # left empty
        (hgt.EINVAL, [2, 2], [5, 5], [1, 1]),   # the same op twice
        (hgt.EINVAL, [2, 2], [3, 3], [0, 1]),   # the same pair twice
    ]
    for code, e, v, i in cases:
        rc = g.apply_vertex_ops(dev(e, np.int32), dev(v, np.int32), dev(i, np.uint8), raise_on_error=False)
        assert rc == code, (rc, code, e, v, i)
        after = ([g.triad_counts(f) for f in ALL], g.export_h2v()[1].tolist(), g.export_v2h()[1].tolist())
        assert after == before
    _ops(p, np.array([2, 0]), np.array([4, 5]), np.array([False, True]), "valid after errors")
    compare_store(p.g, p.o, "valid after errors")
    compare_counts(p.g, p.o, ALL, "valid after errors")
    p.close()
