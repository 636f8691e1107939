"""GPU parity of the batched form: many independent graphs updated by one
hgt_apply_batches call (shared triad launches over (graph, hyperedge) work
items) against the CPU oracle, graph by graph, exactly."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2512_21009_amd import workloads as W

from .gpu_harness import Pair, apply_many, compare_counts, compare_store, dev

pytestmark = pytest.mark.gpu

ALL = ("hyperedge", "incident_vertex", "temporal")


def _mixed_streams(seed, n_batches=2):
    """Graphs of uneven size and different tracked families."""
    out = []
    for k, st in enumerate(W.batched(seed=seed, n_graphs=6, e_lo=150, e_hi=3000, b_lo=5, b_hi=400, card_hi=96)):
        out.append((st, ("hyperedge",)))
    for k in range(2):
        st = W.plain_stream(f"p{k}", 120 + 40 * k, 300 + 100 * k, ("uniform", 1, 9), 1.0, 0.0, n_batches, 50, 60,
                            seed * 10 + k)
        out.append((st, ("hyperedge", "incident_vertex")))
    st = W.temporal_stream("t", 60, 150, 30, n_batches, 2.0, 1, 6, 7.0, 700, 150, seed + 5)
    out.append((st, ALL))
    st = W.temporal_stream("t2", 80, 200, 40, n_batches, 2.0, 2, 8, 5.0, 900, 200, seed + 6)
    out.append((st, ("temporal",)))
    return out


@pytest.mark.parametrize("seed", [11, 12])
def test_batched_matches_oracle(gpu_lib, seed):
    specs = _mixed_streams(seed)
    pairs = [Pair(st, track=tr) for st, tr in specs]
    for k, p in enumerate(pairs):
        compare_counts(p.g, p.o, p.track, f"graph {k} build")
    n_rounds = max(len(st.batches) for st, _ in specs)
    for r in range(n_rounds):
        act = [(p, st.batches[r]) for p, (st, _) in zip(pairs, specs) if r < len(st.batches)]
        apply_many([a for a, _ in act], [b for _, b in act], f"round {r}")
        for k, p in enumerate(pairs):
            compare_counts(p.g, p.o, p.track, f"round {r} graph {k}")
            compare_store(p.g, p.o, f"round {r} graph {k}")
    for p in pairs:
        p.close()


def test_batched_rejects_only_the_bad_batch(gpu_lib):
    from paper_2512_21009_amd import hgt
    specs = _mixed_streams(21, n_batches=1)[:4]
    pairs = [Pair(st, track=tr) for st, tr in specs]
    bad = 2
    before = pairs[bad].g.triad_counts("hyperedge")
    items, fins = [], []
    for k, (p, (st, _)) in enumerate(zip(pairs, specs)):
        args, fin = p.prepare(st.batches[0], f"graph {k}")
        if k == bad:  # delete an ID that is not live
            args = (dev([p.o.next_id + 5], np.int32),) + args[1:]
        items.append((p.g,) + args)
        fins.append(fin)
    rc, status, outs = hgt.apply_batches(items, raise_on_error=False)
    assert rc == hgt.ENOENT and status[bad] == hgt.ENOENT
    assert all(s == hgt.OK for k, s in enumerate(status) if k != bad)
    for k, (p, fin, out) in enumerate(zip(pairs, fins, outs)):
        if k == bad:
            assert p.g.triad_counts("hyperedge") == before
            continue
        fin(out)
        compare_counts(p.g, p.o, p.track, f"graph {k}")
        compare_store(p.g, p.o, f"graph {k}")
    for p in pairs:
        p.close()


def test_batched_rejects_repeated_graph(gpu_lib):
    from paper_2512_21009_amd import hgt
    st, tr = _mixed_streams(31, n_batches=1)[6]
    p = Pair(st, track=tr)
    args, _ = p.prepare(st.batches[0])
    rc, status, _ = hgt.apply_batches([(p.g,) + args, (p.g,) + args], raise_on_error=False)
    assert rc == hgt.EINVAL
    compare_counts(p.g, p.o, p.track, "unchanged")
    p.close()


@pytest.mark.parametrize("stage", [1, 3])
def test_batched_every_kernel_path(gpu_lib, monkeypatch, stage):
    """Work items handed from stage to stage carry their graph."""
    monkeypatch.setenv("HGT_FORCE_STAGE", str(stage))
    specs = _mixed_streams(41 + stage, n_batches=1)[:8]
    pairs = [Pair(st, track=tr) for st, tr in specs]
    for k, p in enumerate(pairs):
        compare_counts(p.g, p.o, p.track, f"stage {stage} graph {k} build")
    apply_many(pairs, [st.batches[0] for st, _ in specs], f"stage {stage}")
    for k, p in enumerate(pairs):
        compare_counts(p.g, p.o, p.track, f"stage {stage} graph {k}")
    for p in pairs:
        p.close()
