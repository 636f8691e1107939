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


@pytest.mark.parametrize("choice", [0, 1, 2, 3, 4, 5, 6])
def test_graph_launch_every_tuned_choice(gpu_lib, monkeypatch, choice):
    """Rounds launched as captured HIP graphs (the executable updated in place
    from the second round on) under each of the autotuner's launch choices,
    forced, give the oracle's counts and store exactly."""
    monkeypatch.setenv("HGT_TUNE_FORCE", str(choice))
    specs = _mixed_streams(51 + choice, n_batches=3)
    pairs = [Pair(st, track=tr) for st, tr in specs]
    for r in range(3):
        act = [(p, st.batches[r]) for p, (st, _) in zip(pairs, specs) if r < len(st.batches)]
        apply_many([a for a, _ in act], [b for _, b in act], f"choice {choice} round {r}", graph=True, autotune=True)
        for k, p in enumerate(pairs):
            compare_counts(p.g, p.o, p.track, f"choice {choice} round {r} graph {k}")
            compare_store(p.g, p.o, f"choice {choice} round {r} graph {k}")
    # every round ran as a captured graph (the default stream's rounds are captured on
    # a stream of the library's own)
    assert sum(p.g.info()["graph_launches"] for p in pairs) == 3
    for p in pairs:
        p.close()


def _churn_rounds(st, n_rounds, k, seed):
    """Rounds that delete k live hyperedges and insert their rows again under
    fresh handles: every round has the same shape (same changes, same degrees)."""
    rng = np.random.default_rng(seed)
    ini = st.initial
    live = rng.choice(ini.n, size=k, replace=False).astype(np.int64)
    rows = ini.rows(live)
    t0 = int(ini.ts.max()) + 1 if ini.ts is not None else 0
    nxt = ini.n
    out = []
    for r in range(n_rounds):
        handles = np.arange(nxt, nxt + k, dtype=np.int64)
        ins = W.CSR(rows.offsets, rows.members)
        if ini.ts is not None:  # inserted timestamps never go back in time
            ins.ts = t0 + r * k + np.arange(k, dtype=np.int64)
        out.append(W.Batch(del_handles=live.copy(), ins=ins, ins_handles=handles))
        live, nxt = handles, nxt + k
    return out


def test_autotuner_settles_and_writes_its_cache(gpu_lib, tmp_path):
    """Rounds of one shape, autotuned: after every choice has been timed the
    tuner keeps one for the round's key and appends it to its cache file; the
    counts stay exact throughout.  (The cache path is read once per process,
    so this runs in a child process with its own HGT_TUNE_CACHE.)"""
    import os
    import subprocess
    import sys
    cache = tmp_path / "tune.txt"
    env = dict(os.environ, HGT_TUNE_CACHE=str(cache))
    env.pop("HGT_TUNE_FORCE", None)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from tests import test_gpu_batched as T\n"
        "T._autotune_child()\n" % root)
    r = subprocess.run([sys.executable, "-c", code], env=env, cwd=root, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert "settled" in r.stdout, r.stdout[-2000:]
    lines = [ln.split() for ln in cache.read_text().splitlines() if ln.strip()]
    assert len(lines) >= 1 and all(len(ln) == 7 for ln in lines)
    assert all(0 <= int(ln[1]) < 7 for ln in lines)


def _autotune_child():
    import torch
    from paper_2512_21009_amd import hgt
    hgt.load()
    specs = _mixed_streams(61, n_batches=1)[6:9]  # hyperedge + incident-vertex, and the temporal graphs
    pairs = [Pair(st, track=tr) for st, tr in specs]
    rounds = [_churn_rounds(st, 18, 12, 70 + k) for k, (st, _) in enumerate(specs)]
    for r in range(18):
        apply_many(pairs, [rs[r] for rs in rounds], f"tuned round {r}", graph=(r % 2 == 0), autotune=True)
        torch.cuda.synchronize()
        if r % 6 == 5:
            for k, p in enumerate(pairs):
                compare_counts(p.g, p.o, p.track, f"tuned round {r} graph {k}")
    n = hgt.tune_flush()
    for k, p in enumerate(pairs):
        compare_counts(p.g, p.o, p.track, f"tuned end graph {k}")
        compare_store(p.g, p.o, f"tuned end graph {k}")
    for p in pairs:
        p.close()
    print(f"settled {n}", flush=True)
    assert n >= 1
