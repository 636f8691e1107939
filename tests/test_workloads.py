"""Host-side checks of the seeded input generators (shapes and stream
consistency; no GPU)."""
import numpy as np

from paper_2512_21009_amd import workloads as W


def _check_stream(st):
    live = set(range(st.initial.n))
    for b in st.batches:
        assert set(b.del_handles.tolist()) <= live, "deletion of a handle that is not live"
        assert len(set(b.del_handles.tolist())) == len(b.del_handles)
        live -= set(b.del_handles.tolist())
        assert not (set(b.ins_handles.tolist()) & live)
        live |= set(b.ins_handles.tolist())
        for i in range(b.ins.n):
            r = b.ins.row(i)
            assert len(np.unique(r)) == len(r) and r.max() < st.n_vertices


def test_generators_are_deterministic_and_consistent():
    a = W.medium(scale=0.001, n_batches=2)
    b = W.medium(scale=0.001, n_batches=2)
    assert np.array_equal(a.initial.members, b.initial.members)
    _check_stream(a)
    for st in W.batched(n_graphs=4, e_lo=100, e_hi=400, b_lo=5, b_hi=50, card_hi=40, n_batches=2):
        _check_stream(st)
        assert st.n_vertices >= 40


def test_power_law_cards_bounds_and_tail():
    rng = np.random.default_rng(1)
    c = W.power_law_cards(rng, 200000, 2.5, 2, 64)
    assert c.min() == 2 and c.max() <= 64
    # P(k) ~ k^-2.5: the ratio of the counts of 2 and 4 is about 2^2.5
    r = (c == 2).sum() / (c == 4).sum()
    assert 5.0 < r < 6.4


def test_served_requests_and_timestamps():
    sv = W.served(n_tenants=5, total_edges=3000, n_requests=30, req_hi=100, card_hi=30, pop_q=30.0, size_lo=100,
                  size_hi=1000, window_us=10_000)
    assert len(sv.arrivals) == 30
    times = [a[0] for a in sv.arrivals]
    assert times == sorted(times)
    for st in sv.tenants:
        _check_stream(st)
        last = int(st.initial.ts.max()) if st.initial.n else 0
        for b in st.batches:
            if b.ins.n:
                assert (np.diff(b.ins.ts) >= 0).all() and int(b.ins.ts[0]) >= last
                last = int(b.ins.ts[-1])
    per = {}
    for _, t, k, fam in sv.arrivals:
        assert k == per.get(t, 0)  # the k-th request of a tenant arrives k-th
        per[t] = k + 1
        assert fam in W.FAMILIES


def test_dyadic_stream_is_a_simple_graph():
    """Every hyperedge has two members and no edge is ever present twice."""
    st = W.dyadic(n_vertices=500, n_edges=3000, n_batches=3, n_changes=600, seed=W.SEED_BASE + 61)
    live = {}
    for h, r in enumerate(st.initial.members.reshape(-1, 2).tolist()):
        assert r[0] != r[1]
        live[h] = tuple(sorted(r))
    assert len(set(live.values())) == len(live) == 3000
    for b in st.batches:
        assert (np.diff(b.ins.offsets.astype(np.int64)) == 2).all()
        for h in b.del_handles.tolist():
            live.pop(h)
        for h, r in zip(b.ins_handles.tolist(), b.ins.members.reshape(-1, 2).tolist()):
            live[h] = tuple(sorted(r))
        assert len(set(live.values())) == len(live)
