"""GPU tests of the served form: requests from many tenants merged into
continuous-batching rounds give, request by request, the results of applying
each request alone, and those equal the CPU oracle's."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2512_21009_amd import workloads as W

from .gpu_harness import dev

pytestmark = pytest.mark.gpu

FAM = ("hyperedge", "incident_vertex", "temporal")


def _mini(seed=5, n_tenants=7, n_requests=40):
    return W.served(seed=seed, n_tenants=n_tenants, total_edges=4000, n_requests=n_requests, req_lo=1, req_hi=300,
                    card_hi=40, pop_q=40.0, size_lo=200, size_hi=2000, window_us=200_000)


def _add_tenants(srv, sv):
    for st in sv.tenants:
        ini = st.initial
        srv.add_tenant(st.n_vertices, dev(ini.offsets, np.int64), dev(ini.members, np.int32), dev(ini.ts, np.int64),
                       track=FAM, window=st.window)


def _args(st, b, hid):
    del_ids = np.array([hid[h] for h in b.del_handles], np.uint32)
    ins = b.ins
    return (del_ids, ins.offsets.astype(np.uint64), ins.members.astype(np.uint32), ins.ts.astype(np.int64))


def _alone_with_oracle(gpu_lib, sv):
    """Each request submitted after the previous one completed; every result
    checked against the oracle.  Returns the arguments and results."""
    srv = gpu_lib.Server(hbm_budget_bytes=1 << 30, arena_bytes=64 << 20)
    _add_tenants(srv, sv)
    oracles = [orc.OracleGraph(st.n_vertices, st.initial.offsets, st.initial.members, ts=st.initial.ts,
                               window=st.window) for st in sv.tenants]
    hid = [dict((h, h) for h in range(st.initial.n)) for st in sv.tenants]
    args, results = [], []
    for (t_us, tn, k, fam) in sv.arrivals:
        st = sv.tenants[tn]
        b = st.batches[k]
        a = _args(st, b, hid[tn])
        res = srv.wait(srv.submit(tn, *a))
        assert res["status"] == gpu_lib.OK, res["status"]
        assert res["round_size"] == 1
        o = oracles[tn]
        rc, oids = o.apply_batch(a[0].astype(np.int64), b.ins.offsets, b.ins.members, b.ins.ts)
        assert rc == orc.OK
        assert res["ids"].tolist() == oids.tolist(), f"request {len(args)}: IDs"
        for h, i in zip(b.ins_handles, res["ids"]):
            hid[tn][int(h)] = int(i)
        want = {"hyperedge": o.he_counts(), "incident_vertex": o.iv_counts(), "temporal": o.temporal_counts()}
        for f in FAM:
            assert np.array_equal(np.array(res[f], np.uint64), want[f]), f"request {len(args)} tenant {tn}: {f}"
        args.append((tn, a))
        results.append(res)
    srv.close()
    return args, results


@pytest.mark.parametrize("launch", ["stream", "graph_tuned"])
def test_served_mix_equals_alone_and_oracle(gpu_lib, launch):
    sv = _mini()
    args, alone = _alone_with_oracle(gpu_lib, sv)
    # the mix: every request submitted at once, merged into rounds by the server
    # (rounds launched kernel by kernel, or as captured HIP graphs with the
    # autotuner picking the launch choices)
    kw = {} if launch == "stream" else {"graph": True, "autotune": True}
    srv = gpu_lib.Server(hbm_budget_bytes=1 << 30, arena_bytes=64 << 20, **kw)
    _add_tenants(srv, sv)
    tickets = [srv.submit(tn, *a) for tn, a in args]
    mixed = [srv.wait(t) for t in tickets]
    info = srv.info()
    srv.close()
    assert info["max_round_size"] > 1 and info["rounds"] < len(args), info
    for i, (a, m) in enumerate(zip(alone, mixed)):
        assert m["status"] == a["status"] == gpu_lib.OK
        assert m["ids"].tolist() == a["ids"].tolist(), f"request {i}: IDs"
        for f in FAM:
            assert m[f] == a[f], f"request {i}: {f} counts differ alone vs mix"
        assert m["t_submit_ns"] <= m["t_admit_ns"] <= m["t_done_ns"]


def test_served_budget_and_arena_limits(gpu_lib):
    sv = _mini(seed=6, n_tenants=4, n_requests=12)
    args, alone = _alone_with_oracle(gpu_lib, sv)
    # a footprint budget of one byte: every request runs in a round of its own
    srv = gpu_lib.Server(hbm_budget_bytes=1, arena_bytes=64 << 20)
    _add_tenants(srv, sv)
    tickets = [srv.submit(tn, *a) for tn, a in args]
    mixed = [srv.wait(t) for t in tickets]
    assert srv.info()["max_round_size"] == 1
    for a, m in zip(alone, mixed):
        for f in FAM:
            assert m[f] == a[f]
    srv.close()
    # an arena smaller than a request: refused at submit
    srv = gpu_lib.Server(hbm_budget_bytes=1 << 30, arena_bytes=4096)
    _add_tenants(srv, sv)
    big = max(args, key=lambda ta: len(ta[1][2]))
    with pytest.raises(gpu_lib.HgtError) as e:
        srv.submit(big[0], *big[1])
    assert e.value.code == gpu_lib.ENOMEM
    srv.close()


def test_served_rejected_request_leaves_tenant_unchanged(gpu_lib):
    sv = _mini(seed=7, n_tenants=3, n_requests=10)
    args, alone = _alone_with_oracle(gpu_lib, sv)
    srv = gpu_lib.Server(hbm_budget_bytes=1 << 30, arena_bytes=64 << 20)
    _add_tenants(srv, sv)
    tn0, a0 = args[0]
    bad = (np.array([10 ** 6], np.uint32),) + a0[1:]  # deletes an ID that is not live
    t_bad = srv.submit(tn0, *bad)
    tickets = [srv.submit(tn, *a) for tn, a in args]
    r_bad = srv.wait(t_bad)
    assert r_bad["status"] == gpu_lib.ENOENT
    mixed = [srv.wait(t) for t in tickets]
    for a, m in zip(alone, mixed):
        assert m["status"] == gpu_lib.OK
        for f in FAM:
            assert m[f] == a[f]
    srv.close()
