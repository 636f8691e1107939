"""Host-side helpers of bench.py: the roofline figure of the dominant kernel
group and the committed counter traffic it reports."""
import json
import os

import pytest

import bench


def _prof(**groups):
    return {k: dict(launches=v[0], total_ms=v[1], algo_bytes=v[2], events=0, aux=0) for k, v in groups.items()}


def test_roofline_takes_the_dominant_group():
    prof = _prof(he_hist_global=(4, 40.0, 8_000_000_000), iv_pairs=(4, 60.0, 4_000_000_000),
                 store_plan=(2, 1.0, 0))
    rl = bench.roofline_of(prof)
    assert rl["kernel"] == "iv_pairs"
    assert rl["avg_launch_ms"] == pytest.approx(15.0)
    assert rl["algo_bytes_per_launch"] == 1_000_000_000
    # achieved = algorithmic bytes / summed time: 4 GB in 60 ms
    assert rl["achieved"] == pytest.approx(4e9 / 60e-3 / 1e9, rel=1e-3)
    assert rl["frac"] == pytest.approx(rl["achieved"] / bench.HBM_PEAK_GBS, rel=1e-3)


def test_roofline_store_only_joins_plan_and_commit():
    prof = _prof(store_plan=(2, 3.0, 0), store_commit=(2, 1.0, 40_000_000))
    rl = bench.roofline_of(prof, store_only=True)
    assert rl["kernel"] == "store_plan+store_commit"
    assert rl["avg_launch_ms"] == pytest.approx(2.0)
    assert rl["achieved"] == pytest.approx(40e6 / 4e-3 / 1e9, rel=1e-3)


def test_traffic_only_for_the_sources_it_was_taken_on(tmp_path, monkeypatch):
    prof_dir = tmp_path / "profiles"
    prof_dir.mkdir()
    doc = {"source_sha256": bench.source_digest(), "workload": "w",
           "groups": {"g": {"fetch_bytes_per_launch": 100, "write_bytes_per_launch": 20}}}
    (prof_dir / "w_traffic.json").write_text(json.dumps(doc))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # the digest is taken over the sources under ROOT; keep the real ones
    digest = doc["source_sha256"]
    monkeypatch.setattr(bench, "source_digest", lambda: digest)
    assert bench.traffic_of("w", "g") == 120
    assert bench.traffic_of("w", "other") is None
    assert bench.traffic_of("missing", "g") is None
    doc["source_sha256"] = "0" * 64
    (prof_dir / "w_traffic.json").write_text(json.dumps(doc))
    assert bench.traffic_of("w", "g") is None


def test_committed_traffic_matches_the_sources():
    """The committed counter summaries were taken on the current HIP sources."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for wl, group in (("medium", "iv_pairs"), ("temporal", "temporal")):
        with open(os.path.join(root, "profiles", f"{wl}_traffic.json")) as f:
            assert json.load(f)["source_sha256"] == bench.source_digest(), wl
        assert bench.traffic_of(wl, group) > 0


def _fake_result(workload, **extra):
    r = {k: 1 for k in bench.LEG_KEYS}
    r["config"] = {"workload": workload, "launch": "graph"}
    r.update(extra)
    return r


def test_legs_are_reported_and_a_failing_leg_is_contained(monkeypatch):
    """The default (Medium) line carries a temporal and a batched leg; a leg
    that raises reports its error instead of taking the line down."""
    import types
    import paper_2512_21009_amd.workloads as W
    calls = []

    def fake_single(la, st, track, name, wl):
        calls.append(("single", la.warmup, la.steps, la.prof_steps, track, name))
        return _fake_result(wl)

    def fake_batched(la, only):
        calls.append(("batched", la.warmup, la.steps, la.prof_steps, tuple(only)))
        return _fake_result("b", plain={"value": 1}, stream={"value": 6}, graph={"value": 6},
                            speedup_vs_plain=6.0), []

    monkeypatch.setattr(bench, "bench_single", fake_single)
    monkeypatch.setattr(bench, "bench_batched", fake_batched)
    monkeypatch.setattr(W, "temporal", lambda scale, n_batches: types.SimpleNamespace(scale=scale, n=n_batches))
    args = bench.parse(["--quiet"])
    assert args.legs == "temporal,batched"
    legs = bench.run_legs(args)
    assert set(legs) == {"temporal", "batched"}
    assert legs["temporal"]["workload"] == bench.WL_TEMPORAL
    assert legs["batched"]["speedup_vs_plain"] == 6.0 and legs["batched"]["launch"] == "graph"
    assert ("single", 1, 2, 1, ("temporal",), "temporal") in calls
    assert ("batched", 1, 2, 1, ("plain", "stream", "graph")) in calls
    # the caller's arguments are left as they were
    assert (args.warmup, args.steps) == (1, 9)

    def broken(la, only):
        raise RuntimeError("no box")

    monkeypatch.setattr(bench, "bench_batched", broken)
    legs = bench.run_legs(bench.parse(["--quiet", "--legs", "batched,nosuch"]))
    assert legs["batched"]["error"] == "RuntimeError: no box"
    assert "unknown leg" in legs["nosuch"]["error"]
