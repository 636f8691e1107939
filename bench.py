#!/usr/bin/env python
"""Hyperedge updates/s including the triad-count update, on one MI355X.

A step is one batch through the whole hot path: validation and
canonicalisation, the triad deltas on the old graph, the store delete/insert,
the deltas on the new graph and the count update.  Inputs are synthetic and
resident in HBM before timing starts.  Workloads (--config):

  medium   (default) 1M vertices, 2M hyperedges, cardinality power law 2.5 on
           [2,64], vertex popularity (rank + 1e4)^-1.1, batches of 50k inserts
           + 50k deletions of uniformly chosen live hyperedges; hyperedge and
           incident-vertex triads.
  temporal 500k vertices, 4M hyperedges, cardinality power law 2.2 on [2,128],
           Poisson arrivals at 1e3/s, batches of 200k arrivals with expiry of
           hyperedges older than 3600 s; temporal triads within 600 s.
  batched  256 graphs, |E| log-uniform in [1k,200k], |V| = |E|/2, cardinality
           power law 2.5 on [2,256], per-graph batches log-uniform in [10,50k]
           (60% inserts); hyperedge triads.  Every round is timed twice on
           identical copies: one hgt_apply_batch call per graph (plain) and one
           hgt_apply_batches call for all graphs (batched).
  served   64 tenants totalling 20M hyperedges (|V_t| = |E_t|/2), cardinality
           power law 2.0 on [2,256], popularity (rank + 3e3)^-1.3, Poisson
           timestamps, every family tracked (temporal window 600 s); requests
           of log-uniform size in [1,1e5] (half inserts) for uniform tenants.
           All requests are first applied one at a time with hgt_apply_batch
           on one copy of the tenants (plain), then submitted together to a
           request server holding another copy (served); every request's
           counts must agree.  p50/p99 are per request, submission to completion.

Prints one JSON line.  Only one GPU is used.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "hyperedge updates/sec incl. triad-count update; p50/p99 batch latency"


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=9)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--prof-steps", type=int, default=2,
                    help="batches applied after the timed region with HIP-event profiling on (roofline)")
    ap.add_argument("--phases", action="store_true",
                    help="also record the hyperedge-delta stages' wall-clock phase timers in the profiled pass")
    ap.add_argument("--config", choices=("medium", "temporal", "batched", "served", "dyadic", "static", "sweep",
                                         "horizontal", "literal-store"),
                    default="medium")
    ap.add_argument("--sweep-sizes", default="20e6,30e6,40e6,55e6", help="sweep: hyperedge counts")
    ap.add_argument("--requests", type=int, default=256, help="served: number of requests")
    ap.add_argument("--launch", choices=("stream", "graph", "tuned"), default="graph",
                    help="served: rounds launched kernel by kernel, as captured HIP graphs, or as graphs with the "
                         "autotuner's launch choices")
    ap.add_argument("--rate-multiples", default="0.5,1,2,4",
                    help="served: offered request rates as multiples of the plain path's request rate")
    ap.add_argument("--scale", type=float, default=1.0, help="workload scale (1.0 = the named configuration)")
    ap.add_argument("--cpu-sample", type=int, default=600, help="updates in the oracle's timed sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-static-baseline", action="store_true",
                    help="skip the oracle's one-thread static recount of the scaled-down workload")
    ap.add_argument("--legs", default="temporal,batched",
                    help="medium only: further workloads measured in the same run and reported in the same JSON "
                         "line under 'legs' (temporal at full size; batched, one call per graph against one call "
                         "for all); 'none' for none")
    ap.add_argument("--quiet", action="store_true")
    return ap.parse_args(argv)


def log(args, *a):
    if not args.quiet:
        print("[bench]", *a, file=sys.stderr, flush=True)


def to_dev(a, dt):
    import numpy as np
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).astype(dt)).to("cuda:0")


def roofline_of(prof, store_only=False):
    """Dominant kernel group of the timed region: its algorithmic bytes per
    launch over its average launch duration (HIP events on the launch stream).
    Store only (no triad family): the store's planning and commit groups
    together, against the update's algorithmic bytes (counted by the commit)."""
    if store_only and "store_commit" in prof and "store_plan" in prof:
        pl, cm = prof["store_plan"], prof["store_commit"]
        ms = pl["total_ms"] + cm["total_ms"]
        n = max(1, cm["launches"])
        achieved = cm["algo_bytes"] / (ms * 1e6) if ms > 0 else 0.0
        return {"bound": "hbm", "kernel": "store_plan+store_commit", "achieved": round(achieved, 2),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                "avg_launch_ms": round(ms / n, 4), "algo_bytes_per_launch": int(cm["algo_bytes"] // n)}
    live = [(n, r) for n, r in prof.items() if r["launches"]]
    dom_name, dom = max(live, key=lambda kv: kv[1]["total_ms"])
    achieved = dom["algo_bytes"] / (dom["total_ms"] * 1e6) if dom["total_ms"] > 0 else 0.0
    return {"bound": "hbm", "kernel": dom_name, "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
            "avg_launch_ms": round(dom["total_ms"] / dom["launches"], 4),
            "algo_bytes_per_launch": int(dom["algo_bytes"] // dom["launches"])}


def source_digest():
    """sha256 over the HIP sources: counter figures taken on other sources are stale."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2512_21009_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode() + b"\0" + fh.read())
    return h.hexdigest()


def traffic_of(workload, group):
    """HBM bytes per launch of `group` from the committed rocprofv3 counter
    summary of this workload (FETCH_SIZE + WRITE_SIZE, each scaled by a plain
    copy of known size), or None when there is none for these sources."""
    path = os.path.join(ROOT, "profiles", f"{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("source_sha256") != source_digest():
        return None
    g = t.get("groups", {}).get(group)
    if not g:
        return None
    return int(g["fetch_bytes_per_launch"] + g["write_bytes_per_launch"])


def log_profile(args, prof):
    for name, r in prof.items():
        if r["launches"]:
            gbs = r["algo_bytes"] / (r["total_ms"] * 1e6) if r["total_ms"] > 0 else 0.0
            log(args, f"  {name:16s} launches={r['launches']:5d} total={r['total_ms']:9.2f}ms "
                      f"algo={r['algo_bytes'] / 1e9:8.3f}GB ({gbs:7.1f} GB/s) events={r['events']} aux={r['aux']}")


PHASES = ("prefix", "nbr-hash", "compact", "disjoint", "group", "open", "pairs", "hand-over", "pairs-short",
          "pairs-vpairs", "pairs-long")


def log_phases(args, ctr):
    """Share of wall-clock ticks per phase of each hyperedge-delta stage."""
    for s in range(3):
        ph = [int(x) for x in ctr[16 + 12 * s: 16 + 12 * s + len(PHASES)]]
        tot = sum(ph)
        if tot:
            log(args, f"  stage {s} phases: " + " ".join(f"{n}={100.0 * v / tot:.1f}%" for n, v in zip(PHASES, ph)))
            # the wall clock the kernels read runs at 100 MHz
            log(args, f"  stage {s}: longest single centre {int(ctr[16 + 12 * s + 11]) / 1e5:.2f} ms")
    log(args, f"  aggregated pairs: long runs {int(ctr[12])}, pairs sharing several vertices {int(ctr[13])}, "
              f"centres enumerated {int(ctr[14])}")


def add_profiles(acc, prof):
    for k, r in prof.items():
        a = acc.setdefault(k, dict(launches=0, total_ms=0.0, algo_bytes=0, events=0, aux=0))
        for f in a:
            a[f] += r[f]
    return acc


def calibration_copy():
    """A plain device copy of known size (256 MiB read + 256 MiB written), run
    outside the timed region: profiler byte counters are scaled by it."""
    import torch
    calib = torch.empty(1 << 26, dtype=torch.int32, device="cuda:0")
    calib.fill_(1)
    calib.clone()
    torch.cuda.synchronize()


def ids_of_stream(hgt, st, ins):
    """Deletion IDs of every batch: a store-only replay (no triad families)
    gives the IDs the library assigns, the same as in any tracked copy."""
    import numpy as np
    import torch
    ini = st.initial
    g0 = hgt.Graph.build(st.n_vertices, to_dev(ini.offsets, np.int64), to_dev(ini.members, np.int32), track=())
    n_handles = ini.n + sum(b.ins.n for b in st.batches)
    hid = np.full(n_handles, -1, np.int64)
    hid[: ini.n] = np.arange(ini.n)
    dels = []
    for b, (io, im) in zip(st.batches, ins):
        di = hid[b.del_handles]
        assert (di >= 0).all()
        dt = to_dev(di, np.int32) if len(di) else None
        dels.append(dt)
        out = g0.apply_batch(dt, io, im)
        if out is not None:
            hid[b.ins_handles] = out.cpu().numpy()
    g0.close()
    torch.cuda.synchronize()
    return dels


def bench_single(args, st, track, name, workload):
    """One graph, one hgt_apply_batch call per step."""
    import numpy as np
    import torch
    from paper_2512_21009_amd import hgt
    temporal = "temporal" in track
    ini = st.initial
    off0, mem0 = to_dev(ini.offsets, np.int64), to_dev(ini.members, np.int32)
    ts0 = to_dev(ini.ts, np.int64) if temporal else None
    ins = [(to_dev(b.ins.offsets, np.int64) if b.ins.n else None, to_dev(b.ins.members, np.int32) if b.ins.n else None)
           for b in st.batches]
    its = [to_dev(b.ins.ts, np.int64) if (temporal and b.ins.n) else None for b in st.batches]
    dels = ids_of_stream(hgt, st, ins)
    t0 = time.perf_counter()
    g = hgt.Graph.build(st.n_vertices, off0, mem0, ts0, track=track, window=st.window)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    log(args, f"build with initial counts: {build_s:.2f}s")
    n_b = len(st.batches)
    n_timed_end = args.warmup + args.steps
    for k in range(args.warmup):
        g.apply_batch(dels[k], *ins[k], its[k])
    torch.cuda.synchronize()
    # timed region: no profiling
    lat, n_upd = [], 0
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.warmup, n_timed_end):
        tb = time.perf_counter()
        g.apply_batch(dels[k], *ins[k], its[k])
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - tb)
        n_upd += st.batches[k].n_updates
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    # profiled pass over the next batches (same shape): HIP events around each kernel
    # group on the launch stream and the kernels' algorithmic-byte counters
    g.profile(2 if args.phases else 1)
    for k in range(n_timed_end, n_b):
        g.apply_batch(dels[k], *ins[k], its[k])
    torch.cuda.synchronize()
    prof = g.profile_read()
    if args.phases:
        log_phases(args, g.profile_counters())
    g.profile(0)
    status = g.sync()
    assert status == hgt.OK, status
    value = n_upd / elapsed
    log(args, f"{n_upd} updates in {elapsed:.3f}s -> {value:,.0f} updates/s")
    log(args, f"profiled pass: {n_b - n_timed_end} batches")
    log_profile(args, prof)
    totals = {k: int(sum(g.triad_counts(k))) for k in track}
    g.close()
    calibration_copy()
    lat_ms = np.array(lat) * 1e3
    rl = roofline_of(prof, store_only=not track)
    rl["traffic"] = traffic_of(name, rl["kernel"])
    return {
        "metric": METRIC, "value": round(value, 1), "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(elapsed / max(args.steps, 1) * 1e3, 3),
        "p50_ms": round(float(np.percentile(lat_ms, 50)), 3), "p99_ms": round(float(np.percentile(lat_ms, 99)), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": workload, "scale": args.scale, "batch_updates": int(st.batches[-1].n_updates),
                   "build_s": round(build_s, 3), "triads_total": totals},
        "roofline": rl,
        "roofline_pass": f"{n_b - n_timed_end} batches after the timed region, HIP events on",
    }


BATCHED_VARIANTS = ("plain", "stream", "graph", "tuning", "tuned")


def bench_batched(args, only=BATCHED_VARIANTS):
    """256 graphs; each round applies every graph's next batch.  Identical
    copies take the same rounds (`warmup` untimed, then `steps` timed): one
    call per graph (plain); one call for all with the kernels launched one by
    one (stream); the same launched as one captured HIP graph per round
    (graph); and the graph launch with the autotuner's choices (tuned), after a
    pass over the same rounds on a copy of its own in which the tuner times its
    choices.  The rounds after the timed ones are profiled on the stream copy.
    `only` keeps a subset of the variants (plain and stream always run)."""
    import numpy as np
    import torch
    from paper_2512_21009_amd import hgt
    from paper_2512_21009_amd import workloads as W
    n_timed_beg = args.warmup
    n_timed_end = n_timed_beg + args.steps
    n_b = n_timed_end + max(1, args.prof_steps)
    t0 = time.perf_counter()
    sc = args.scale
    sts = W.batched(n_batches=n_b, e_lo=max(100.0, 1e3 * sc), e_hi=max(1e3, 2e5 * sc), b_hi=max(20.0, 5e4 * sc))
    log(args, f"generated {len(sts)} graphs, {sum(s.initial.n for s in sts)} hyperedges, "
              f"{sum(s.batches[0].n_updates for s in sts)} updates per round in {time.perf_counter() - t0:.1f}s")
    ins = [[(to_dev(b.ins.offsets, np.int64) if b.ins.n else None, to_dev(b.ins.members, np.int32) if b.ins.n else None)
            for b in st.batches] for st in sts]
    dels = []
    for gi, (st, i) in enumerate(zip(sts, ins)):
        dels.append(ids_of_stream(hgt, st, i))
        if gi % 64 == 63:
            log(args, f"deletion IDs replayed for {gi + 1} graphs")
    track = ("hyperedge",)

    def build_all():
        out = []
        for st in sts:
            ini = st.initial
            out.append(hgt.Graph.build(st.n_vertices, to_dev(ini.offsets, np.int64), to_dev(ini.members, np.int32),
                                       track=track))
        torch.cuda.synchronize()
        return out

    ups = [sum(st.batches[k].n_updates for st in sts) for k in range(n_b)]
    variants = [("plain", None), ("stream", {}), ("graph", {"graph": True}),
                ("tuning", {"graph": True, "autotune": True}), ("tuned", {"graph": True, "autotune": True})]
    variants = [v for v in variants if v[0] in only or v[0] in ("plain", "stream")]
    names = [v[0] for v in variants]
    lat, counts, prof = {}, {}, {}
    build_s = 0.0
    settled = None
    for name, kw in variants:
        t0 = time.perf_counter()
        gs = build_all()
        build_s = time.perf_counter() - t0
        lat[name] = []
        log(args, f"{name}: built in {build_s:.2f}s")
        rounds = n_b if name == "stream" else n_timed_end
        for k in range(rounds):
            if name == "stream" and k == n_timed_end:  # the rounds after the timed ones are profiled
                for g in gs:
                    g.profile(2 if args.phases else 1)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            if kw is None:
                for gi, g in enumerate(gs):
                    g.apply_batch(dels[gi][k], *ins[gi][k])
            else:
                hgt.apply_batches([(g, dels[gi][k]) + ins[gi][k] for gi, g in enumerate(gs)], **kw)
            torch.cuda.synchronize()
            dt = time.perf_counter() - tb
            if n_timed_beg <= k < n_timed_end:
                lat[name].append(dt)
            log(args, f"{name}: round {k} ({ups[k]} updates) {dt * 1e3:.1f} ms")
            if name == "stream" and k == n_timed_end - 1:
                counts["stream@timed"] = [g.triad_counts("hyperedge") for g in gs]
        if name == "stream":
            for g in gs:
                add_profiles(prof, g.profile_read())
            if args.phases:  # counters of all graphs: sums, and the maxima of the longest-centre slots
                ctrs = [list(g.profile_counters()) for g in gs]
                tot = [sum(c[i] for c in ctrs) for i in range(len(ctrs[0]))]
                for st_ in range(3):
                    tot[16 + 12 * st_ + 11] = max(c[16 + 12 * st_ + 11] for c in ctrs)
                log_phases(args, tot)
        counts[name] = [g.triad_counts("hyperedge") for g in gs]
        for g in gs:
            assert g.sync() == hgt.OK
            g.close()
        log(args, f"{name}: {sum(ups[n_timed_beg:n_timed_end]) / sum(lat[name]):,.0f} updates/s "
                  f"(build {build_s:.2f}s)")
        if name == "tuning":
            settled = hgt.tune_flush()
    for name in names:
        if name != "stream":
            assert counts[name] == counts["stream@timed"], f"{name} and stream counts differ"
    total = sum(sum(c) for c in counts["stream@timed"])
    calibration_copy()
    n_upd = sum(ups[n_timed_beg:n_timed_end])
    rate = {name: n_upd / sum(lat[name]) for name, _ in variants}
    ms = {name: np.array(lat[name]) * 1e3 for name, _ in variants}
    best = max((n for n in ("stream", "graph", "tuned") if n in names), key=lambda n: rate[n])
    log(args, ", ".join(f"{n} {rate[n]:,.0f}" for n in names if n != "tuning") +
        f" updates/s; tuner keys settled: {settled}")
    log_profile(args, prof)

    def leg(n):
        return {"value": round(rate[n], 1), "ms_per_step": round(float(ms[n].mean()), 3),
                "p50_ms": round(float(np.percentile(ms[n], 50)), 3), "p99_ms": round(float(np.percentile(ms[n], 99)), 3)}

    return {
        "metric": METRIC, "value": round(rate[best], 1), "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": n_timed_beg, "ms_per_step": round(float(ms[best].mean()), 3),
        "p50_ms": round(float(np.percentile(ms[best], 50)), 3), "p99_ms": round(float(np.percentile(ms[best], 99)), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "batched: 256 graphs, |E| log-uniform [1k,200k], |V|=|E|/2, card power-law 2.5 on "
                               "[2,256], batches log-uniform [10,50k] (60% inserts), hyperedge triads",
                   "scale": sc, "round_updates": int(np.mean(ups[n_timed_beg:n_timed_end])),
                   "build_s_per_copy": round(build_s, 3), "launch": best,
                   "he_triads_total": int(total)},
        **{n: leg(n) for n in names if n != "tuning"},
        "tuner_keys_settled": settled,
        "speedup_vs_plain": round(rate[best] / rate["plain"], 3),
        "roofline": roofline_of(prof),
    }, sts


def bench_served(args):
    """Served form: every request is first applied alone, one at a time, on one
    copy of the tenants (plain); then, on another copy held by a request
    server, the requests arrive as a Poisson stream: consecutive segments of the
    generator's arrival sequence are replayed at rates that are multiples of
    the plain path's request rate (the arrival gaps rescaled), the last
    segment submitted at once (saturation).  Every served result must equal the
    plain one.  p50/p99 per rate are per request, submission to completion."""
    import numpy as np
    import torch
    from paper_2512_21009_amd import hgt
    from paper_2512_21009_amd import workloads as W
    fams = W.FAMILIES
    t0 = time.perf_counter()
    sc = args.scale
    gen_rate = 1000.0  # requests/s of the generator's arrival process
    sv = W.served(total_edges=20e6 * sc, n_requests=args.requests, req_hi=max(10.0, 1e5 * sc), card_hi=256,
                  rate_per_s=gen_rate)
    n_req = len(sv.arrivals)
    log(args, f"generated {len(sv.tenants)} tenants, {sum(t.initial.n for t in sv.tenants)} hyperedges, "
              f"{n_req} requests in {time.perf_counter() - t0:.1f}s")
    ins = [[(to_dev(b.ins.offsets, np.int64) if b.ins.n else None, to_dev(b.ins.members, np.int32) if b.ins.n else None)
            for b in st.batches] for st in sv.tenants]
    dels = [ids_of_stream(hgt, st, i) for st, i in zip(sv.tenants, ins)]
    log(args, "deletion IDs replayed")
    del_host = [[d.cpu().numpy().astype(np.uint32) if d is not None else np.zeros(0, np.uint32) for d in dl]
                for dl in dels]
    its = [[to_dev(b.ins.ts, np.int64) if b.ins.n else None for b in st.batches] for st in sv.tenants]

    def build_args(st):
        ini = st.initial
        return (st.n_vertices, to_dev(ini.offsets, np.int64), to_dev(ini.members, np.int32), to_dev(ini.ts, np.int64))

    t0 = time.perf_counter()
    plain = []
    for i, st in enumerate(sv.tenants):
        plain.append(hgt.Graph.build(*build_args(st), track=fams, window=st.window))
        torch.cuda.synchronize()
        if i % 16 == 15:
            log(args, f"plain: {i + 1} tenants built, {time.perf_counter() - t0:.1f}s")
    build_s = time.perf_counter() - t0
    ups = [sv.tenants[tn].batches[k].n_updates for (_, tn, k, _) in sv.arrivals]
    # plain: one request at a time, in arrival order
    lat_p, want = [], []
    for i, (_, tn, k, fam) in enumerate(sv.arrivals):
        g = plain[tn]
        torch.cuda.synchronize()
        tb = time.perf_counter()
        g.apply_batch(dels[tn][k], *ins[tn][k], its[tn][k])
        torch.cuda.synchronize()
        lat_p.append(time.perf_counter() - tb)
        want.append(g.triad_counts(fam))
        if i % 64 == 63:
            log(args, f"plain: {i + 1} requests, {sum(lat_p):.2f}s")
    for g in plain:
        assert g.sync() == hgt.OK
        g.close()
    del plain
    plain_rate = n_req / sum(lat_p)
    # served: a server over an identical copy
    srv = hgt.Server(hbm_budget_bytes=64 << 30, arena_bytes=2 << 30, graph=args.launch != "stream",
                     autotune=args.launch == "tuned")
    for i, st in enumerate(sv.tenants):
        srv.add_tenant(*build_args(st), track=fams, window=st.window)
        if i % 16 == 15:
            log(args, f"server: {i + 1} tenants built")
    torch.cuda.synchronize()
    reqs = []
    for (_, tn, k, fam) in sv.arrivals:
        b = sv.tenants[tn].batches[k]
        reqs.append((tn, del_host[tn][k], b.ins.offsets.astype(np.uint64), b.ins.members.astype(np.uint32),
                     b.ins.ts.astype(np.int64)))
    mults = [float(x) for x in args.rate_multiples.split(",")]
    seg = np.array_split(np.arange(n_req), len(mults) + 1)  # the last segment: all at once
    arr_us = np.array([a[0] for a in sv.arrivals])
    res = [None] * n_req
    sweep = []
    for si, idx in enumerate(seg):
        rate = plain_rate * mults[si] if si < len(mults) else float("inf")
        offs = (arr_us[idx] - arr_us[idx[0]]) * 1e-6 * (gen_rate / rate) if si < len(mults) else np.zeros(len(idx))
        t_start = time.perf_counter()
        tickets = []
        for j, off in zip(idx, offs):
            while time.perf_counter() - t_start < off:
                time.sleep(min(0.001, max(0.0, off - (time.perf_counter() - t_start))))
            tickets.append((j, srv.submit(*reqs[j])))
        for j, t in tickets:
            res[j] = srv.wait(t)
        el = time.perf_counter() - t_start
        lat = np.array([(res[j]["t_done_ns"] - res[j]["t_submit_ns"]) * 1e-6 for j in idx])
        n_u = int(sum(ups[j] for j in idx))
        sweep.append({"rate_req_per_s": None if rate == float("inf") else round(rate, 2),
                      "offered": "all at once" if rate == float("inf") else f"{mults[si]}x plain request rate",
                      "requests": len(idx), "updates_per_s": round(n_u / el, 1),
                      "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
                      "plain_updates_per_s": round(n_u / sum(lat_p[j] for j in idx), 1)})
        log(args, f"served segment {si}: {sweep[-1]}")
    info = srv.info()
    for i, (r, (_, tn, k, fam)) in enumerate(zip(res, sv.arrivals)):
        assert r["status"] == hgt.OK, (i, r["status"])
        assert r[fam] == want[i], f"request {i}: served and plain counts differ"
    srv.close()
    calibration_copy()
    sat = sweep[-1]
    v_s = sat["updates_per_s"]
    v_p = sat["plain_updates_per_s"]
    lp = np.array(lat_p) * 1e3
    log(args, f"saturation: served {v_s:,.0f} updates/s vs plain {v_p:,.0f} ({v_s / v_p:.2f}x); "
              f"rounds {info['rounds']}, largest round {info['max_round_size']}, rounds in flight {info['max_inflight_seen']}")
    return {
        "metric": METRIC, "value": v_s, "unit": "updates/s", "n_gpus": 1, "steps": n_req, "warmup": 0,
        "ms_per_step": None, "p50_ms": sat["p50_ms"], "p99_ms": sat["p99_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "served: 64 tenants, |V_t|=|E_t|/2, card power-law 2.0 on [2,256] (cap), popularity "
                               "(rank+3e3)^-1.3, Poisson timestamps, requests log-uniform [1,1e5*scale] (half "
                               "inserts), all families tracked, Poisson arrivals swept to saturation",
                   "scale": sc, "total_hyperedges": int(sum(t.initial.n for t in sv.tenants)), "requests": n_req,
                   "build_s": round(build_s, 3), "rounds": info["rounds"], "max_round_size": info["max_round_size"],
                   "max_rounds_in_flight": info["max_inflight_seen"], "launch": args.launch},
        "plain": {"value": v_p, "request_rate": round(plain_rate, 2), "p50_ms": round(float(np.percentile(lp, 50)), 3),
                  "p99_ms": round(float(np.percentile(lp, 99)), 3)},
        "speedup_vs_plain": round(v_s / v_p, 3),
        "rate_sweep": sweep,
        "roofline": None,
    }, sv


def bench_static(args):
    """The paper's comparison setting on the Medium workload: each batch applied
    incrementally (timed), then the counts of the resulting hypergraph
    recomputed from scratch on the GPU (a build of the live hyperedges, which
    counts every triad of both families; timed, inputs resident in HBM)."""
    import numpy as np
    import torch
    from paper_2512_21009_amd import hgt
    from paper_2512_21009_amd import workloads as W
    n_b = args.warmup + args.steps
    st = W.medium(q=1.0e4, scale=args.scale, n_batches=n_b)
    track = ("hyperedge", "incident_vertex")
    ins = [(to_dev(b.ins.offsets, np.int64), to_dev(b.ins.members, np.int32)) for b in st.batches]
    dels = ids_of_stream(hgt, st, ins)
    ini = st.initial
    g = hgt.Graph.build(st.n_vertices, to_dev(ini.offsets, np.int64), to_dev(ini.members, np.int32), track=track)
    inc, rec, n_upd = [], [], 0
    for k in range(n_b):
        torch.cuda.synchronize()
        tb = time.perf_counter()
        g.apply_batch(dels[k], *ins[k])
        torch.cuda.synchronize()
        t_inc = time.perf_counter() - tb
        if k < args.warmup:
            continue
        inc.append(t_inc)
        n_upd += st.batches[k].n_updates
        off, mem, live = g.export_h2v()
        rows = np.nonzero(live)[0].astype(np.int64)
        lens = np.diff(off.astype(np.int64))[rows]
        r_off = np.zeros(len(rows) + 1, np.int64)
        r_off[1:] = np.cumsum(lens)
        d_off, d_mem = to_dev(r_off, np.int64), to_dev(mem, np.int32)  # dead rows are empty: mem is the live rows
        torch.cuda.synchronize()
        tb = time.perf_counter()
        g2 = hgt.Graph.build(st.n_vertices, d_off, d_mem, track=track)
        torch.cuda.synchronize()
        rec.append(time.perf_counter() - tb)
        same = all(g2.triad_counts(f) == g.triad_counts(f) for f in track)
        g2.close()
        assert same, "static recount and incremental counts differ"
        log(args, f"batch {k}: incremental {inc[-1] * 1e3:.1f} ms, static recount {rec[-1] * 1e3:.1f} ms")
    g.close()
    inc_ms, rec_ms = np.array(inc) * 1e3, np.array(rec) * 1e3
    return {
        "metric": METRIC, "value": round(n_upd / sum(inc), 1), "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(float(inc_ms.mean()), 3),
        "p50_ms": round(float(np.percentile(inc_ms, 50)), 3), "p99_ms": round(float(np.percentile(inc_ms, 99)), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "static recount vs incremental on medium: 1M vertices, 2M hyperedges, batches 50k ins "
                               "+ 50k del, hyperedge + incident-vertex triads", "scale": args.scale},
        "static_recount": {"ms_p50": round(float(np.percentile(rec_ms, 50)), 3),
                           "incremental_ms_p50": round(float(np.percentile(inc_ms, 50)), 3),
                           "speedup_incremental_over_static": round(float(np.percentile(rec_ms, 50)
                                                                          / np.percentile(inc_ms, 50)), 2)},
        "roofline": None,
    }, st


def bench_sweep(args):
    """The paper's scaling sweep: random hypergraphs of the given sizes,
    |V| = |E|/3, cardinality power law 3.0 on [2, 8192] (the library's
    largest cardinality; the paper's maximum is 10000 and its law is not
    stated), 50k changes per batch (half deletions), hyperedge triads.  One
    point per size."""
    import numpy as np
    import torch
    from paper_2512_21009_amd import hgt
    from paper_2512_21009_amd import workloads as W
    n_b = args.warmup + args.steps
    points = []
    for n in [int(float(x)) for x in args.sweep_sizes.split(",")]:
        t0 = time.perf_counter()
        st = W.random_hypergraph(n, alpha=3.0, n_batches=n_b)
        log(args, f"sweep {n}: generated in {time.perf_counter() - t0:.1f}s ({st.initial.members.size} incidences)")
        ins = [(to_dev(b.ins.offsets, np.int64), to_dev(b.ins.members, np.int32)) for b in st.batches]
        dels = ids_of_stream(hgt, st, ins)
        log(args, f"sweep {n}: deletion IDs replayed")
        ini = st.initial
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = hgt.Graph.build(st.n_vertices, to_dev(ini.offsets, np.int64), to_dev(ini.members, np.int32),
                            track=("hyperedge",))
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        log(args, f"sweep {n}: built in {build_s:.1f}s")
        lat, n_upd = [], 0
        for k in range(n_b):
            torch.cuda.synchronize()
            tb = time.perf_counter()
            g.apply_batch(dels[k], *ins[k])
            torch.cuda.synchronize()
            if k >= args.warmup:
                lat.append(time.perf_counter() - tb)
                n_upd += st.batches[k].n_updates
        assert g.sync() == hgt.OK
        g.close()
        del ins, dels
        torch.cuda.empty_cache()
        ms = float(np.mean(lat)) * 1e3
        points.append({"hyperedges": n, "vertices": st.n_vertices, "incidences": int(ini.members.size),
                       "build_s": round(build_s, 3), "ms_per_batch": round(ms, 3),
                       "updates_per_s": round(n_upd / sum(lat), 1)})
        log(args, f"sweep {n}: build {build_s:.1f}s, {ms:.1f} ms per 50k-change batch")
    last = points[-1]
    return {
        "metric": METRIC, "value": last["updates_per_s"], "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": last["ms_per_batch"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "random hypergraph sweep: |V| = |E|/3, card power-law 3.0 on [2,8192], uniform "
                               "popularity, 50k changes per batch, hyperedge triads; value at the largest size"},
        "sweep": points, "roofline": None,
    }


def bench_horizontal(args):
    """Horizontal operations on the Medium workload (the paper's incident-vertex
    modification batches): batches of 100k ops (half insertions of a vertex
    into a hyperedge, half deletions of a member) on uniform hyperedges,
    hyperedge + incident-vertex triads updated; updates = ops."""
    import numpy as np
    import torch
    from paper_2512_21009_amd import hgt
    from paper_2512_21009_amd import workloads as W
    n_b = args.warmup + args.steps
    st = W.medium(q=1.0e4, scale=args.scale, n_batches=0)
    t0 = time.perf_counter()
    ops = W.vertex_op_batches(st, n_b, max(2, int(100_000 * args.scale)))
    log(args, f"generated {n_b} batches of {len(ops[0].edge_ids)} vertex ops in {time.perf_counter() - t0:.1f}s")
    dev_ops = [(to_dev(o.edge_ids, np.int32), to_dev(o.vertices, np.int32), to_dev(o.insert.astype(np.uint8), np.uint8))
               for o in ops]
    ini = st.initial
    track = ("hyperedge", "incident_vertex")
    g = hgt.Graph.build(st.n_vertices, to_dev(ini.offsets, np.int64), to_dev(ini.members, np.int32), track=track)
    lat, n_upd = [], 0
    for k in range(n_b):
        torch.cuda.synchronize()
        tb = time.perf_counter()
        g.apply_vertex_ops(*dev_ops[k])
        torch.cuda.synchronize()
        if k >= args.warmup:
            lat.append(time.perf_counter() - tb)
            n_upd += len(ops[k].edge_ids)
    assert g.sync() == hgt.OK
    totals = {f: int(sum(g.triad_counts(f))) for f in track}
    g.close()
    ms = np.array(lat) * 1e3
    return {
        "metric": METRIC, "value": round(n_upd / sum(lat), 1), "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(float(ms.mean()), 3),
        "p50_ms": round(float(np.percentile(ms, 50)), 3), "p99_ms": round(float(np.percentile(ms, 99)), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "horizontal: medium (1M vertices, 2M hyperedges), batches of 100k incident-vertex "
                               "ops (50k insertions, 50k deletions) on uniform hyperedges, hyperedge + "
                               "incident-vertex triads", "scale": args.scale, "triads_total": totals},
        "roofline": None,
    }


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args, st, families):
    """The oracle as it is, on this host, per update: one sample batch (the
    first batch's first n/2 deletions and n/2 inserts) applied with the
    oracle's batch semantics (incidence maps rebuilt) and the change of every
    tracked family counted by definition (hyperedge / temporal: the triads
    holding a changed hyperedge before and after; incident-vertex: the closed
    forms restricted to the pairs of the changed hyperedges), timed together on
    all host threads.  Beside it, the paper's static mode: a full recount of
    every tracked family on one thread, on the same workload scaled down to a
    few thousand hyperedges (at full size it takes hours to days on one
    thread)."""
    import numpy as np
    from oracle import oracle as orc

    lib = orc.lib()
    threads = int(lib.orc_max_threads())
    ini = st.initial
    temporal = "temporal" in families
    o = orc.OracleGraph(st.n_vertices, ini.offsets, ini.members, ts=ini.ts if temporal else None, window=st.window)
    b = st.batches[0]
    half = max(1, args.cpu_sample // 2)
    dels = b.del_handles[:half]  # the first batch deletes handles of the initial graph (= oracle IDs)
    sub = b.ins.rows(np.arange(min(half, b.ins.n)))
    t0 = time.perf_counter()
    old = o.copy()
    status, ids = o.apply_batch(dels, sub.offsets, sub.members, sub.ts if temporal else None)
    assert status == orc.OK
    what = ["batch applied, maps rebuilt"]
    if "hyperedge" in families or temporal:
        orc.delta_by_definition(old, o, dels, ids, he="hyperedge" in families, temporal=temporal)
        what.append(" and ".join(f for f in ("hyperedge", "temporal") if f in families) + " delta by definition")
    if "incident_vertex" in families:
        orc.iv_delta_by_definition(old, o, dels, ids)
        what.append("incident-vertex delta by definition")
    el = time.perf_counter() - t0
    n = len(dels) + sub.n
    log(args, f"cpu oracle: {n} updates in {el:.2f}s on {threads} threads")
    out = {"value": round(n / el, 2), "unit": "updates/s", "cores": threads, "kind": "oracle",
           "sample": f"{len(dels)} deletions + {sub.n} inserts of the first batch of {st.name}; " + ", ".join(what)
                     + f"; {el:.1f}s", "cpu_model": host_cpu_model()}
    small_scale = {"medium": 0.001, "temporal": 0.0005}.get(st.name)
    small = {"medium": W_medium, "temporal": W_temporal}.get(st.name)
    if small is not None and not args.no_static_baseline:
        s2 = small(small_scale)
        lib.orc_set_threads(1)
        try:
            g = orc.OracleGraph(s2.n_vertices, s2.initial.offsets, s2.initial.members,
                                ts=s2.initial.ts if temporal else None, window=s2.window)
            t0 = time.perf_counter()
            if "hyperedge" in families:
                g.he_counts()
            if "incident_vertex" in families:
                g.iv_counts()
            if temporal:
                g.temporal_counts()
            el1 = time.perf_counter() - t0
        finally:
            lib.orc_set_threads(threads)
        log(args, f"cpu oracle, static recount on one thread at scale {small_scale}: {el1:.2f}s")
        out["static_recount_1thread"] = {"seconds": round(el1, 3), "scale": small_scale, "hyperedges": s2.initial.n,
                                         "families": list(families)}
    return out


WL_TEMPORAL = ("temporal: 500k vertices, 4M hyperedges, card power-law 2.2 on [2,128], Poisson arrivals 1e3/s, "
               "batches of 200k arrivals, expiry 3600 s, temporal triads within 600 s")
LEG_KEYS = ("value", "unit", "steps", "warmup", "ms_per_step", "p50_ms", "p99_ms", "roofline")


def run_legs(args):
    """Further workloads measured after the headline one, each on a fresh graph
    (or set of graphs) with one untimed and two timed steps and one profiled
    step: `temporal` (the temporal configuration at the run's scale) and
    `batched` (the 256-graph rounds: one call per graph, one call for all
    launched kernel by kernel, and one call launched as a captured HIP graph,
    all on the same rounds).  A leg that fails reports its error and never
    takes the headline line down."""
    import argparse
    from paper_2512_21009_amd import workloads as W
    legs = {}
    for name in [s for s in args.legs.split(",") if s]:
        la = argparse.Namespace(**vars(args))
        la.warmup, la.steps, la.prof_steps, la.phases = 1, 2, 1, False
        t0 = time.perf_counter()
        try:
            if name == "temporal":
                st = W.temporal(scale=la.scale, n_batches=la.warmup + la.steps + la.prof_steps)
                r = bench_single(la, st, ("temporal",), "temporal", WL_TEMPORAL)
                leg = {k: r[k] for k in LEG_KEYS}
            elif name == "batched":
                r, _ = bench_batched(la, only=("plain", "stream", "graph"))
                leg = {k: r[k] for k in LEG_KEYS + ("plain", "stream", "graph", "speedup_vs_plain")}
                leg["launch"] = r["config"]["launch"]
            else:
                raise ValueError(f"unknown leg {name!r}")
            leg["workload"] = r["config"]["workload"]
        except Exception as e:  # noqa: BLE001 -- reported in the line
            leg = {"error": f"{type(e).__name__}: {e}"}
        leg["wall_s"] = round(time.perf_counter() - t0, 1)
        log(args, f"leg {name}: {leg.get('value', leg.get('error'))} ({leg['wall_s']} s)")
        legs[name] = leg
    return legs


def W_medium(scale):
    from paper_2512_21009_amd import workloads as W
    return W.medium(q=1.0e4, scale=scale, n_batches=1)


def W_temporal(scale):
    from paper_2512_21009_amd import workloads as W
    return W.temporal(scale=scale, n_batches=1)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1", "n_gpus": args.gpus}),
              flush=True)
        sys.exit(2)
    from paper_2512_21009_amd import hgt, workloads as W

    hgt.load()
    n_b = args.warmup + args.steps + max(1, args.prof_steps)
    t0 = time.perf_counter()
    if args.config == "batched":
        out, sts = bench_batched(args)
        cpu_st, fam = sorted(sts, key=lambda s: s.initial.n)[len(sts) // 2], ("hyperedge",)
    elif args.config == "static":
        out, cpu_st = bench_static(args)
        fam = ("hyperedge", "incident_vertex")
    elif args.config == "sweep":
        out, cpu_st, fam = bench_sweep(args), None, None
    elif args.config == "horizontal":
        out, cpu_st, fam = bench_horizontal(args), None, None
    elif args.config == "served":
        out, sv = bench_served(args)
        busy = sorted((t for t in sv.tenants if t.batches), key=lambda s: s.initial.n)
        cpu_st, fam = busy[len(busy) // 2], W.FAMILIES
    else:
        if args.config == "medium":
            st = W.medium(q=1.0e4, scale=args.scale, n_batches=n_b)
            track = ("hyperedge", "incident_vertex")
            wl = ("medium: 1M vertices, 2M hyperedges, card power-law 2.5 on [2,64], popularity (rank+1e4)^-1.1, "
                  "batches 50k ins + 50k del, hyperedge + incident-vertex triads")
        elif args.config == "literal-store":
            # the literal Zipf(1.1) popularity of Medium (q = 0: one vertex in about a third of
            # the hyperedges), the store alone
            st = W.medium(q=0.0, scale=args.scale, n_batches=n_b)
            track = ()
            wl = ("medium, literal popularity: 1M vertices, 2M hyperedges, card power-law 2.5 on [2,64], "
                  "popularity rank^-1.1, batches 50k ins + 50k del, store only (no triad family)")
        elif args.config == "dyadic":
            st = W.dyadic(n_batches=n_b)
            track = ("incident_vertex",)
            wl = ("dyadic: graph of 1M vertices, 8M distinct edges (popularity (rank+1e3)^-0.8), batches 50k edge "
                  "insertions + 50k deletions, incident-vertex triads (type 3 = triangles)")
        else:
            st = W.temporal(scale=args.scale, n_batches=n_b)
            track = ("temporal",)
            wl = WL_TEMPORAL
        log(args, f"generated {st.initial.n} hyperedges, {n_b} batches in {time.perf_counter() - t0:.1f}s")
        out = bench_single(args, st, track, args.config, wl)
        # no oracle sample on the literal popularity: its by-definition deltas at the hub
        # take the CPU far past the baseline's budget
        cpu_st, fam = (None, None) if args.config.startswith("literal") else (st, track)
    out["cpu_baseline"] = None if (args.no_cpu_baseline or cpu_st is None) else cpu_baseline(args, cpu_st, fam)
    if args.config == "medium" and args.legs != "none":
        out["legs"] = run_legs(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
