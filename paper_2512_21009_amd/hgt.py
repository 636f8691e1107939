"""Python binding of the HIP triad-count library (ctypes over include/hgt.h).

Argument marshalling only: every step of the batch update and of the triad
counting runs in the library's HIP kernels.  PyTorch supplies device memory
(tensor data pointers) and the current HIP stream.  The library must be built
(`python -m paper_2512_21009_amd.build`); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhgt.so")

OK, EINVAL, ENOENT, EDUP, EORDER, ENOMEM, ENOTTRACKED, EDEVICE, EPOISONED = 0, -1, -2, -3, -4, -5, -6, -7, -8
HYPEREDGE, INCIDENT_VERTEX, TEMPORAL = 0, 1, 2
N_CLASSES = {HYPEREDGE: 30, INCIDENT_VERTEX: 3, TEMPORAL: 96}
MAX_CARD = 8192
_NAMES = {"hyperedge": HYPEREDGE, "incident_vertex": INCIDENT_VERTEX, "iv": INCIDENT_VERTEX, "temporal": TEMPORAL}


class HgtError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = _lib.hgt_status_str(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")


class BuildDesc(ctypes.Structure):
    _fields_ = [
        ("n_vertices", ctypes.c_uint32),
        ("n_edges", ctypes.c_uint64),
        ("offsets", ctypes.c_void_p),
        ("members", ctypes.c_void_p),
        ("timestamps", ctypes.c_void_p),
        ("track_mask", ctypes.c_uint32),
        ("temporal_window", ctypes.c_int64),
        ("edge_capacity", ctypes.c_uint64),
        ("pool_words", ctypes.c_uint64),
        ("stream", ctypes.c_void_p),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("n_vertices", ctypes.c_uint32),
        ("track_mask", ctypes.c_uint32),
        ("next_id", ctypes.c_uint64),
        ("n_live", ctypes.c_uint64),
        ("n_incidences", ctypes.c_uint64),
        ("edge_capacity", ctypes.c_uint64),
        ("h2v_pool_words", ctypes.c_uint64),
        ("h2v_used_words", ctypes.c_uint64),
        ("v2h_pool_words", ctypes.c_uint64),
        ("v2h_used_words", ctypes.c_uint64),
        ("temporal_window", ctypes.c_int64),
        ("batches", ctypes.c_uint64),
        ("compactions", ctypes.c_uint64),
        ("graph_launches", ctypes.c_uint64),
    ]


class KernelTime(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 24),
        ("launches", ctypes.c_uint64),
        ("total_ms", ctypes.c_double),
        ("algo_bytes", ctypes.c_uint64),
        ("events", ctypes.c_uint64),
        ("aux", ctypes.c_uint64),
    ]


class Batch(ctypes.Structure):
    _fields_ = [
        ("graph", ctypes.c_void_p),
        ("del_ids", ctypes.c_void_p),
        ("n_del", ctypes.c_uint64),
        ("ins_offsets", ctypes.c_void_p),
        ("ins_members", ctypes.c_void_p),
        ("n_ins_members", ctypes.c_uint64),
        ("ins_ts", ctypes.c_void_p),
        ("n_ins", ctypes.c_uint64),
        ("out_ins_ids", ctypes.c_void_p),
        ("status", ctypes.c_int32),
        ("pad0", ctypes.c_int32),
    ]


class ServerDesc(ctypes.Structure):
    _fields_ = [
        ("hbm_budget_bytes", ctypes.c_uint64),
        ("arena_bytes", ctypes.c_uint64),
        ("max_round", ctypes.c_uint32),
        ("max_inflight", ctypes.c_uint32),
        ("launch_flags", ctypes.c_uint32),
        ("pad0", ctypes.c_uint32),
    ]


class Request(ctypes.Structure):
    _fields_ = [
        ("del_ids", ctypes.c_void_p),
        ("n_del", ctypes.c_uint64),
        ("ins_offsets", ctypes.c_void_p),
        ("ins_members", ctypes.c_void_p),
        ("n_ins_members", ctypes.c_uint64),
        ("ins_ts", ctypes.c_void_p),
        ("n_ins", ctypes.c_uint64),
        ("out_ins_ids_host", ctypes.c_void_p),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("tenant", ctypes.c_uint32),
        ("he", ctypes.c_uint64 * 30),
        ("iv", ctypes.c_uint64 * 3),
        ("temporal", ctypes.c_uint64 * 96),
        ("t_submit_ns", ctypes.c_uint64),
        ("t_admit_ns", ctypes.c_uint64),
        ("t_done_ns", ctypes.c_uint64),
        ("round", ctypes.c_uint64),
        ("round_size", ctypes.c_uint32),
        ("pad0", ctypes.c_uint32),
    ]


class ServerInfo(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in ("rounds", "requests_done", "requests_pending", "requests_running",
                                               "footprint_in_use", "arena_in_use", "max_round_size",
                                               "max_inflight_seen")]


_lib = None

EXPORTS = ["hgt_build", "hgt_apply_batch", "hgt_apply_batch_noalloc", "hgt_apply_batches", "hgt_apply_batches_ex",
           "hgt_tune_flush", "hgt_apply_vertex_ops", "hgt_compact", "hgt_triad_counts", "hgt_sync", "hgt_destroy", "hgt_status_str",
           "hgt_get_info", "hgt_export_h2v", "hgt_export_v2h", "hgt_class_codes", "hgt_profile",
           "hgt_profile_read", "hgt_profile_counters", "hgt_server_create", "hgt_server_add_tenant", "hgt_server_tenant_graph",
           "hgt_server_submit", "hgt_server_wait", "hgt_server_query", "hgt_server_get_info", "hgt_server_destroy",
           "hgt_snapshot", "hgt_restore", "hgt_snap_bytes", "hgt_snap_load", "hgt_snap_free"]


def load(path: str = LIB_PATH):
    """Load libhgt.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2512_21009_amd.build`")
    # torch first: the library then binds to the HIP runtime torch has loaded,
    # so torch's streams and allocations belong to the runtime it calls
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P, U64, U32, I64, I32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64, ctypes.c_int
    lib.hgt_build.argtypes = [ctypes.POINTER(BuildDesc), ctypes.POINTER(P)]
    lib.hgt_apply_batch.argtypes = [P, P, U64, P, P, U64, P, U64, P, P]
    lib.hgt_apply_batch_noalloc.argtypes = [P, P, U64, P, P, U64, P, U64, P, P]
    lib.hgt_apply_batches.argtypes = [P, U32, P]
    lib.hgt_apply_batches_ex.argtypes = [P, U32, P, U32]
    lib.hgt_tune_flush.argtypes = [ctypes.POINTER(U32)]
    lib.hgt_apply_vertex_ops.argtypes = [P, P, P, P, U64, P]
    lib.hgt_compact.argtypes = [P, P]
    lib.hgt_triad_counts.argtypes = [P, I32, I64, P, U32]
    lib.hgt_sync.argtypes = [P, ctypes.POINTER(I32)]
    lib.hgt_destroy.argtypes = [P]
    lib.hgt_status_str.argtypes = [I32]
    lib.hgt_status_str.restype = ctypes.c_char_p
    lib.hgt_get_info.argtypes = [P, ctypes.POINTER(Info)]
    lib.hgt_export_h2v.argtypes = [P, P, P, P]
    lib.hgt_export_v2h.argtypes = [P, P, P]
    lib.hgt_class_codes.argtypes = [I32, P, U32]
    lib.hgt_profile.argtypes = [P, I32]
    lib.hgt_profile_read.argtypes = [P, P, U32, ctypes.POINTER(U32)]
    lib.hgt_profile_counters.argtypes = [P, P, U32, ctypes.POINTER(U32)]
    lib.hgt_server_create.argtypes = [ctypes.POINTER(ServerDesc), ctypes.POINTER(P)]
    lib.hgt_server_add_tenant.argtypes = [P, ctypes.POINTER(BuildDesc), ctypes.POINTER(U32)]
    lib.hgt_server_tenant_graph.argtypes = [P, U32, ctypes.POINTER(P)]
    lib.hgt_server_submit.argtypes = [P, U32, ctypes.POINTER(Request), ctypes.POINTER(U64)]
    lib.hgt_server_wait.argtypes = [P, U64, ctypes.POINTER(Result)]
    lib.hgt_server_query.argtypes = [P, U64, ctypes.POINTER(I32)]
    lib.hgt_server_get_info.argtypes = [P, ctypes.POINTER(ServerInfo)]
    lib.hgt_server_destroy.argtypes = [P]
    lib.hgt_snapshot.argtypes = [P, ctypes.POINTER(P), P]
    lib.hgt_restore.argtypes = [P, P, P]
    lib.hgt_snap_bytes.argtypes = [P, P, U64, ctypes.POINTER(U64)]
    lib.hgt_snap_load.argtypes = [P, U64, ctypes.POINTER(P)]
    lib.hgt_snap_free.argtypes = [P]
    for name in EXPORTS:
        getattr(lib, name).restype = getattr(lib, name).restype or ctypes.c_int
    lib.hgt_status_str.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _stream(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr() if t.numel() else None


def _check_dtype(t, allowed, name):
    if t is not None and t.dtype not in allowed:
        raise TypeError(f"{name}: dtype {t.dtype} not in {allowed}")


def _mask(track: Sequence) -> int:
    m = 0
    for t in track:
        m |= 1 << (_NAMES[t] if isinstance(t, str) else int(t))
    return m


def class_codes(kind) -> List[int]:
    lib = load()
    k = _NAMES[kind] if isinstance(kind, str) else int(kind)
    n = lib.hgt_class_codes(k, None, 0)
    if n < 0:
        raise HgtError(n, "class_codes")
    arr = (ctypes.c_int32 * n)()
    lib.hgt_class_codes(k, ctypes.cast(arr, ctypes.c_void_p), n)
    return list(arr)


def _batch_args(del_ids, ins_offsets, ins_members, ins_ts):
    import torch
    _check_dtype(del_ids, (torch.int32, torch.uint32), "del_ids")
    _check_dtype(ins_offsets, (torch.int64, torch.uint64), "ins_offsets")
    _check_dtype(ins_members, (torch.int32, torch.uint32), "ins_members")
    _check_dtype(ins_ts, (torch.int64,), "ins_ts")
    n_del = 0 if del_ids is None else int(del_ids.numel())
    n_ins = 0 if ins_offsets is None else int(ins_offsets.numel() - 1)
    n_mem = 0 if ins_members is None else int(ins_members.numel())
    return n_del, n_ins, n_mem


BATCHES_GRAPH = 1
BATCHES_AUTOTUNE = 2


def apply_batches(items, stream=None, raise_on_error: bool = True, graph: bool = False, autotune: bool = False):
    """Batched form: items = [(graph, del_ids, ins_offsets, ins_members, ins_ts), ...]
    with distinct graphs.  Applies all of them in one call (one wait, shared
    triad launches).  graph=True launches the round as one captured HIP graph;
    autotune=True lets the library's autotuner pick the launch choices.
    Returns the list of assigned-ID tensors (or, with raise_on_error=False,
    (first_status, [status...], [ids...]))."""
    import torch
    lib = load()
    n = len(items)
    arr = (Batch * max(n, 1))()
    outs = []
    for i, it in enumerate(items):
        g, del_ids, ins_offsets, ins_members, ins_ts = (list(it) + [None] * 5)[:5]
        n_del, n_ins, n_mem = _batch_args(del_ids, ins_offsets, ins_members, ins_ts)
        out = torch.empty(n_ins, dtype=torch.int32, device=ins_offsets.device) if n_ins else None
        outs.append(out)
        b = arr[i]
        b.graph = g._h.value
        b.del_ids = _ptr(del_ids)
        b.n_del = n_del
        b.ins_offsets = _ptr(ins_offsets) if n_ins else None
        b.ins_members = _ptr(ins_members)
        b.n_ins_members = n_mem
        b.ins_ts = _ptr(ins_ts)
        b.n_ins = n_ins
        b.out_ins_ids = _ptr(out) if n_ins else None
    flags = (BATCHES_GRAPH if graph else 0) | (BATCHES_AUTOTUNE if autotune else 0)
    rc = lib.hgt_apply_batches_ex(ctypes.cast(arr, ctypes.c_void_p), n, _stream(stream), flags)
    status = [arr[i].status for i in range(n)]
    if raise_on_error:
        if rc != OK:
            raise HgtError(rc, f"hgt_apply_batches (statuses {status})")
        return outs
    return rc, status, outs


def tune_flush() -> int:
    """Waits for the autotuner's timed rounds; returns how many round keys have
    a kept launch choice."""
    lib = load()
    k = ctypes.c_uint32(0)
    rc = lib.hgt_tune_flush(ctypes.byref(k))
    if rc != OK:
        raise HgtError(rc, "hgt_tune_flush")
    return int(k.value)


def _build_desc(n_vertices, offsets, members, timestamps, track, window, edge_capacity, pool_words):
    import torch
    _check_dtype(offsets, (torch.int64, torch.uint64), "offsets")
    _check_dtype(members, (torch.int32, torch.uint32), "members")
    _check_dtype(timestamps, (torch.int64,), "timestamps")
    d = BuildDesc()
    d.n_vertices = int(n_vertices)
    d.n_edges = int(offsets.numel() - 1)
    d.offsets = _ptr(offsets)
    d.members = _ptr(members)
    d.timestamps = _ptr(timestamps)
    d.track_mask = _mask(track)
    d.temporal_window = int(window)
    d.edge_capacity = int(edge_capacity)
    d.pool_words = int(pool_words)
    return d


class Graph:
    """A hypergraph resident on the current GPU with incrementally maintained
    triad counts (hyperedge 30 classes, incident-vertex 3 types, temporal 96)."""

    def __init__(self, handle: int, window: int, track_mask: int):
        self._h = ctypes.c_void_p(handle)
        self.window = window
        self.track_mask = track_mask

    # ------------------------------------------------------------------ build
    @classmethod
    def build(cls, n_vertices: int, offsets, members, timestamps=None, track=("hyperedge",), window: int = 0,
              edge_capacity: int = 0, pool_words: int = 0, stream=None) -> "Graph":
        """offsets: int64 device tensor [E+1]; members: int32/uint32 device
        tensor; timestamps: int64 device tensor [E] (temporal)."""
        lib = load()
        d = _build_desc(n_vertices, offsets, members, timestamps, track, window, edge_capacity, pool_words)
        d.stream = _stream(stream)
        out = ctypes.c_void_p()
        rc = lib.hgt_build(ctypes.byref(d), ctypes.byref(out))
        if rc != OK:
            raise HgtError(rc, "hgt_build")
        return cls(out.value, int(window), d.track_mask)

    # ------------------------------------------------------------------ update
    def apply_batch(self, del_ids=None, ins_offsets=None, ins_members=None, ins_ts=None, out_ids=None,
                    stream=None, raise_on_error: bool = True, noalloc: bool = False):
        """Delete del_ids (int32 device tensor), then insert the CSR batch.
        Returns the int32 device tensor of assigned IDs (or (status, ids)
        with raise_on_error=False).  noalloc=True calls
        hgt_apply_batch_noalloc (out_ids, when given, keeps the call free of
        allocations on the Python side too)."""
        import torch
        lib = load()
        n_del = 0 if del_ids is None else int(del_ids.numel())
        n_ins = 0 if ins_offsets is None else int(ins_offsets.numel() - 1)
        _check_dtype(del_ids, (torch.int32, torch.uint32), "del_ids")
        _check_dtype(ins_offsets, (torch.int64, torch.uint64), "ins_offsets")
        _check_dtype(ins_members, (torch.int32, torch.uint32), "ins_members")
        _check_dtype(ins_ts, (torch.int64,), "ins_ts")
        n_mem = 0 if ins_members is None else int(ins_members.numel())
        if out_ids is None and n_ins:
            dev = ins_offsets.device
            out_ids = torch.empty(n_ins, dtype=torch.int32, device=dev)
        fn = lib.hgt_apply_batch_noalloc if noalloc else lib.hgt_apply_batch
        rc = fn(self._h, _ptr(del_ids), n_del, _ptr(ins_offsets) if n_ins else None,
                _ptr(ins_members), n_mem, _ptr(ins_ts), n_ins,
                _ptr(out_ids) if n_ins else None, _stream(stream))
        if raise_on_error:
            if rc != OK:
                raise HgtError(rc, "hgt_apply_batch_noalloc" if noalloc else "hgt_apply_batch")
            return out_ids
        return rc, out_ids

    def apply_vertex_ops(self, edge_ids, vertices, insert, stream=None, raise_on_error: bool = True):
        """Horizontal operations: insert (insert[i] true) or delete vertices[i]
        in hyperedge edge_ids[i] (int32 / int32 / uint8 or bool device tensors).
        Returns the status (raises on error unless raise_on_error=False)."""
        import torch
        n = int(edge_ids.numel())
        _check_dtype(edge_ids, (torch.int32, torch.uint32), "edge_ids")
        _check_dtype(vertices, (torch.int32, torch.uint32), "vertices")
        _check_dtype(insert, (torch.uint8, torch.bool), "insert")
        if int(vertices.numel()) != n or int(insert.numel()) != n:
            raise ValueError("edge_ids, vertices and insert must have the same length")
        rc = load().hgt_apply_vertex_ops(self._h, _ptr(edge_ids), _ptr(vertices), _ptr(insert), n, _stream(stream))
        if rc != OK and raise_on_error:
            raise HgtError(rc, "hgt_apply_vertex_ops")
        return rc

    # ------------------------------------------------------------------ queries
    def triad_counts(self, kind, window: Optional[int] = None) -> List[int]:
        lib = load()
        k = _NAMES[kind] if isinstance(kind, str) else int(kind)
        n = N_CLASSES[k]
        arr = (ctypes.c_uint64 * n)()
        w = (self.window if window is None else int(window)) if k == TEMPORAL else 0
        rc = lib.hgt_triad_counts(self._h, k, w, ctypes.cast(arr, ctypes.c_void_p), n)
        if rc != OK:
            raise HgtError(rc, "hgt_triad_counts")
        return list(arr)

    def sync(self) -> int:
        st = ctypes.c_int(0)
        rc = load().hgt_sync(self._h, ctypes.byref(st))
        if rc != OK:
            raise HgtError(rc, "hgt_sync")
        return st.value

    def info(self) -> dict:
        inf = Info()
        rc = load().hgt_get_info(self._h, ctypes.byref(inf))
        if rc != OK:
            raise HgtError(rc, "hgt_get_info")
        return {f: getattr(inf, f) for f, _ in Info._fields_}

    def compact(self, stream=None):
        """Move every live incidence list into fresh pools (see hgt_compact)."""
        rc = load().hgt_compact(self._h, _stream(stream))
        if rc != OK:
            raise HgtError(rc, "hgt_compact")

    def profile(self, enable=True):
        """Reset the per-kernel-group profile and set its level: 0/False off,
        1/True HIP events + byte counters, 2 also the phase timers."""
        level = int(enable) if not isinstance(enable, bool) else (1 if enable else 0)
        rc = load().hgt_profile(self._h, level)
        if rc != OK:
            raise HgtError(rc, "hgt_profile")

    def profile_read(self) -> dict:
        """{group: {launches, total_ms, algo_bytes, events, aux}}"""
        n = ctypes.c_uint32(0)
        rows = (KernelTime * 16)()
        rc = load().hgt_profile_read(self._h, ctypes.cast(rows, ctypes.c_void_p), 16, ctypes.byref(n))
        if rc != OK:
            raise HgtError(rc, "hgt_profile_read")
        out = {}
        for r in rows[: n.value]:
            out[r.name.decode()] = dict(launches=r.launches, total_ms=r.total_ms, algo_bytes=r.algo_bytes,
                                        events=r.events, aux=r.aux)
        return out

    def profile_counters(self):
        """Raw profile counters (see hgt_profile_counters)."""
        import numpy as np
        out = np.zeros(64, np.uint64)
        n = ctypes.c_uint32(0)
        rc = load().hgt_profile_counters(self._h, out.ctypes.data, 64, ctypes.byref(n))
        if rc != OK:
            raise HgtError(rc, "hgt_profile_counters")
        return out[: min(n.value, 64)]

    def export_h2v(self):
        """(offsets, members, live) numpy arrays indexed by ID."""
        import numpy as np
        inf = self.info()
        n = inf["next_id"]
        off = np.zeros(n + 1, np.uint64)
        mem = np.zeros(max(inf["n_incidences"], 1), np.uint32)
        live = np.zeros(max(n, 1), np.uint8)
        rc = load().hgt_export_h2v(self._h, off.ctypes.data, mem.ctypes.data, live.ctypes.data)
        if rc != OK:
            raise HgtError(rc, "hgt_export_h2v")
        return off, mem[: int(off[-1])], live[:n]

    def export_v2h(self):
        import numpy as np
        inf = self.info()
        off = np.zeros(inf["n_vertices"] + 1, np.uint64)
        mem = np.zeros(max(inf["n_incidences"], 1), np.uint32)
        rc = load().hgt_export_v2h(self._h, off.ctypes.data, mem.ctypes.data)
        if rc != OK:
            raise HgtError(rc, "hgt_export_v2h")
        return off, mem[: int(off[-1])]

    # ------------------------------------------------------------------ snapshots
    def snapshot(self, stream=None) -> "Snapshot":
        """Host copy of the graph's whole state (see hgt_snapshot)."""
        out = ctypes.c_void_p()
        rc = load().hgt_snapshot(self._h, ctypes.byref(out), _stream(stream))
        if rc != OK:
            raise HgtError(rc, "hgt_snapshot")
        return Snapshot(out.value)

    def restore(self, snap: "Snapshot", stream=None):
        """Replace the graph's state by the snapshot's (also clears a poisoned graph)."""
        rc = load().hgt_restore(self._h, snap._h, _stream(stream))
        if rc != OK:
            raise HgtError(rc, "hgt_restore")

    def close(self):
        if self._h and self._h.value:
            load().hgt_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Snapshot:
    """A graph snapshot held by the library in host memory; to_bytes() gives
    its documented byte form and from_bytes() loads (and checks) one."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)

    def to_bytes(self) -> bytes:
        lib = load()
        n = ctypes.c_uint64(0)
        rc = lib.hgt_snap_bytes(self._h, None, 0, ctypes.byref(n))
        if rc != OK:
            raise HgtError(rc, "hgt_snap_bytes")
        buf = ctypes.create_string_buffer(n.value)
        rc = lib.hgt_snap_bytes(self._h, ctypes.cast(buf, ctypes.c_void_p), n.value, ctypes.byref(n))
        if rc != OK:
            raise HgtError(rc, "hgt_snap_bytes")
        return buf.raw

    @classmethod
    def from_bytes(cls, data: bytes) -> "Snapshot":
        lib = load()
        out = ctypes.c_void_p()
        buf = ctypes.create_string_buffer(bytes(data), len(data))
        rc = lib.hgt_snap_load(ctypes.cast(buf, ctypes.c_void_p), len(data), ctypes.byref(out))
        if rc != OK:
            raise HgtError(rc, "hgt_snap_load")
        return cls(out.value)

    def save(self, path: str):
        """Write the byte form to a file (a checkpoint another process can restore)."""
        with open(path, "wb") as f:
            f.write(self.to_bytes())

    @classmethod
    def load_file(cls, path: str) -> "Snapshot":
        with open(path, "rb") as f:
            return cls.from_bytes(f.read())

    def close(self):
        if self._h and self._h.value:
            load().hgt_snap_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """The served form: resident tenants, requests submitted from host arrays
    (copied at submit), applied in continuous-batching rounds by the
    library's server thread."""

    def __init__(self, hbm_budget_bytes: int = 8 << 30, arena_bytes: int = 0, max_round: int = 0,
                 max_inflight: int = 0, graph: bool = False, autotune: bool = False):
        lib = load()
        flags = (BATCHES_GRAPH if graph else 0) | (BATCHES_AUTOTUNE if autotune else 0)
        d = ServerDesc(int(hbm_budget_bytes), int(arena_bytes), int(max_round), int(max_inflight), flags, 0)
        out = ctypes.c_void_p()
        rc = lib.hgt_server_create(ctypes.byref(d), ctypes.byref(out))
        if rc != OK:
            raise HgtError(rc, "hgt_server_create")
        self._h = out
        self._ids = {}      # ticket -> (numpy out-ID buffer, keep-alive inputs)
        self._track = {}

    def add_tenant(self, n_vertices: int, offsets, members, timestamps=None, track=("hyperedge",), window: int = 0,
                   edge_capacity: int = 0, pool_words: int = 0) -> int:
        d = _build_desc(n_vertices, offsets, members, timestamps, track, window, edge_capacity, pool_words)
        t = ctypes.c_uint32()
        rc = load().hgt_server_add_tenant(self._h, ctypes.byref(d), ctypes.byref(t))
        if rc != OK:
            raise HgtError(rc, "hgt_server_add_tenant")
        self._track[t.value] = (d.track_mask, int(window))
        return t.value

    def tenant_graph(self, tenant: int) -> "Graph":
        """A non-owning Graph view of the tenant (for queries while it is idle)."""
        out = ctypes.c_void_p()
        rc = load().hgt_server_tenant_graph(self._h, int(tenant), ctypes.byref(out))
        if rc != OK:
            raise HgtError(rc, "hgt_server_tenant_graph")
        g = Graph(out.value, self._track[tenant][1], self._track[tenant][0])
        g.close = lambda: None  # the server owns it
        return g

    def submit(self, tenant: int, del_ids=None, ins_offsets=None, ins_members=None, ins_ts=None) -> int:
        """Host numpy arrays (del_ids u32, ins_offsets u64 [n+1], ins_members u32,
        ins_ts i64).  Returns the ticket."""
        import numpy as np
        r = Request()
        keep = []

        def arr(a, dt):
            if a is None:
                return None, 0
            a = np.ascontiguousarray(np.asarray(a).astype(dt, copy=False))
            keep.append(a)
            return (a.ctypes.data if a.size else None), a.size
        r.del_ids, r.n_del = arr(del_ids, np.uint32)
        off, n_off = arr(ins_offsets, np.uint64)
        r.n_ins = max(n_off - 1, 0)
        r.ins_offsets = off if r.n_ins else None
        r.ins_members, r.n_ins_members = arr(ins_members, np.uint32)
        r.ins_ts, _ = arr(ins_ts, np.int64)
        ids = np.zeros(max(r.n_ins, 1), np.uint32)
        r.out_ins_ids_host = ids.ctypes.data if r.n_ins else None
        t = ctypes.c_uint64()
        rc = load().hgt_server_submit(self._h, int(tenant), ctypes.byref(r), ctypes.byref(t))
        if rc != OK:
            raise HgtError(rc, "hgt_server_submit")
        self._ids[t.value] = (ids[: r.n_ins], keep)
        return t.value

    def wait(self, ticket: int) -> dict:
        res = Result()
        rc = load().hgt_server_wait(self._h, int(ticket), ctypes.byref(res))
        ids, _ = self._ids.pop(ticket, (None, None))
        if rc == EINVAL and res.t_submit_ns == 0:
            raise HgtError(rc, "hgt_server_wait")
        return {"status": res.status, "tenant": res.tenant, "hyperedge": list(res.he),
                "incident_vertex": list(res.iv), "temporal": list(res.temporal), "ids": ids,
                "t_submit_ns": res.t_submit_ns, "t_admit_ns": res.t_admit_ns, "t_done_ns": res.t_done_ns,
                "round": res.round, "round_size": res.round_size}

    def query(self, ticket: int) -> bool:
        d = ctypes.c_int(0)
        rc = load().hgt_server_query(self._h, int(ticket), ctypes.byref(d))
        if rc != OK:
            raise HgtError(rc, "hgt_server_query")
        return bool(d.value)

    def info(self) -> dict:
        inf = ServerInfo()
        rc = load().hgt_server_get_info(self._h, ctypes.byref(inf))
        if rc != OK:
            raise HgtError(rc, "hgt_server_get_info")
        return {f: getattr(inf, f) for f, _ in ServerInfo._fields_}

    def close(self):
        if self._h and self._h.value:
            load().hgt_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
