"""Plain CPU oracle for dynamic-hypergraph triad counts.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the GPU library or its binding.

The oracle keeps the live hyperedge set in numpy arrays indexed by ID, applies
a batch by the paper's semantics and, after every batch, rebuilds the incidence
maps from scratch and recounts by full enumeration (C code in hgt_oracle.c).
A second mode counts a batch's delta by definition: the triads of the new
graph that contain an inserted hyperedge minus the triads of the old graph that
contain a deleted one.

Batch semantics (paper Sec. III-B, Alg. 1 and 2, Alg. 3 step 3):
 * deletions are applied first, then insertions;
 * deleted IDs must be live and distinct; a rejected batch changes nothing;
 * inserted member lists are sets: sorted, at least one vertex, vertex ids
   below n_vertices, no repeats;
 * ID reuse: with F the ascending list of free IDs (IDs freed earlier and this
   batch's deletions), the j-th insert (0-based, batch order) gets F[j]; inserts
   beyond |F| get fresh consecutive IDs starting at the next unused ID.  This is
   the "j-th available node" rule of Alg. 2 (thread j finds the j-th available
   block) with blocks identified by their hyperedge ID; the first initial
   hyperedge gets ID 0;
 * temporal graphs: every inserted timestamp is at least the largest timestamp
   inserted before, and timestamps within a batch are non-decreasing; equal
   timestamps are ordered by arrival sequence.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hgt_oracle.c")
_LIB = os.path.join(_HERE, "libhgt_oracle.so")

N_HE = 30
N_TMP = 96
N_IV = 3

OK, EINVAL, ENOENT, EDUP, EORDER = "ok", "einval", "enoent", "edup", "eorder"


def build_library(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, -O2, OpenMP over centres, no GPU code)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build_library())
        P = ctypes.c_void_p
        U64, U32, I64 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64
        _lib.orc_count_full.argtypes = [U64, P, P, P, U32, P, P, I64, P, P]
        _lib.orc_count_full.restype = ctypes.c_int
        _lib.orc_count_containing.argtypes = [U64, P, P, P, U32, P, P, I64, P, P, P]
        _lib.orc_count_containing.restype = ctypes.c_int
        _lib.orc_count_iv.argtypes = [U64, P, P, P, U32, P]
        _lib.orc_count_iv.restype = ctypes.c_int
        _lib.orc_iv_partial.argtypes = [U64, P, P, P, U32, P, U64, P]
        _lib.orc_iv_partial.restype = ctypes.c_int
        _lib.orc_pairs_of.argtypes = [P, P, P, U64, P]
        _lib.orc_pairs_of.restype = U64
        _lib.orc_set_threads.argtypes = [ctypes.c_int]
        _lib.orc_he_class_of_code.argtypes = [ctypes.c_int]
        _lib.orc_tmp_class_of_code.argtypes = [ctypes.c_int]
        _lib.orc_he_class_codes.argtypes = [P]
        _lib.orc_tmp_class_codes.argtypes = [P]
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def he_class_codes() -> np.ndarray:
    n = lib().orc_n_he_classes()
    out = np.zeros(n, dtype=np.int32)
    lib().orc_he_class_codes(_p(out))
    return out


def tmp_class_codes() -> np.ndarray:
    n = lib().orc_n_tmp_classes()
    out = np.zeros(n, dtype=np.int32)
    lib().orc_tmp_class_codes(_p(out))
    return out


def he_class_of_code(code: int) -> int:
    return lib().orc_he_class_of_code(int(code))


def tmp_class_of_code(code: int) -> int:
    return lib().orc_tmp_class_of_code(int(code))


def canonical_rows(offsets: np.ndarray, members: np.ndarray):
    """Sort each row; return (offsets u64, members u32, ok) where ok is False
    when a row is empty or repeats a vertex."""
    offsets = np.asarray(offsets, dtype=np.uint64)
    members = np.asarray(members, dtype=np.uint32)
    n = len(offsets) - 1
    lens = np.diff(offsets.astype(np.int64))
    if n == 0:
        return offsets, members, True
    if (lens < 1).any():
        return offsets, members, False
    row = np.repeat(np.arange(n, dtype=np.int64), lens)
    order = np.lexsort((members, row))
    m = members[order]
    same_row = row[1:] == row[:-1]
    dup = (m[1:] == m[:-1]) & same_row
    return offsets, m, not bool(dup.any())


class OracleGraph:
    """Live hyperedge set with the batch semantics above."""

    def __init__(self, n_vertices: int, offsets, members, ts=None, window: int = 0):
        offsets, members, ok = canonical_rows(offsets, members)
        if not ok or (len(members) and int(members.max()) >= n_vertices):
            raise ValueError("invalid initial hypergraph")
        n = len(offsets) - 1
        self.n_vertices = int(n_vertices)
        self.temporal = ts is not None
        self.window = int(window)
        self.off = offsets.astype(np.uint64)
        self.mem = members.astype(np.uint32)
        self.live = np.ones(n, dtype=np.uint8)
        self.ts = np.asarray(ts, dtype=np.int64).copy() if ts is not None else np.zeros(n, np.int64)
        self.seq = np.arange(n, dtype=np.uint64)
        self.next_id = n
        self.next_seq = n
        self.last_ts = int(self.ts.max()) if (self.temporal and n) else np.iinfo(np.int64).min

    # ------------------------------------------------------------------ #
    @property
    def n_slots(self) -> int:
        return len(self.live)

    def lens(self) -> np.ndarray:
        return np.diff(self.off.astype(np.int64))

    def row(self, i: int) -> np.ndarray:
        return self.mem[int(self.off[i]):int(self.off[i + 1])]

    def live_ids(self) -> np.ndarray:
        return np.nonzero(self.live)[0].astype(np.uint32)

    def free_ids(self) -> np.ndarray:
        return np.nonzero(self.live[: self.next_id] == 0)[0].astype(np.int64)

    def copy(self) -> "OracleGraph":
        g = OracleGraph.__new__(OracleGraph)
        g.__dict__.update({k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in self.__dict__.items()})
        return g

    # ------------------------------------------------------------------ #
    def apply_batch(self, del_ids, ins_offsets, ins_members, ins_ts=None):
        """Returns (status, assigned_ids).  On error the state is unchanged."""
        del_ids = np.asarray(del_ids, dtype=np.int64)
        ins_offsets = np.asarray(ins_offsets, dtype=np.uint64)
        ins_members = np.asarray(ins_members, dtype=np.uint32)
        n_ins = len(ins_offsets) - 1
        # --- deletions ---
        if len(del_ids):
            if (del_ids < 0).any() or (del_ids >= self.next_id).any():
                return ENOENT, None
            if not self.live[del_ids].all():
                return ENOENT, None
            if len(np.unique(del_ids)) != len(del_ids):
                return EDUP, None
        # --- insertions ---
        io, im, ok = canonical_rows(ins_offsets, ins_members)
        if not ok or (len(im) and int(im.max()) >= self.n_vertices):
            return EINVAL, None
        if self.temporal and n_ins:
            if ins_ts is None:
                return EINVAL, None
            t = np.asarray(ins_ts, dtype=np.int64)
            if (n_ins > 1 and (np.diff(t) < 0).any()) or int(t[0]) < self.last_ts:
                return EORDER, None
        # --- ID assignment: j-th insert takes the j-th smallest free ID ---
        F = np.union1d(self.free_ids(), del_ids)
        k = min(n_ins, len(F))
        assigned = np.concatenate([F[:k], np.arange(self.next_id, self.next_id + (n_ins - k))]).astype(np.int64)
        new_next = self.next_id + (n_ins - k)
        # --- rebuild state ---
        cap = max(new_next, self.n_slots)
        lens = np.zeros(cap, dtype=np.int64)
        lens[: self.n_slots] = self.lens()
        live = np.zeros(cap, dtype=np.uint8)
        live[: self.n_slots] = self.live
        lens[del_ids] = 0
        live[del_ids] = 0
        ins_lens = np.diff(io.astype(np.int64))
        lens[assigned] = ins_lens
        live[assigned] = 1
        src_old = np.zeros(cap, dtype=bool)
        src_old[: self.n_slots] = live[: self.n_slots].astype(bool)
        src_old[assigned] = False
        off = np.zeros(cap + 1, dtype=np.uint64)
        np.cumsum(lens, out=off[1:])
        mem = np.zeros(int(off[-1]), dtype=np.uint32)
        old_ids = np.nonzero(src_old)[0]
        for ids, s_off, s_mem in ((old_ids, self.off, self.mem), (assigned, io, im)):
            if len(ids) == 0:
                continue
            src_rows = ids if s_off is self.off else np.arange(len(ids))
            ln = (s_off[src_rows + 1] - s_off[src_rows]).astype(np.int64)
            if ln.sum() == 0:
                continue
            dst_start = np.repeat(off[ids].astype(np.int64), ln)
            src_start = np.repeat(s_off[src_rows].astype(np.int64), ln)
            within = np.arange(int(ln.sum()), dtype=np.int64) - np.repeat(np.cumsum(ln) - ln, ln)
            mem[dst_start + within] = s_mem[src_start + within]
        ts = np.zeros(cap, dtype=np.int64)
        ts[: self.n_slots] = self.ts
        seq = np.zeros(cap, dtype=np.uint64)
        seq[: self.n_slots] = self.seq
        if n_ins:
            if self.temporal:
                ts[assigned] = np.asarray(ins_ts, dtype=np.int64)
                self.last_ts = max(self.last_ts, int(np.max(ins_ts)))
            seq[assigned] = self.next_seq + np.arange(n_ins, dtype=np.uint64)
            self.next_seq += n_ins
        self.off, self.mem, self.live, self.ts, self.seq = off, mem, live, ts, seq
        self.next_id = int(new_next)
        return OK, assigned.astype(np.uint32)

    # ------------------------------------------------------------------ #
    def apply_vertex_ops(self, edge_ids, vertices, insert):
        """Incident-vertex insertions and deletions inside live hyperedges (the
        paper's horizontal operations, Sec. III-B): op i inserts vertices[i]
        into hyperedge edge_ids[i] (insert[i] true) or deletes it from it.
        Every modified hyperedge keeps its ID, timestamp and arrival sequence.
        Rejected (state unchanged) when an ID is not live (ENOENT), a vertex is
        out of range, the same (hyperedge, vertex) appears twice, a deleted
        vertex is not a member, an inserted one already is, or a hyperedge
        would be left empty (EINVAL).  Returns (status, ascending modified IDs)."""
        edge_ids = np.asarray(edge_ids, dtype=np.int64)
        vertices = np.asarray(vertices, dtype=np.int64)
        insert = np.asarray(insert, dtype=bool)
        if len(edge_ids) == 0:
            return OK, np.zeros(0, np.int64)
        if (edge_ids < 0).any() or (edge_ids >= self.next_id).any() or not self.live[edge_ids].all():
            return ENOENT, None
        if (vertices < 0).any() or (vertices >= self.n_vertices).any():
            return EINVAL, None
        pairs = edge_ids * self.n_vertices + vertices
        if len(np.unique(pairs)) != len(pairs):
            return EINVAL, None
        new_rows = {}
        for h in np.unique(edge_ids).tolist():
            row = set(self.row(h).tolist())
            sel = edge_ids == h
            for v, ins in zip(vertices[sel].tolist(), insert[sel].tolist()):
                if ins:
                    if v in row:
                        return EINVAL, None
                    row.add(v)
                else:
                    if v not in row:
                        return EINVAL, None
                    row.remove(v)
            if not row:
                return EINVAL, None
            new_rows[h] = np.array(sorted(row), dtype=np.uint32)
        old_lens = self.lens()
        lens = old_lens.copy()
        for h, r in new_rows.items():
            lens[h] = len(r)
        off = np.zeros(self.n_slots + 1, dtype=np.uint64)
        np.cumsum(lens, out=off[1:])
        mem = np.zeros(int(off[-1]), dtype=np.uint32)
        # unmodified rows move as they are, then the new rows are written
        keep = old_lens > 0
        keep[list(new_rows)] = False
        ids = np.nonzero(keep)[0]
        ln = old_lens[ids]
        if ln.sum():
            within = np.arange(int(ln.sum()), dtype=np.int64) - np.repeat(np.cumsum(ln) - ln, ln)
            mem[np.repeat(off[ids].astype(np.int64), ln) + within] = \
                self.mem[np.repeat(self.off[ids].astype(np.int64), ln) + within]
        for h, r in new_rows.items():
            mem[int(off[h]):int(off[h + 1])] = r
        self.off, self.mem = off, mem
        return OK, np.array(sorted(new_rows), dtype=np.int64)

    def _args(self):
        return (self.n_slots, _p(self.off), _p(self.mem), _p(self.live), self.n_vertices)

    def he_counts(self) -> np.ndarray:
        out = np.zeros(N_HE, dtype=np.uint64)
        rc = lib().orc_count_full(*self._args(), _p(self.ts), _p(self.seq), self.window, _p(out), None)
        assert rc == 0
        return out

    def temporal_counts(self, window: Optional[int] = None) -> np.ndarray:
        out = np.zeros(N_TMP, dtype=np.uint64)
        w = self.window if window is None else int(window)
        rc = lib().orc_count_full(*self._args(), _p(self.ts), _p(self.seq), w, None, _p(out))
        assert rc == 0
        return out

    def iv_counts(self) -> np.ndarray:
        out = np.zeros(N_IV, dtype=np.uint64)
        rc = lib().orc_count_iv(*self._args(), _p(out))
        assert rc == 0
        return out

    def counts_containing(self, ids: Sequence[int], window: Optional[int] = None, he: bool = True,
                          temporal: bool = True):
        """(he u64[30], temporal u64[96]) of the triads containing >= 1 of ids;
        a family switched off (or temporal on a graph without timestamps) is
        returned as zeros without being counted."""
        marked = np.zeros(self.n_slots, dtype=np.uint8)
        ids = np.asarray(ids, dtype=np.int64)
        if len(ids):
            marked[ids] = 1
        he_out = np.zeros(N_HE, dtype=np.uint64)
        tm = np.zeros(N_TMP, dtype=np.uint64)
        w = self.window if window is None else int(window)
        rc = lib().orc_count_containing(*self._args(), _p(self.ts), _p(self.seq), w, _p(marked),
                                        _p(he_out) if he else None, _p(tm) if (self.temporal and temporal) else None)
        assert rc == 0
        return he_out, tm

    def pairs_of(self, ids: Sequence[int]) -> np.ndarray:
        """Distinct vertex pairs (u << 32 | v, u < v, ascending) inside the rows of ids."""
        ids = np.asarray(ids, dtype=np.uint64)
        if len(ids) == 0:
            return np.zeros(0, np.uint64)
        lens = (self.off[ids.astype(np.int64) + 1] - self.off[ids.astype(np.int64)]).astype(np.int64)
        out = np.zeros(max(1, int((lens * (lens - 1) // 2).sum())), dtype=np.uint64)
        n = lib().orc_pairs_of(_p(self.off), _p(self.mem), _p(ids), len(ids), _p(out))
        return out[:n].copy()

    def iv_partial(self, keys: np.ndarray):
        """(sum over the listed pairs of m_p w_p, sum over the triangles with a
        listed pair of m m m): the two closed-form sums restricted to keys."""
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        out = np.zeros(2, dtype=np.uint64)
        rc = lib().orc_iv_partial(*self._args(), _p(keys), len(keys), _p(out))
        assert rc == 0
        return out


def delta_by_definition(old: OracleGraph, new: OracleGraph, del_ids, ins_ids, he: bool = True,
                        temporal: bool = True):
    """Per-class change of the hyperedge and temporal counts from old to new:
    triads of new containing an inserted hyperedge minus triads of old
    containing a deleted one (mod 2^64)."""
    he_d, tm_d = old.counts_containing(del_ids, he=he, temporal=temporal)
    he_i, tm_i = new.counts_containing(ins_ids, he=he, temporal=temporal)
    return he_i - he_d, tm_i - tm_d


def _choose3(d: np.ndarray) -> np.ndarray:
    d = d.astype(np.uint64)
    return np.where(d >= 3, d * (d - np.uint64(1)) * (d - np.uint64(2)) // np.uint64(6), np.uint64(0))


def iv_delta_by_definition(old: OracleGraph, new: OracleGraph, del_ids, ins_ids) -> np.ndarray:
    """Change of the incident-vertex counts [T1, T2, T3] from old to new
    (mod 2^64), from the closed forms restricted to the vertex pairs inside a
    deleted or inserted hyperedge: only those pairs change m_p and w_p, and
    only triangles holding one of them change their product.
      dT1 = sum_ins C(|h|,3) - sum_del C(|h|,3)
      dT2 = d(sum_p m_p w_p) - 3 dT1
      dT3 = d(sum over triangles of m m m) - dT1 - dT2"""
    del_ids = np.asarray(del_ids, dtype=np.int64)
    ins_ids = np.asarray(ins_ids, dtype=np.int64)
    keys = np.union1d(old.pairs_of(del_ids), new.pairs_of(ins_ids)).astype(np.uint64)
    so = old.iv_partial(keys)
    sn = new.iv_partial(keys)
    with np.errstate(over="ignore"):
        t1 = np.uint64(_choose3(new.lens()[ins_ids]).sum(dtype=np.uint64)) - \
             np.uint64(_choose3(old.lens()[del_ids]).sum(dtype=np.uint64))
        ds = sn[0] - so[0]
        dx = sn[1] - so[1]
        d2 = ds - np.uint64(3) * t1
        d3 = dx - t1 - d2
    return np.array([t1, d2, d3], dtype=np.uint64)
