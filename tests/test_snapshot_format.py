"""CPU checks of the snapshot byte form (include/hgt.h, "snapshot and
restore"): a snapshot written here from the documented layout loads, its
bytes come back unchanged, and every kind of damage -- to the header, the
checksum or the structure of the incidence maps -- is refused with
HGT_EINVAL.  hgt_snap_load runs on the host only, so no GPU is needed."""
import ctypes
import struct

import numpy as np
import pytest

from .test_abi import _lib_path

EINVAL = -1
N_COUNTS = 129
HE, IV, TMP = 1, 2, 4


def checksum(payload: bytes) -> int:
    h = 0xCBF29CE484222325
    for (w,) in struct.iter_unpack("<Q", payload):
        h = ((h ^ w) * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


def _pad8(b: bytes) -> bytes:
    return b + b"\0" * (-len(b) % 8)


class Spec:
    """A small consistent graph state: rows[i] is the sorted member list of
    ID i, or None for a free ID."""

    def __init__(self, n_vertices=10, track=HE | IV | TMP, window=50):
        self.nv, self.track, self.window = n_vertices, track, window
        self.rows = [[0, 1, 2], None, [1, 3], [2, 3, 4, 9], [5]]
        self.ts = [10, 0, 12, 15, 20]
        self.seq = [0, 0, 2, 3, 4]
        self.next_seq = 5
        self.counts = np.arange(N_COUNTS, dtype=np.uint64)

    def sections(self):
        """Every field of the layout, in order, as numpy arrays (before padding)."""
        n = len(self.rows)
        h_off, h_len, h_cap, h2v = [], [], [], []
        for r in self.rows:
            cap = 0 if r is None else max(4, 1 << (len(r) - 1).bit_length())
            h_off.append(len(h2v) if cap else 0)
            h_len.append(0 if r is None else len(r))
            h_cap.append(cap)
            h2v += (r or []) + [0] * (cap - len(r or []))
        v_lists = [[i for i, r in enumerate(self.rows) if r is not None and v in r] for v in range(self.nv)]
        v_off, v_len, v_cap, v2h, v2h_ts = [], [], [], [], []
        for lst in v_lists:
            cap = len(lst) + 1 if lst else 0
            v_off.append(len(v2h) if cap else 0)
            v_len.append(len(lst))
            v_cap.append(cap)
            v2h += lst + [0] * (cap - len(lst))
            v2h_ts += [self.ts[i] for i in lst] + [0] * (cap - len(lst))
        bm = np.zeros((n + 63) // 64, np.uint64)
        for i, r in enumerate(self.rows):
            if r is None:
                bm[i >> 6] |= np.uint64(1 << (i & 63))
        u64, u32, i64 = np.uint64, np.uint32, np.int64
        sec = {
            "counts": self.counts.astype(u64), "h_off": np.array(h_off, u64), "h_len": np.array(h_len, u32),
            "h_cap": np.array(h_cap, u32), "h_seq": np.array(self.seq, u64),
            "h_ts": np.array(self.ts, i64) if self.track & TMP else None, "free_bm": bm,
            "h2v": np.array(h2v, u32), "hist": np.zeros(2 * len(h2v), u32) if self.track & HE else None,
            "v_off": np.array(v_off, u64), "v_len": np.array(v_len, u32), "v_cap": np.array(v_cap, u32),
            "v2h": np.array(v2h, u32), "v2h_ts": np.array(v2h_ts, i64) if self.track & TMP else None,
        }
        return sec

    def encode(self, edit=None, fix_checksum=True, header_edit=None):
        sec = self.sections()
        if edit:
            edit(sec)
        payload = b"".join(_pad8(a.tobytes()) for a in sec.values() if a is not None)
        live = [r for r in self.rows if r is not None]
        hdr = dict(version=1, track=self.track, nv=self.nv, n_counts=N_COUNTS, window=self.window,
                   next_id=len(self.rows), h_bump=len(sec["h2v"]), v_bump=len(sec["v2h"]), next_seq=self.next_seq,
                   n_live=len(live), n_inc=sum(map(len, live)),
                   last_ts=max(self.ts) if self.track & TMP else -(1 << 63), payload=len(payload),
                   checksum=checksum(payload))
        if header_edit:
            header_edit(hdr)
        if not fix_checksum:
            hdr["checksum"] ^= 1
        head = b"HGTSNAP1" + struct.pack("<IIIIqQQQQQQqQQ", hdr["version"], hdr["track"], hdr["nv"], hdr["n_counts"],
                                         hdr["window"], hdr["next_id"], hdr["h_bump"], hdr["v_bump"],
                                         hdr["next_seq"], hdr["n_live"], hdr["n_inc"], hdr["last_ts"],
                                         hdr["payload"], hdr["checksum"])
        head += b"\0" * (128 - len(head))
        return head + payload


@pytest.fixture(scope="module")
def lib():
    lib = ctypes.CDLL(_lib_path())
    P, U64 = ctypes.c_void_p, ctypes.c_uint64
    lib.hgt_snap_load.argtypes = [P, U64, ctypes.POINTER(P)]
    lib.hgt_snap_bytes.argtypes = [P, P, U64, ctypes.POINTER(U64)]
    lib.hgt_snap_free.argtypes = [P]
    return lib


def load(lib, data: bytes):
    out = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(data, len(data))
    rc = lib.hgt_snap_load(ctypes.cast(buf, ctypes.c_void_p), len(data), ctypes.byref(out))
    return rc, out


@pytest.mark.parametrize("track", [HE | IV | TMP, HE, IV, TMP, HE | IV])
def test_valid_snapshot_loads_and_round_trips(lib, track):
    data = Spec(track=track).encode()
    rc, snap = load(lib, data)
    assert rc == 0
    n = ctypes.c_uint64(0)
    assert lib.hgt_snap_bytes(snap, None, 0, ctypes.byref(n)) == 0 and n.value == len(data)
    buf = ctypes.create_string_buffer(len(data))
    assert lib.hgt_snap_bytes(snap, ctypes.cast(buf, ctypes.c_void_p), len(data) - 8, ctypes.byref(n)) == EINVAL
    assert lib.hgt_snap_bytes(snap, ctypes.cast(buf, ctypes.c_void_p), len(data), ctypes.byref(n)) == 0
    assert buf.raw == data
    assert lib.hgt_snap_free(snap) == 0


def test_empty_graph_snapshot_loads(lib):
    s = Spec()
    s.rows, s.ts, s.seq, s.next_seq = [], [], [], 0
    s.track = HE | IV
    assert load(lib, s.encode())[0] == 0


def test_header_damage_is_refused(lib):
    good = Spec().encode()
    assert load(lib, good[:-8])[0] == EINVAL                  # truncated
    assert load(lib, good + b"\0" * 8)[0] == EINVAL           # trailing words
    assert load(lib, good[:-3])[0] == EINVAL                  # not whole words
    assert load(lib, b"HGTSNAP2" + good[8:])[0] == EINVAL     # magic
    for key, val in (("version", 2), ("n_counts", 128), ("track", 8), ("nv", 0), ("window", -1),
                     ("payload", len(good) - 136)):
        assert load(lib, Spec().encode(header_edit=lambda h: h.__setitem__(key, val)))[0] == EINVAL, key


def test_checksum_damage_is_refused(lib):
    assert load(lib, Spec().encode(fix_checksum=False))[0] == EINVAL
    data = bytearray(Spec().encode())
    data[128 + 8 * N_COUNTS + 3] ^= 0x10  # one bit of h_off, checksum left as it was
    assert load(lib, bytes(data))[0] == EINVAL


def _edit(name, fn):
    return lambda sec: fn(sec[name])


@pytest.mark.parametrize("case", [
    "member_out_of_range", "row_not_ascending", "row_past_pool", "live_len_zero", "len_over_cap",
    "v2h_missing_incidence", "v2h_names_free_id", "v2h_not_ascending", "v2h_ts_differs", "seq_not_below_next",
    "free_bit_above_next_id", "n_live_wrong", "n_inc_wrong", "ts_after_last",
])
def test_structural_damage_is_refused(lib, case):
    """Each edit keeps the header and checksum consistent with the payload, so
    only the structural checks can catch it."""
    s = Spec()
    he, hdr = None, None
    if case == "member_out_of_range":
        s.rows[0] = [0, 1, 10]
    elif case == "row_not_ascending":
        he = _edit("h2v", lambda a: a.__setitem__(slice(0, 2), [1, 0]))
    elif case == "row_past_pool":
        he = _edit("h_off", lambda a: a.__setitem__(4, 10 ** 6))
    elif case == "live_len_zero":
        he = _edit("h_len", lambda a: a.__setitem__(4, 0))
    elif case == "len_over_cap":
        he = _edit("h_cap", lambda a: a.__setitem__(3, 2))
    elif case == "v2h_missing_incidence":
        def drop(sec):  # vertex 9 loses its only hyperedge; v2h then misses (3, 9)
            sec["v_len"][9] = 0
        he = drop
        hdr = None
    elif case == "v2h_names_free_id":
        def free_id(sec):  # vertex 0 lists free ID 1 in place of ID 0
            sec["v2h"][sec["v_off"][0]] = 1
        he = free_id
    elif case == "v2h_not_ascending":
        def swap(sec):  # vertex 3 lists IDs 2 and 3; swap them
            o = int(sec["v_off"][3])
            sec["v2h"][o], sec["v2h"][o + 1] = sec["v2h"][o + 1], sec["v2h"][o]
        he = swap
    elif case == "v2h_ts_differs":
        he = _edit("v2h_ts", lambda a: a.__setitem__(0, 11))
    elif case == "seq_not_below_next":
        s.next_seq = 4
    elif case == "free_bit_above_next_id":
        he = _edit("free_bm", lambda a: a.__setitem__(0, a[0] | np.uint64(1 << 5)))
    elif case == "n_live_wrong":
        hdr = lambda h: h.__setitem__("n_live", h["n_live"] + 1)  # noqa: E731
    elif case == "n_inc_wrong":
        hdr = lambda h: h.__setitem__("n_inc", h["n_inc"] - 1)  # noqa: E731
    elif case == "ts_after_last":
        hdr = lambda h: h.__setitem__("last_ts", 19)  # noqa: E731
    assert load(lib, s.encode())[0] == 0 or case in ("member_out_of_range", "seq_not_below_next")
    assert load(lib, s.encode(edit=he, header_edit=hdr))[0] == EINVAL, case


@pytest.mark.parametrize("seed", range(4))
def test_random_graphs_load_and_damage_is_refused(lib, seed):
    """Seeded random states spanning several bitmap words (some IDs free, rows
    up to 12 members): each loads; then one incidence is dropped from the v2h
    map, one member is pushed out of range, or a free ID is marked live, with
    header and checksum kept consistent, and each is refused."""
    rng = np.random.default_rng(seed)
    s = Spec(n_vertices=40, track=HE | IV if seed % 2 else HE | IV | TMP)
    n = 150 + seed
    s.rows = [None if rng.random() < 0.2 else sorted(rng.choice(40, rng.integers(1, 13), replace=False).tolist())
              for _ in range(n)]
    s.ts = sorted(rng.integers(0, 1000, n).tolist())
    s.seq = list(range(n))
    s.next_seq = n
    assert load(lib, s.encode())[0] == 0
    live = [i for i, r in enumerate(s.rows) if r is not None]
    victim = int(rng.choice(live))
    v = s.rows[victim][0]

    def drop_incidence(sec):  # the victim disappears from its first member's list
        o, ln = int(sec["v_off"][v]), int(sec["v_len"][v])
        lst = [x for x in sec["v2h"][o:o + ln] if x != victim]
        sec["v2h"][o:o + ln - 1] = lst
        sec["v_len"][v] = ln - 1

    def member_out_of_range(sec):
        sec["h2v"][int(sec["h_off"][victim]) + len(s.rows[victim]) - 1] = 40

    free = [i for i, r in enumerate(s.rows) if r is None]

    def free_marked_live(sec):
        i = free[0]
        sec["free_bm"][i >> 6] &= ~np.uint64(1 << (i & 63))

    for edit in (drop_incidence, member_out_of_range, free_marked_live):
        # with free_marked_live, n_live is raised too, so only the structure is wrong
        hdr = (lambda h: h.__setitem__("n_live", h["n_live"] + 1)) if edit is free_marked_live else None
        assert load(lib, s.encode(edit=edit, header_edit=hdr))[0] == EINVAL, edit.__name__


def test_binding_saves_and_loads_checkpoint_files(tmp_path):
    """Snapshot.load_file / save (the binding's checkpoint files) keep the
    bytes exactly, and a damaged file is refused."""
    from paper_2512_21009_amd import hgt
    _lib_path()
    data = Spec().encode()
    src = tmp_path / "a.snap"
    src.write_bytes(data)
    snap = hgt.Snapshot.load_file(str(src))
    dst = tmp_path / "b.snap"
    snap.save(str(dst))
    assert dst.read_bytes() == data
    snap.close()
    src.write_bytes(data[:-8])
    with pytest.raises(hgt.HgtError) as e:
        hgt.Snapshot.load_file(str(src))
    assert e.value.code == hgt.EINVAL
