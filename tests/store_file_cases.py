"""Stored-summary files built byte by byte for the host-side file check: one
consistent two-table file (the layout gj_summary_save writes) and damaged
copies of it, each of which the check must refuse.  Layout, little-endian:
magic "GJSUMM01"; int32 version, n_tables, projected, with_rows; int64 join
size; per table int32 k, sep, pcol, parent, is_root (+4 bytes padding) and
int64 entries, groups, rows; then per table its keys (column-major int32),
c, U, D, F, pre (int64), for t >= 1 the edge's s (int32), M, D (int64) and
one 16-byte child record (first, end, c0, st0 int32) per parent entry, and
with rows the (count, first) int32 pairs and the grouped row ids."""
import struct

import numpy as np

HDR = struct.Struct("<8s4iq")
TAB = struct.Struct("<5i4xqqq")

# root T0(A,B): rows 3, entries 2 (counts 1 and 2); T1(B,C) child on B: rows 2, entries 2, one group
T0 = dict(k=2, sep=0, pcol=0, parent=-1, is_root=1, entries=2, groups=2, rows=3)
T1 = dict(k=2, sep=0, pcol=1, parent=0, is_root=0, entries=2, groups=1, rows=2)


def _i32(a):
    return np.asarray(a, dtype="<i4").tobytes()


def _i64(a):
    return np.asarray(a, dtype="<i8").tobytes()


def sections(with_rows=True):
    """(name, bytes) of every section in file order."""
    out = []
    out += [("t0.key0", _i32([1, 2])), ("t0.key1", _i32([5, 5]))]
    for nm, v in (("c", [1, 2]), ("U", [2, 2]), ("D", [1, 1]), ("F", [2, 4]), ("pre", [0, 2])):
        out.append(("t0." + nm, _i64(v)))
    out += [("t1.key0", _i32([5, 5])), ("t1.key1", _i32([7, 8]))]
    for nm, v in (("c", [1, 1]), ("U", [1, 1]), ("D", [3, 3]), ("F", [3, 3]), ("pre", [0, 1])):
        out.append(("t1." + nm, _i64(v)))
    out += [("t1.s", _i32([5])), ("t1.M", _i64([2])), ("t1.Dg", _i64([3]))]
    rec = b"".join(struct.pack("<4i", 0, 2, 1, 0) for _ in range(T0["entries"]))
    out.append(("t1.crec", rec))
    if with_rows:
        out.insert(7, ("t0.ccs", _i32([1, 0, 2, 1])))
        out.insert(8, ("t0.rows", _i32([2, 0, 1])))
        out += [("t1.ccs", _i32([1, 0, 1, 1])), ("t1.rows", _i32([1, 0]))]
    return out


VERSION = 2


def build(with_rows=True, tables=(T0, T1), join_size=6, version=VERSION, magic=b"GJSUMM01", secs=None):
    b = HDR.pack(magic, version, len(tables), 0, 1 if with_rows else 0, join_size)
    for t in tables:
        b += TAB.pack(t["k"], t["sep"], t["pcol"], t["parent"], t["is_root"], t["entries"], t["groups"], t["rows"])
    for _, s in (secs if secs is not None else sections(with_rows)):
        b += s
    return b


def _patch_section(name, data, with_rows=True):
    return [(n, data if n == name else s) for n, s in sections(with_rows)]


def damaged():
    """(reason, file bytes) pairs the check must refuse."""
    good = build()
    bad = [
        ("empty file", b""),
        ("wrong magic", build(magic=b"GJSUMM02")),
        ("older version (32-byte child records)", build(version=1)),
        ("newer version", build(version=VERSION + 1)),
        ("zero tables", HDR.pack(b"GJSUMM01", VERSION, 0, 0, 1, 6)),
        ("negative join size", build(join_size=-1)),
        ("truncated table headers", good[: HDR.size + TAB.size + 5]),
        ("truncated last section", good[:-3]),
        ("data after the last section", good + b"\0"),
        ("key count 0", build(tables=(dict(T0, k=0), T1))),
        ("parent after child", build(tables=(T0, dict(T1, parent=1)))),
        ("separator column out of range", build(tables=(T0, dict(T1, sep=2)))),
        ("parent column out of range", build(tables=(T0, dict(T1, pcol=2)))),
        ("more entries than rows", build(tables=(dict(T0, entries=4), T1))),
        ("entry count 0", build(secs=_patch_section("t0.c", _i64([1, 0])))),
        ("child record past the child's entries",
         build(secs=_patch_section("t1.crec", struct.pack("<4i", 0, 3, 1, 0) * 2))),
        ("child record with first > end",
         build(secs=_patch_section("t1.crec", struct.pack("<4i", 2, 1, 1, 0) * 2))),
        ("row range past the table", build(secs=_patch_section("t0.ccs", _i32([1, 0, 2, 2])))),
        ("row id out of range", build(secs=_patch_section("t1.rows", _i32([1, 2])))),
    ]
    return bad
