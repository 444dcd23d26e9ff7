"""ctypes wrapper over the CPU oracle (``liboracle.so``).  TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It never touches the HIP library and the HIP library
never touches it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "gj_oracle.cpp")
SRCS = [SRC, os.path.join(HERE, "gj_natural.cpp")]
MAXK = 8

OVERFLOW = 3
RANGE = 6
NOT_IN_RESULT = 2


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (host only; no HIP headers)."""
    stale = not os.path.exists(LIB) or any(os.path.getmtime(LIB) < os.path.getmtime(f) for f in SRCS)
    if force or stale:
        cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread", *SRCS, "-o", LIB + ".tmp"]
        subprocess.check_call(cmd)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class _Q(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_rows", C.c_void_p), ("n_keys", C.c_void_p),
                ("cols", C.c_void_p), ("parent", C.c_void_p), ("sep_col", C.c_void_p),
                ("parent_col", C.c_void_p)]


_lib = None


def _declare(L):
    """Argument and return types of every exported oracle function."""
    vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
    L.orc_open.restype = vp
    L.orc_open.argtypes = [vp]
    L.orc_close.argtypes = [vp]
    L.orc_join_size.argtypes = [vp, vp]
    L.orc_join_size.restype = C.c_int
    L.orc_factor.argtypes = [vp, C.c_int, vp, vp, vp, vp]
    L.orc_factor.restype = i64
    L.orc_summary_table.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp]
    L.orc_summary_table.restype = i64
    L.orc_summary_edge.argtypes = [vp, C.c_int, vp, vp, vp]
    L.orc_summary_edge.restype = i64
    L.orc_fanouts.argtypes = [vp, C.c_int, vp]
    L.orc_materialize.argtypes = [vp, i64, vp]
    L.orc_materialize_range.argtypes = [vp, i64, i64, i64, vp]
    L.orc_materialize_range.restype = i64
    L.orc_materialize.restype = i64
    L.orc_brute_force.argtypes = [vp, i64, vp]
    L.orc_brute_force.restype = i64
    L.orc_sort_canonical.argtypes = [vp, vp, i64]
    L.orc_n_levels.argtypes = [vp]
    L.orc_n_levels.restype = C.c_int
    L.orc_gfjs.argtypes = [vp, vp, i64, vp, vp, vp]
    L.orc_unrank.argtypes = [vp, i64, vp]
    L.orc_unrank.restype = C.c_int
    L.orc_rank.argtypes = [vp, vp, vp]
    L.orc_rank.restype = C.c_int
    L.orc_weighted.argtypes = [vp, vp, vp]
    L.orc_weighted.restype = C.c_double
    L.orc_weighted_fd.argtypes = [vp, vp, C.c_int, vp, i64, C.c_double, C.c_int, vp]
    L.orc_projection.argtypes = [vp, vp, vp, vp]
    L.orc_projection.restype = C.c_int
    L.orc_projected_table.argtypes = [vp, vp, C.c_int, vp, vp, vp, vp, vp]
    L.orc_projected_table.restype = i64
    L.orc_check_tuples.argtypes = [vp, vp, i64, C.c_int]
    L.orc_check_tuples.restype = i64
    L.orc_nat_open.restype = vp
    L.orc_nat_open.argtypes = [i32, vp, vp, vp, vp]
    L.orc_nat_close.argtypes = [vp]
    L.orc_nat_materialize.argtypes = [vp, i64, vp]
    L.orc_nat_materialize.restype = i64
    L.orc_nat_brute_force.argtypes = [vp, i64, vp]
    L.orc_nat_brute_force.restype = i64
    return L


def load_at(path: str):
    """The oracle library at `path` (a build of these sources elsewhere, e.g.
    a sanitizer build or a test's scratch copy), with its types declared."""
    return _declare(C.CDLL(path))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = _declare(C.CDLL(LIB))
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class Oracle:
    """Row-level reference for one query (see gj_oracle.cpp for definitions)."""

    def __init__(self, q, L=None):
        """`L`: an oracle library from load_at (default: the one built here)."""
        self.q = q
        self.L = L if L is not None else lib()
        n = q.n_tables
        self._cols = [[np.ascontiguousarray(c, dtype=np.int32) for c in tb] for tb in q.tables]
        self._nrows = np.array([q.n_rows(t) for t in range(n)], dtype=np.int64)
        self._nkeys = np.array([len(tb) for tb in q.tables], dtype=np.int32)
        ptrs = np.zeros(n * MAXK, dtype=np.uint64)
        for t in range(n):
            for c, col in enumerate(self._cols[t]):
                ptrs[t * MAXK + c] = col.ctypes.data
        self._ptrs = ptrs
        self._par = np.array(q.parent, dtype=np.int32)
        self._sep = np.array(q.sep_col, dtype=np.int32)
        self._pcol = np.array(q.parent_col, dtype=np.int32)
        self._qs = _Q(n, self._nrows.ctypes.data, self._nkeys.ctypes.data, ptrs.ctypes.data,
                      self._par.ctypes.data, self._sep.ctypes.data, self._pcol.ctypes.data)
        self.h = self.L.orc_open(C.byref(self._qs))

    def close(self):
        if self.h:
            self.L.orc_close(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n(self):
        return self.q.n_tables

    def join_size(self):
        """(|Q|, overflow flag)."""
        out = np.zeros(1, dtype=np.int64)
        rc = self.L.orc_join_size(self.h, _p(out))
        return int(out[0]), rc == OVERFLOW

    def factor(self, t):
        N = self.q.n_rows(t)
        k = len(self.q.tables[t])
        keys = np.zeros((max(N, 1), k), dtype=np.int32)
        cnt = np.zeros(max(N, 1), dtype=np.int64)
        start = np.zeros(max(N, 1), dtype=np.int64)
        perm = np.zeros(max(N, 1), dtype=np.int32)
        M = self.L.orc_factor(self.h, t, _p(keys), _p(cnt), _p(start), _p(perm))
        return dict(keys=keys[:M], count=cnt[:M], start=start[:M], perm=perm[:N])

    def summary_table(self, t):
        N = self.q.n_rows(t)
        k = len(self.q.tables[t])
        cap = max(N, 1)
        keys = np.zeros((cap, k), dtype=np.int32)
        arrs = [np.zeros(cap, dtype=np.int64) for _ in range(4)]
        m = self.L.orc_summary_table(self.h, t, _p(keys), *[_p(a) for a in arrs])
        return dict(keys=keys[:m], c=arrs[0][:m], U=arrs[1][:m], D=arrs[2][:m], F=arrs[3][:m])

    def summary_edge(self, t):
        N = self.q.n_rows(t)
        cap = max(N, 1)
        s = np.zeros(cap, dtype=np.int32)
        M = np.zeros(cap, dtype=np.int64)
        D = np.zeros(cap, dtype=np.int64)
        m = self.L.orc_summary_edge(self.h, t, _p(s), _p(M), _p(D))
        return dict(s=s[:m], M=M[:m], D=D[:m])

    def fanouts(self, t):
        out = np.zeros(max(self.q.n_rows(t), 1), dtype=np.int64)
        self.L.orc_fanouts(self.h, t, _p(out))
        return out[: self.q.n_rows(t)]

    def materialize(self, limit=None):
        if limit is None:
            limit = self.join_size()[0]
        if limit > 200_000_000:
            raise MemoryError(f"refusing to materialize {limit} tuples in host memory")
        out = np.zeros((max(limit, 1), self.n), dtype=np.int32)
        m = self.L.orc_materialize(self.h, int(limit), _p(out))
        return out[:m]

    def materialize_range(self, lo, hi, limit):
        """Result tuples whose root row is in [lo, hi), first `limit` in DFS order."""
        out = np.zeros((max(limit, 1), self.n), dtype=np.int32)
        m = self.L.orc_materialize_range(self.h, int(lo), int(hi), int(limit), _p(out))
        return out[:m]

    def materialize_threads(self, limit, threads):
        """`threads` DFS expansions side by side, thread i over the i-th of
        `threads` equal ranges of root rows, each writing up to limit/threads
        tuples into its own buffer (ctypes drops the GIL during the calls).
        Returns the parts in range order."""
        import concurrent.futures as cf

        n0 = self.q.n_rows(0)
        cuts = [n0 * i // threads for i in range(threads + 1)]
        each = max(1, limit // threads)
        with cf.ThreadPoolExecutor(max_workers=threads) as ex:
            return list(ex.map(lambda i: self.materialize_range(cuts[i], cuts[i + 1], each), range(threads)))

    def brute_force(self, limit=10**7):
        out = np.zeros((limit, self.n), dtype=np.int32)
        m = self.L.orc_brute_force(self.h, int(limit), _p(out))
        return out[:m]

    def sort_canonical(self, tuples):
        t = np.ascontiguousarray(tuples, dtype=np.int32).copy()
        self.L.orc_sort_canonical(self.h, _p(t), int(t.shape[0]))
        return t

    def canonical_result(self):
        return self.sort_canonical(self.materialize())

    def gfjs(self, sorted_tuples):
        """Per result column: list of (value, freq) runs (Definition 1 per prefix)."""
        st = np.ascontiguousarray(sorted_tuples, dtype=np.int32)
        L = self.L.orc_n_levels(self.h)
        cnt = st.shape[0]
        vals = np.zeros((L, max(cnt, 1)), dtype=np.int32)
        freqs = np.zeros((L, max(cnt, 1)), dtype=np.int64)
        nr = np.zeros(L, dtype=np.int64)
        self.L.orc_gfjs(self.h, _p(st), cnt, _p(vals), _p(freqs), _p(nr))
        return [(vals[i, : nr[i]].copy(), freqs[i, : nr[i]].copy()) for i in range(L)]

    def check_tuples(self, tuples, threads=8):
        """-1 if every row-id tuple (count x n, int64) is a join tuple coming
        strictly after its predecessor in the result order; else the index of
        the first one that is not."""
        t = np.ascontiguousarray(tuples, dtype=np.int64)
        return int(self.L.orc_check_tuples(self.h, _p(t), int(t.shape[0]), int(threads)))

    def unrank(self, R):
        out = np.zeros(self.n, dtype=np.int32)
        rc = self.L.orc_unrank(self.h, int(R), _p(out))
        if rc != 0:
            raise IndexError(R)
        return out

    def rank(self, tup):
        t = np.ascontiguousarray(tup, dtype=np.int32)
        out = np.zeros(1, dtype=np.int64)
        rc = self.L.orc_rank(self.h, _p(t), _p(out))
        if rc != 0:
            raise ValueError("tuple is not in the join result")
        return int(out[0])

    def _wptrs(self, w):
        if w is None:
            return None, None
        ws = [np.ascontiguousarray(x, dtype=np.float64) for x in w]
        ptrs = np.array([x.ctypes.data for x in ws], dtype=np.uint64)
        return ws, ptrs

    def weighted(self, w=None, grads=True):
        """(W, [dW/dw per table]) in __float128, rounded to float64."""
        ws, ptrs = self._wptrs(w)
        g = [np.zeros(max(self.q.n_rows(t), 1)) for t in range(self.n)] if grads else None
        gp = np.array([x.ctypes.data for x in g], dtype=np.uint64) if grads else None
        W = self.L.orc_weighted(self.h, _p(ptrs) if ptrs is not None else None,
                               _p(gp) if gp is not None else None)
        return W, ([x[: self.q.n_rows(t)] for t, x in enumerate(g)] if grads else None)

    def weighted_fd(self, w, t, rows, hfrac=0.25, threads=1):
        ws, ptrs = self._wptrs(w)
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        out = np.zeros(len(rows))
        self.L.orc_weighted_fd(self.h, _p(ptrs), int(t), _p(rows), len(rows), float(hfrac),
                              int(threads), _p(out))
        return out

    # -- early projections (Sec. 3.7) ------------------------------------------
    def projection(self, mask):
        """(supported, normalized mask, kept flags) for output-attribute masks
        (bit c of mask[t] = key column c of table t)."""
        m = np.ascontiguousarray(mask, dtype=np.uint32)
        out = np.zeros(self.n, dtype=np.uint32)
        kept = np.zeros(self.n, dtype=np.int32)
        rc = self.L.orc_projection(self.h, _p(m), _p(out), _p(kept))
        return rc == 0, out, kept.astype(bool)

    def projected_columns(self, mask):
        """Result columns of the projected result as (table, column) pairs:
        the root's output columns in declared order, then for every further
        kept table its output columns other than the separator."""
        ok, m, kept = self.projection(mask)
        if not ok:
            raise ValueError("projection not supported")
        cols = []
        for t in range(self.n):
            if not kept[t]:
                continue
            for c in range(len(self.q.tables[t])):
                if (int(m[t]) >> c) & 1 and (t == 0 or c != self.q.sep_col[t]):
                    cols.append((t, c))
        return cols

    def projected_result(self, mask):
        """The projected result by definition: every result tuple restricted to
        the output attributes (multiplicities kept), sorted by all of them."""
        cols = self.projected_columns(mask)
        rows = self.materialize()
        if not cols:
            return np.zeros((len(rows), 0), np.int32)
        vals = np.stack([self.q.tables[t][c][rows[:, t]] for t, c in cols], axis=1).astype(np.int32)
        order = np.lexsort(vals.T[::-1])
        return vals[order]

    def projected_table(self, mask, t):
        m = np.ascontiguousarray(mask, dtype=np.uint32)
        ok, mn, kept = self.projection(mask)
        if not ok or not kept[t]:
            raise ValueError("table is not kept by this projection")
        k = bin(int(mn[t])).count("1")
        cap = max(self.q.n_rows(t), 1)
        keys = np.zeros((cap, max(k, 1)), dtype=np.int32)
        arrs = [np.zeros(cap, dtype=np.int64) for _ in range(4)]
        e = self.L.orc_projected_table(self.h, _p(m), int(t), _p(keys), *[_p(a) for a in arrs])
        return dict(keys=keys[:e, :k], c=arrs[0][:e], U=arrs[1][:e], D=arrs[2][:e], F=arrs[3][:e])


class NaturalOracle:
    """Natural join over named attributes (cyclic queries included): tables is
    a list of lists of int32 columns, attrs[t][c] the attribute id of column c
    of table t.  See gj_natural.cpp for the definitions."""

    def __init__(self, tables, attrs):
        self.tables = [[np.ascontiguousarray(c, dtype=np.int32) for c in tb] for tb in tables]
        self.attrs = [list(map(int, a)) for a in attrs]
        n = len(tables)
        self.n = n
        self._nrows = np.array([len(tb[0]) if tb else 0 for tb in self.tables], dtype=np.int64)
        self._nkeys = np.array([len(tb) for tb in self.tables], dtype=np.int32)
        ptrs = np.zeros(n * MAXK, dtype=np.uint64)
        at = np.zeros(n * MAXK, dtype=np.int32)
        for t in range(n):
            for c, col in enumerate(self.tables[t]):
                ptrs[t * MAXK + c] = col.ctypes.data
                at[t * MAXK + c] = self.attrs[t][c]
        self._ptrs, self._at = ptrs, at
        self.h = lib().orc_nat_open(n, _p(self._nrows), _p(self._nkeys), _p(ptrs), _p(at))

    def close(self):
        if self.h:
            lib().orc_nat_close(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def join_size(self):
        return int(lib().orc_nat_materialize(self.h, 2**62, None))

    def materialize(self, limit=None):
        if limit is None:
            limit = self.join_size()
        if limit > 200_000_000:
            raise MemoryError(f"refusing to materialize {limit} tuples in host memory")
        out = np.zeros((max(limit, 1), self.n), dtype=np.int32)
        m = lib().orc_nat_materialize(self.h, int(limit), _p(out))
        return out[:m]

    def brute_force(self, limit=10**7):
        out = np.zeros((limit, self.n), dtype=np.int32)
        m = lib().orc_nat_brute_force(self.h, int(limit), _p(out))
        return out[:m]

    def attribute_values(self, rows, attr_order):
        """Values of the given attributes for result rows (row-id tuples)."""
        where = {}
        for t in range(self.n):
            for c, a in enumerate(self.attrs[t]):
                where.setdefault(a, (t, c))
        if len(rows) == 0:
            return np.zeros((0, len(attr_order)), np.int32)
        return np.stack([self.tables[where[a][0]][where[a][1]][rows[:, where[a][0]]] for a in attr_order],
                        axis=1).astype(np.int32)

    def sorted_values(self, attr_order, rows=None):
        """The result as values of attr_order (each tuple keeps its
        multiplicity), sorted lexicographically in that order."""
        v = self.attribute_values(self.materialize() if rows is None else rows, attr_order)
        if v.shape[0] == 0 or v.shape[1] == 0:
            return v
        return v[np.lexsort(v.T[::-1])]

    def potential(self, subset, var_order):
        """Joint potential of the tables in `subset` (the product of their
        frequency tables, Sec. 3.2.1): the distinct value tuples of their
        natural join over var_order, ascending, with their counts."""
        sub = NaturalOracle([self.tables[t] for t in subset], [self.attrs[t] for t in subset])
        v = sub.sorted_values(var_order)
        sub.close()
        if v.shape[0] == 0:
            return v, np.zeros(0, np.int64)
        keys, counts = np.unique(v, axis=0, return_counts=True)
        return keys.astype(np.int32), counts.astype(np.int64)
