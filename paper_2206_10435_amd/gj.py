"""Thin ctypes binding over ``libgj.so`` (the C ABI declared in include/gj.h).

Argument marshalling only: every step of the join runs in the library's HIP
kernels.  PyTorch provides device memory (its caching allocator is handed to
the library as the allocator callback) and the stream.  If the library is
missing this module raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgj.so")

GJ_OK, GJ_E_INVALID, GJ_E_GRAPH, GJ_E_OVERFLOW, GJ_E_OOM, GJ_E_DEVICE, GJ_E_RANGE = range(7)
STATUS_NAMES = {0: "GJ_OK", 1: "GJ_E_INVALID", 2: "GJ_E_GRAPH", 3: "GJ_E_OVERFLOW", 4: "GJ_E_OOM",
                5: "GJ_E_DEVICE", 6: "GJ_E_RANGE"}
MAX_TABLES, MAX_KEYS, MAX_CHILDREN, MAX_ATTRS = 16, 8, 8, 64


class GJError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class _Table(C.Structure):
    _fields_ = [("n_rows", C.c_int64), ("n_keys", C.c_int32), ("keys", C.c_void_p)]


class _Graph(C.Structure):
    _fields_ = [("n_tables", C.c_int32), ("parent", C.c_void_p), ("sep_col", C.c_void_p),
                ("parent_col", C.c_void_p)]


class _FactorView(C.Structure):
    _fields_ = [("n_entries", C.c_int64), ("n_rows", C.c_int64), ("n_keys", C.c_int32),
                ("keys", C.c_void_p * MAX_KEYS), ("count", C.c_void_p), ("start", C.c_void_p),
                ("end", C.c_void_p), ("perm", C.c_void_p)]


class _SummaryView(C.Structure):
    _fields_ = [("n_entries", C.c_int64), ("n_keys", C.c_int32), ("keys", C.c_void_p * MAX_KEYS),
                ("c", C.c_void_p), ("U", C.c_void_p), ("D", C.c_void_p), ("F", C.c_void_p),
                ("pre", C.c_void_p)]


class _EdgeView(C.Structure):
    _fields_ = [("n", C.c_int64), ("s", C.c_void_p), ("M", C.c_void_p), ("D", C.c_void_p)]


class _NatQuery(C.Structure):
    _fields_ = [("n_tables", C.c_int32), ("n_keys", C.c_void_p), ("attr", C.c_void_p)]


class _JTree(C.Structure):
    _fields_ = [("n_attrs", C.c_int32), ("attr_id", C.c_int32 * MAX_ATTRS),
                ("elim_order", C.c_int32 * MAX_ATTRS), ("n_fill", C.c_int32), ("n_cliques", C.c_int32),
                ("clique", C.c_uint64 * MAX_ATTRS), ("parent", C.c_int32 * MAX_ATTRS),
                ("table_clique", C.c_int32 * MAX_TABLES)]


class _PotView(C.Structure):
    _fields_ = [("n_entries", C.c_int64), ("n_vars", C.c_int32), ("attr", C.c_int32 * MAX_ATTRS),
                ("keys", C.c_void_p * MAX_ATTRS), ("freq", C.c_void_p)]


class Tune(C.Structure):
    _fields_ = [("sort_items", C.c_int32), ("radix_bits", C.c_int32), ("desum_rounds", C.c_int32),
                ("desum_stage", C.c_int32), ("batch_task_rows", C.c_int32), ("desum_general", C.c_int32),
                ("sort_local_rows", C.c_int32)]


class SummaryFileInfo(C.Structure):
    _fields_ = [("n_tables", C.c_int32), ("projected", C.c_int32), ("with_rows", C.c_int32),
                ("join_size", C.c_int64), ("entries", C.c_int64 * 16), ("rows", C.c_int64 * 16),
                ("bytes", C.c_int64)]


class DesumLaunch(C.Structure):
    _fields_ = [("stage", C.c_int32), ("tuples_per_lane", C.c_int32), ("kernel_tables", C.c_int32),
                ("change_bits", C.c_int32), ("seg_bytes", C.c_int32), ("blocks", C.c_int64),
                ("lds_bytes", C.c_int64), ("lds_used", C.c_int64)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

_lib = None

# every exported function: name -> (restype, argtypes)
_vp, _i32, _i64, _sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
SIGNATURES = {
    "gj_ctx_create": (C.c_int, [C.c_int, _vp, ALLOC_FN, FREE_FN, _vp, _vp]),
    "gj_ctx_destroy": (None, [_vp]),
    "gj_last_error": (C.c_char_p, [_vp]),
    "gj_validate": (C.c_int, [_vp, _vp]),
    "gj_build_factors": (C.c_int, [_vp, _vp, _vp, _vp]),
    "gj_factor_table": (C.c_int, [_vp, _i32, _vp]),
    "gj_factor_sort": (C.c_int, [_vp, _i32, _vp]),
    "gj_free_factors": (None, [_vp]),
    "gj_summarize": (C.c_int, [_vp, _vp, _vp, _vp]),
    "gj_summarize_batch": (C.c_int, [_vp, _vp, _i32, _vp, _vp, _vp]),
    "gj_summary_table": (C.c_int, [_vp, _i32, _vp]),
    "gj_summary_edge": (C.c_int, [_vp, _i32, _vp]),
    "gj_summary_join_size": (_i64, [_vp]),
    "gj_free_summary": (None, [_vp]),
    "gj_desummarize": (C.c_int, [_vp, _vp, _i64, _i64, _i32, _vp, _vp]),
    "gj_result_columns": (_i32, [_vp]),
    "gj_unroll_gfjs": (C.c_int, [_vp, _vp, _i64, _i64, _vp, _vp, _vp]),
    "gj_weighted_forward": (C.c_int, [_vp, _vp, _vp, _i32, _vp, _vp]),
    "gj_weighted_backward": (C.c_int, [_vp, _vp, _vp, _vp]),
    "gj_free_wstate": (None, [_vp]),
    "gj_weighted_grad_noalloc": (C.c_int, [_vp, _vp, _vp, _i32, _vp, _vp, _vp]),
    "gj_batch_create": (C.c_int, [_vp, _i32, _vp, _vp, _vp, _vp, _vp]),
    "gj_batch_launch": (C.c_int, [_vp, _vp]),
    "gj_batch_launch_eager": (C.c_int, [_vp, _vp]),
    "gj_batch_launch_kernels": (C.c_int, [_vp, _vp]),
    "gj_batch_launch_persistent": (C.c_int, [_vp, _vp]),
    "gj_batch_info": (C.c_int, [_vp, _vp, _vp, _vp]),
    "gj_batch_join_sizes": (_vp, [_vp]),
    "gj_batch_status": (_vp, [_vp]),
    "gj_batch_summary": (C.c_int, [_vp, _i32, _vp]),
    "gj_free_batch": (None, [_vp]),
    "gj_download": (C.c_int, [_vp, _vp, _vp, _sz]),
    "gj_ctx_set_tune": (C.c_int, [_vp, _vp]),
    "gj_desum_launch_config": (C.c_int, [_i32, _i32, _i32, _i64, _vp, _vp]),
    "gj_desum_kernel": (C.c_int, [_vp, _vp, _vp]),
    "gj_colset_create": (C.c_int, [_vp, _vp, _i32, _vp, _vp, _vp]),
    "gj_free_colset": (None, [_vp]),
    "gj_desummarize_values": (C.c_int, [_vp, _vp, _vp, _i64, _i64, _vp, _vp]),
    "gj_summarize_projected": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "gj_summary_n_tables": (_i32, [_vp]),
    "gj_desummarize_projected": (C.c_int, [_vp, _vp, _i64, _i64, _vp, _vp]),
    "gj_summary_save": (C.c_int, [_vp, _vp, C.c_char_p, _i32, _vp]),
    "gj_summary_load": (C.c_int, [_vp, C.c_char_p, _vp]),
    "gj_summary_file_check": (C.c_int, [C.c_char_p, _vp]),
    "gj_junction_tree_build": (C.c_int, [_vp, _vp]),
    "gj_potential_join": (C.c_int, [_vp, _vp, _vp, _vp]),
    "gj_potential_table": (C.c_int, [_vp, _vp]),
    "gj_free_potential": (None, [_vp]),
    "gj_summarize_cyclic": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "gj_result_attribute": (_i32, [_vp, _i32]),
}


def load_library(path: str = LIB_PATH):
    """Load libgj.so (raises if it has not been built: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing; build it with `python -m paper_2206_10435_amd.build`")
    L = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(rc: int, ctx_h=None):
    """Raise GJError with the message the library recorded for context `ctx_h`
    (None: for the calling thread, the calls that take no context)."""
    if rc != GJ_OK:
        raise GJError(rc, load_library().gj_last_error(ctx_h).decode())


def _graph_struct(parent, sep_col, parent_col):
    n = len(parent)
    arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.int32)) for a in (parent, sep_col, parent_col)]
    return _Graph(n, *[a.ctypes.data for a in arrs]), arrs


def validate(n_rows: Sequence[int], n_keys: Sequence[int], parent, sep_col, parent_col) -> None:
    """Host-only graph validation (no device work); raises GJError."""
    L = load_library()
    keep = []
    tabs = (_Table * len(n_rows))()
    for t, (n, k) in enumerate(zip(n_rows, n_keys)):
        fake = (C.c_void_p * max(k, 1))(*([1] * max(k, 1)))  # non-null column placeholders
        keep.append(fake)
        tabs[t] = _Table(int(n), int(k), C.cast(fake, C.c_void_p))
    g, arrs = _graph_struct(parent, sep_col, parent_col)
    _check(L.gj_validate(tabs, C.byref(g)))


def desum_launch_config(n_tables: int, rowid_bytes: int, n_cols: int, n_rows: int,
                        tune: Optional[Tune] = None) -> dict:
    """Launch shape of the expansion kernel for these arguments (host only)."""
    L = load_library()
    out = DesumLaunch()
    _check(L.gj_desum_launch_config(int(n_tables), int(rowid_bytes), int(n_cols), int(n_rows),
                                    C.byref(tune) if tune is not None else None, C.byref(out)))
    return {k: int(getattr(out, k)) for k, _ in DesumLaunch._fields_}


def summary_file_check(path: str) -> dict:
    """Checks a stored summary file on the host (no device): raises GJError if
    it is unreadable, truncated or inconsistent, else returns its header."""
    L = load_library()
    info = SummaryFileInfo()
    _check(L.gj_summary_file_check(os.fsencode(path), C.byref(info)))
    n = info.n_tables
    return {"n_tables": n, "projected": bool(info.projected), "with_rows": bool(info.with_rows),
            "join_size": int(info.join_size), "entries": [int(info.entries[t]) for t in range(n)],
            "rows": [int(info.rows[t]) for t in range(n)], "bytes": int(info.bytes)}


def _natural_struct(attrs):
    n = len(attrs)
    nk = np.array([len(a) for a in attrs], dtype=np.int32)
    at = np.full(n * MAX_KEYS, -1, dtype=np.int32)
    for t, a in enumerate(attrs):
        at[t * MAX_KEYS: t * MAX_KEYS + len(a)] = a
    return _NatQuery(n, nk.ctypes.data, at.ctypes.data), (nk, at)


def junction_tree(attrs) -> dict:
    """Host-only junction tree of a natural-join query (attrs[t][c] = attribute
    id of column c of table t): attribute ids, elimination order, fill-in
    count, maxcliques (as sorted attribute-id lists), parents, table cliques."""
    L = load_library()
    q, keep = _natural_struct(attrs)
    jt = _JTree()
    _check(L.gj_junction_tree_build(C.byref(q), C.byref(jt)))
    ids = [jt.attr_id[i] for i in range(jt.n_attrs)]
    cl = [sorted(ids[i] for i in range(jt.n_attrs) if (jt.clique[c] >> i) & 1) for c in range(jt.n_cliques)]
    return dict(attr_ids=ids, elim_order=[ids[jt.elim_order[i]] for i in range(jt.n_attrs)],
                n_fill=int(jt.n_fill), cliques=cl, parent=[int(jt.parent[c]) for c in range(jt.n_cliques)],
                table_clique=[int(jt.table_clique[t]) for t in range(len(attrs))])


class Context:
    """A device, a stream and PyTorch's caching allocator."""

    def __init__(self, device: int = 0, stream=None, torch_allocator: bool = True, allocator=None):
        """`allocator`: optional (alloc(nbytes) -> device address or 0, free(address))
        Python callables used instead of PyTorch's caching allocator."""
        import torch

        self.torch = torch
        self.L = load_library()
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        sptr = self.stream.cuda_stream
        self._live = {}
        if allocator is not None:
            user_alloc, user_free = allocator

            def _alloc(nbytes, user):
                try:
                    return user_alloc(int(nbytes)) or None
                except Exception:
                    return None

            def _free(ptr, user):
                try:
                    user_free(ptr)
                except Exception:
                    pass

            self._alloc_cb = ALLOC_FN(_alloc)
            self._free_cb = FREE_FN(_free)
        elif torch_allocator:
            alloc_fn = torch.cuda.caching_allocator_alloc
            delete_fn = torch.cuda.caching_allocator_delete
            stream_ = self.stream

            def _alloc(nbytes, user):
                try:
                    return alloc_fn(int(nbytes), device, stream_)
                except Exception:
                    return None

            def _free(ptr, user):
                try:
                    delete_fn(ptr)
                except Exception:
                    pass  # interpreter shutdown: the process is releasing the device anyway

            self._alloc_cb = ALLOC_FN(_alloc)
            self._free_cb = FREE_FN(_free)
        else:
            self._alloc_cb = ALLOC_FN()
            self._free_cb = FREE_FN()
        h = C.c_void_p()
        _check(self.L.gj_ctx_create(device, C.c_void_p(sptr), self._alloc_cb, self._free_cb, None, C.byref(h)))
        self.h = h

    def _check(self, rc: int):
        _check(rc, self.h)

    def close(self):
        if getattr(self, "h", None):
            self.L.gj_ctx_destroy(self.h)
            self.h = None

    def set_tune(self, sort_items=8, radix_bits=8, desum_rounds=0, desum_stage=4, batch_task_rows=0,
                 desum_general=0, sort_local_rows=1 << 20):
        t = Tune(sort_items, radix_bits, desum_rounds, desum_stage, batch_task_rows, desum_general,
                 sort_local_rows)
        self._check(self.L.gj_ctx_set_tune(self.h, C.byref(t)))

    def desum_kernel(self, s: "Summary") -> str:
        """'unit' when desummarize takes the keyed-lookup expansion for s, else 'general'."""
        k = C.c_int32(-1)
        self._check(self.L.gj_desum_kernel(self.h, s.h, C.byref(k)))
        return "unit" if k.value == 1 else "general"

    def download(self, ptr: int, n: int, dtype) -> np.ndarray:
        out = np.empty(max(n, 0), dtype=dtype)
        if n > 0:
            self._check(self.L.gj_download(self.h, out.ctypes.data_as(C.c_void_p), C.c_void_p(ptr), out.nbytes))
        return out

    # -- stage 1 ------------------------------------------------------------
    def build_factors(self, tables: List[List["torch.Tensor"]], parent, sep_col, parent_col) -> "Factors":
        tabs, keep = _tables_struct(tables)
        g, arrs = _graph_struct(parent, sep_col, parent_col)
        h = C.c_void_p()
        self._check(self.L.gj_build_factors(self.h, tabs, C.byref(g), C.byref(h)))
        return Factors(self, h, len(tables))

    # -- stage 2 ------------------------------------------------------------
    def summarize(self, f: "Factors") -> "Summary":
        h = C.c_void_p()
        q = C.c_int64()
        self._check(self.L.gj_summarize(self.h, f.h, C.byref(h), C.byref(q)))
        return Summary(self, h, f.n_tables, int(q.value))

    def summarize_batch(self, factors: List["Factors"], d_join_sizes, d_status,
                        outs: Optional[List["Summary"]] = None) -> List["Summary"]:
        """Summaries of several factor sets without reading anything back:
        join sizes / statuses go to the int64 / int32 device tensors given.
        Passing the summaries of an earlier call recomputes them in place
        (nothing allocated: capturable in a HIP graph)."""
        import torch

        n = len(factors)
        if d_join_sizes.dtype != torch.int64 or d_status.dtype != torch.int32 or \
                d_join_sizes.numel() < n or d_status.numel() < n:
            raise ValueError("need int64 join-size and int32 status device tensors of n_queries entries")
        fp = (C.c_void_p * max(n, 1))(*[f.h for f in factors])
        op = (C.c_void_p * max(n, 1))(*([s.h for s in outs] if outs is not None else [None] * n))
        self._check(self.L.gj_summarize_batch(self.h, fp, n, op, C.c_void_p(d_join_sizes.data_ptr()),
                                              C.c_void_p(d_status.data_ptr())))
        if outs is not None:
            for s in outs:
                s.refresh()
            return outs
        return [Summary(self, C.c_void_p(op[i]), f.n_tables, None) for i, f in enumerate(factors)]

    def summarize_projected(self, f: "Factors", out_cols) -> "Summary":
        """Early projection: out_cols[t] has bit c set for every output key
        column c of table t.  The summary's tables are the kept tables."""
        m = np.ascontiguousarray([int(x) for x in out_cols], dtype=np.uint32)
        if len(m) != f.n_tables:
            raise ValueError("one mask word per table")
        h = C.c_void_p()
        q = C.c_int64()
        self._check(self.L.gj_summarize_projected(self.h, f.h, m.ctypes.data_as(C.c_void_p), C.byref(h), C.byref(q)))
        return Summary(self, h, int(self.L.gj_summary_n_tables(h)), int(q.value), projected=True)

    def save(self, s: "Summary", path: str, with_rows: bool = True) -> int:
        """Writes the summary to `path`; returns the file size in bytes."""
        nb = C.c_int64()
        self._check(self.L.gj_summary_save(self.h, s.h, os.fsencode(path), 1 if with_rows else 0, C.byref(nb)))
        return int(nb.value)

    def load(self, path: str) -> "Summary":
        h = C.c_void_p()
        self._check(self.L.gj_summary_load(self.h, os.fsencode(path), C.byref(h)))
        js = int(self.L.gj_summary_join_size(h))
        return Summary(self, h, int(self.L.gj_summary_n_tables(h)), js)

    def result_columns(self, s: "Summary") -> int:
        return int(self.L.gj_result_columns(s.h))

    def desummarize_projected(self, s: "Summary", first_row: int, n_rows: int, out) -> int:
        """Writes rows [first_row, first_row + n_rows) as attribute values
        (n_rows x result_columns, row-major int32) into `out`; returns the count."""
        import torch

        nc = self.result_columns(s)
        if out.dtype != torch.int32 or not out.is_contiguous():
            raise ValueError("out must be a contiguous int32 device tensor")
        if out.numel() < n_rows * nc:
            raise ValueError("out is too small")
        nw = C.c_int64()
        self._check(self.L.gj_desummarize_projected(self.h, s.h, int(first_row), int(n_rows),
                                               C.c_void_p(out.data_ptr()), C.byref(nw)))
        return int(nw.value)

    # -- cyclic queries ------------------------------------------------------
    def potential_join(self, tables, attrs) -> dict:
        """Algorithm 1: joint potential of the tables (lists of int32 device
        columns; attrs[t][c] = attribute id) over all their attributes."""
        tabs, keep = _tables_struct(tables)
        q, keep2 = _natural_struct(attrs)
        h = C.c_void_p()
        self._check(self.L.gj_potential_join(self.h, tabs, C.byref(q), C.byref(h)))
        try:
            v = _PotView()
            self._check(self.L.gj_potential_table(h, C.byref(v)))
            n, nv = int(v.n_entries), int(v.n_vars)
            keys = (np.stack([self.download(v.keys[i], n, np.int32) for i in range(nv)], axis=1)
                    if nv else np.zeros((n, 0), np.int32))
            return dict(attrs=[int(v.attr[i]) for i in range(nv)], keys=keys, freq=self.download(v.freq, n, np.int64))
        finally:
            self.L.gj_free_potential(h)

    def summarize_cyclic(self, tables, attrs) -> "Summary":
        """Summary of a natural-join query over named attributes (cycles
        allowed): tables are lists of int32 device columns, attrs[t][c] the
        attribute id of column c of table t.  Expand it with
        desummarize_projected; result_attributes names its columns."""
        tabs, keep = _tables_struct(tables)
        q, keep2 = _natural_struct(attrs)
        h = C.c_void_p()
        js = C.c_int64()
        self._check(self.L.gj_summarize_cyclic(self.h, tabs, C.byref(q), C.byref(h), C.byref(js)))
        return Summary(self, h, int(self.L.gj_summary_n_tables(h)), int(js.value), projected=True)

    def result_attributes(self, s: "Summary"):
        return [int(self.L.gj_result_attribute(s.h, j)) for j in range(self.result_columns(s))]

    # -- stage 3 ------------------------------------------------------------
    def desummarize(self, s: "Summary", first_row: int, n_rows: int, out) -> int:
        """Writes rows [first_row, first_row + n_rows) into `out` (int32 or int64
        device tensor of at least n_rows * n_tables elements); returns the count."""
        import torch

        if out.dtype not in (torch.int32, torch.int64) or not out.is_contiguous():
            raise ValueError("out must be a contiguous int32/int64 device tensor")
        if out.numel() < n_rows * s.n_tables:
            raise ValueError("out is too small")
        nw = C.c_int64()
        self._check(self.L.gj_desummarize(self.h, s.h, int(first_row), int(n_rows), out.element_size(),
                                     C.c_void_p(out.data_ptr()), C.byref(nw)))
        return int(nw.value)

    def colset(self, s: "Summary", columns) -> "ColSet":
        """Value columns for gj_desummarize_values: `columns` is a list of
        (table, int32 device tensor with one value per row of that table)."""
        tabs = np.array([int(t) for t, _ in columns], dtype=np.int32)
        for t, c in columns:
            if str(c.dtype) != "torch.int32" or not c.is_contiguous() or not c.is_cuda:
                raise ValueError("value columns must be contiguous int32 device tensors")
        ptrs = (C.c_void_p * len(columns))(*[c.data_ptr() for _, c in columns])
        h = C.c_void_p()
        self._check(self.L.gj_colset_create(self.h, s.h, len(columns), tabs.ctypes.data_as(C.c_void_p), ptrs,
                                       C.byref(h)))
        return ColSet(self, h, len(columns))

    def desummarize_values(self, s: "Summary", cs: "ColSet", first_row: int, n_rows: int, out) -> int:
        """Writes rows [first_row, first_row + n_rows) as int32 values
        (n_rows x cs.n_cols, row-major) into `out`; returns the count."""
        import torch

        if out.dtype != torch.int32 or not out.is_contiguous():
            raise ValueError("out must be a contiguous int32 device tensor")
        if out.numel() < n_rows * cs.n_cols:
            raise ValueError("out is too small")
        nw = C.c_int64()
        self._check(self.L.gj_desummarize_values(self.h, s.h, cs.h, int(first_row), int(n_rows),
                                            C.c_void_p(out.data_ptr()), C.byref(nw)))
        return int(nw.value)

    def unroll_gfjs(self, s: "Summary", first_row: int, n_rows: int):
        """Paper-literal GFJS of a row range: list of (values, freqs) numpy pairs per result column."""
        import torch

        L = int(self.L.gj_result_columns(s.h))
        vals = [torch.empty(max(n_rows, 1), dtype=torch.int32, device=f"cuda:{self.device}") for _ in range(L)]
        frqs = [torch.empty(max(n_rows, 1), dtype=torch.int64, device=f"cuda:{self.device}") for _ in range(L)]
        vp = (C.c_void_p * L)(*[v.data_ptr() for v in vals])
        fp = (C.c_void_p * L)(*[f.data_ptr() for f in frqs])
        nr = (C.c_int64 * L)()
        self._check(self.L.gj_unroll_gfjs(self.h, s.h, int(first_row), int(n_rows), vp, fp, nr))
        return [(vals[i][: nr[i]].cpu().numpy(), frqs[i][: nr[i]].cpu().numpy()) for i in range(L)]

    # -- weighted ------------------------------------------------------------
    def weighted_forward(self, f: "Factors", weights: List["torch.Tensor"]):
        import torch

        dt = weights[0].dtype
        if dt not in (torch.float32, torch.float64) or any(w.dtype != dt for w in weights):
            raise ValueError("weights must all be float32 or all float64")
        wp = (C.c_void_p * len(weights))(*[w.data_ptr() for w in weights])
        W = torch.empty((), dtype=torch.float64, device=f"cuda:{self.device}")
        st = C.c_void_p()
        self._check(self.L.gj_weighted_forward(self.h, f.h, wp, 1 if dt == torch.float64 else 0,
                                          C.c_void_p(W.data_ptr()), C.byref(st)))
        return W, WState(self, st)

    def weighted_backward(self, st: "WState", gradW, grads: List["torch.Tensor"]):
        gp = (C.c_void_p * len(grads))(*[g.data_ptr() for g in grads])
        self._check(self.L.gj_weighted_backward(self.h, st.h, C.c_void_p(gradW.data_ptr()), gp))

    def weighted_grad_noalloc(self, f: "Factors", weights, W, grads, gradW=None):
        """W into the float64 device scalar `W` and dW/dw into `grads` (one
        tensor per table, the weights' dtype) in one call that allocates
        nothing (the library's fixed scratch array); gradW: optional float64
        device scalar scaling the gradients."""
        import torch

        dt = weights[0].dtype
        if dt not in (torch.float32, torch.float64) or any(w.dtype != dt for w in weights) or \
                any(g.dtype != dt for g in grads) or W.dtype != torch.float64:
            raise ValueError("weights and gradients of one float dtype, W float64")
        wp = (C.c_void_p * len(weights))(*[w.data_ptr() for w in weights])
        gp = (C.c_void_p * len(grads))(*[g.data_ptr() for g in grads])
        self._check(self.L.gj_weighted_grad_noalloc(self.h, f.h, wp, 1 if dt == torch.float64 else 0,
                                                    C.c_void_p(gradW.data_ptr()) if gradW is not None else None,
                                                    C.c_void_p(W.data_ptr()), gp))

    # -- batch ---------------------------------------------------------------
    def batch_create(self, queries: List[dict], tune: Optional[Tune] = None) -> "Batch":
        """queries: dicts with 'tables' (list of lists of int32 device tensors), 'parent',
        'sep_col', 'parent_col'."""
        tabs_all, keep = [], []
        qoff = [0]
        graphs = (_Graph * len(queries))()
        for qi, q in enumerate(queries):
            tabs_all.extend(q["tables"])
            qoff.append(qoff[-1] + len(q["tables"]))
            g, arrs = _graph_struct(q["parent"], q["sep_col"], q["parent_col"])
            keep.append(arrs)
            graphs[qi] = g
        tabs, keep2 = _tables_struct(tabs_all)
        qo = np.array(qoff, dtype=np.int32)
        h = C.c_void_p()
        self._check(self.L.gj_batch_create(self.h, len(queries), qo.ctypes.data_as(C.c_void_p), tabs, graphs,
                                      C.byref(tune) if tune is not None else None, C.byref(h)))
        return Batch(self, h, [len(q["tables"]) for q in queries], keep=(keep, keep2, queries))


def _tables_struct(tables):
    tabs = (_Table * len(tables))()
    keep = []
    for t, cols in enumerate(tables):
        for c in cols:
            if c.dtype.__str__() != "torch.int32" or not c.is_contiguous() or not c.is_cuda:
                raise ValueError("key columns must be contiguous int32 device tensors")
        ptrs = (C.c_void_p * max(len(cols), 1))(*[c.data_ptr() for c in cols])
        keep.append(ptrs)
        n = int(cols[0].numel()) if cols else 0
        tabs[t] = _Table(n, len(cols), C.cast(ptrs, C.c_void_p))
    return tabs, keep


class Factors:
    def __init__(self, ctx: Context, h, n_tables: int):
        self.ctx, self.h, self.n_tables = ctx, h, n_tables

    def __del__(self):
        if getattr(self, "h", None) is not None and self.ctx.h:
            self.ctx.L.gj_free_factors(self.h)
            self.h = None

    def table(self, t: int) -> dict:
        v = _FactorView()
        self.ctx._check(self.ctx.L.gj_factor_table(self.h, t, C.byref(v)))
        M, N, k = int(v.n_entries), int(v.n_rows), int(v.n_keys)
        d = self.ctx.download
        keys = np.stack([d(v.keys[c], M, np.int32) for c in range(k)], axis=1) if k else np.zeros((M, 0), np.int32)
        return dict(keys=keys, start=d(v.start, M, np.int32), end=d(v.end, M, np.int32),
                    count=d(v.count, M, np.int64), perm=d(v.perm, N, np.int32))

    def sort_kind(self, t: int) -> str:
        """How table t was sorted: 'digits' (a global pass per digit), 'buckets'
        (top-digit passes, then an LDS sort of each bucket) or 'buckets_redone'
        (a bucket too long for one block: sorted again by the per-digit passes)."""
        k = C.c_int32(-1)
        self.ctx._check(self.ctx.L.gj_factor_sort(self.h, t, C.byref(k)))
        return ("digits", "buckets", "buckets_redone")[k.value]


class Summary:
    def __init__(self, ctx: Context, h, n_tables: int, join_size: Optional[int], borrowed: bool = False,
                 projected: bool = False):
        self.ctx, self.h, self.n_tables, self._join_size, self.borrowed = ctx, h, n_tables, join_size, borrowed
        self.projected = projected

    @property
    def join_size(self) -> int:
        """The join size (read from the device on first use for a summary made
        by summarize_batch; GJError GJ_E_OVERFLOW if its query overflowed)."""
        if self._join_size is None:
            js = int(self.ctx.L.gj_summary_join_size(self.h))
            if js < 0:
                raise GJError(GJ_E_OVERFLOW, self.ctx.L.gj_last_error(self.ctx.h).decode())
            self._join_size = js
        return self._join_size

    def refresh(self):
        """Forget the cached join size (after the summary was recomputed in place)."""
        self._join_size = None

    def __del__(self):
        if not self.borrowed and getattr(self, "h", None) is not None and self.ctx.h:
            self.ctx.L.gj_free_summary(self.h)
            self.h = None

    def table(self, t: int) -> dict:
        v = _SummaryView()
        self.ctx._check(self.ctx.L.gj_summary_table(self.h, t, C.byref(v)))
        M, k = int(v.n_entries), int(v.n_keys)
        d = self.ctx.download
        keys = np.stack([d(v.keys[c], M, np.int32) for c in range(k)], axis=1)
        return dict(keys=keys, c=d(v.c, M, np.int64), U=d(v.U, M, np.int64), D=d(v.D, M, np.int64),
                    F=d(v.F, M, np.int64), pre=d(v.pre, M, np.int64))

    def edge(self, t: int) -> dict:
        v = _EdgeView()
        self.ctx._check(self.ctx.L.gj_summary_edge(self.h, t, C.byref(v)))
        n = int(v.n)
        d = self.ctx.download
        return dict(s=d(v.s, n, np.int32), M=d(v.M, n, np.int64), D=d(v.D, n, np.int64))


class ColSet:
    def __init__(self, ctx: Context, h, n_cols: int):
        self.ctx, self.h, self.n_cols = ctx, h, n_cols

    def __del__(self):
        if getattr(self, "h", None) is not None and self.ctx.h:
            self.ctx.L.gj_free_colset(self.h)
            self.h = None


class WState:
    def __init__(self, ctx: Context, h):
        self.ctx, self.h = ctx, h

    def __del__(self):
        if getattr(self, "h", None) is not None and self.ctx.h:
            self.ctx.L.gj_free_wstate(self.h)
            self.h = None


class Batch:
    def __init__(self, ctx: Context, h, n_tables: List[int], keep=None):
        self.ctx, self.h, self.n_tables, self._keep = ctx, h, n_tables, keep

    def __del__(self):
        if getattr(self, "h", None) is not None and self.ctx.h:
            self.ctx.L.gj_free_batch(self.h)
            self.h = None

    def launch(self, graph: bool = True, stream=None, mode: Optional[str] = None):
        """mode 'kernels' (the recorded launch-per-stage graph, default),
        'eager' (those launches unrecorded; graph=False) or 'persistent'
        (the one-kernel launch, switched off: raises GJError)."""
        sp = C.c_void_p(stream.cuda_stream) if stream is not None else None
        mode = mode or ("kernels" if graph else "eager")
        fn = {"persistent": self.ctx.L.gj_batch_launch_persistent, "kernels": self.ctx.L.gj_batch_launch,
              "eager": self.ctx.L.gj_batch_launch_eager}[mode]
        self.ctx._check(fn(self.h, sp))

    def info(self) -> dict:
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        self.ctx._check(self.ctx.L.gj_batch_info(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return dict(tasks=a.value, stages=b.value, grid=c.value)

    def results(self):
        nq = len(self.n_tables)
        js = self.ctx.download(self.ctx.L.gj_batch_join_sizes(self.h), nq, np.int64)
        st = self.ctx.download(self.ctx.L.gj_batch_status(self.h), nq, np.int32)
        return js, st

    def summary(self, q: int) -> Summary:
        h = C.c_void_p()
        self.ctx._check(self.ctx.L.gj_batch_summary(self.h, q, C.byref(h)))
        js = int(self.ctx.L.gj_summary_join_size(h))
        return Summary(self.ctx, h, self.n_tables[q], js, borrowed=True)


class WeightedJoinSize:
    """torch.autograd.Function: W = sum over result tuples of the product of row
    weights; backward runs the library's adjoint (downward) kernel."""

    _fn = None

    @classmethod
    def apply(cls, ctx: Context, factors: Factors, *weights):
        if cls._fn is None:
            import torch

            class _F(torch.autograd.Function):
                @staticmethod
                def forward(fctx, gctx, fac, *ws):
                    W, st = gctx.weighted_forward(fac, list(ws))
                    fctx.gctx, fctx.st = gctx, st
                    fctx.shapes = [(w.shape, w.dtype) for w in ws]
                    return W

                @staticmethod
                def backward(fctx, gW):
                    grads = [torch.empty(s, dtype=dt, device=gW.device) for s, dt in fctx.shapes]
                    gW64 = gW.detach().to(torch.float64).contiguous()
                    fctx.gctx.weighted_backward(fctx.st, gW64, grads)
                    return (None, None, *grads)

            cls._fn = _F
        return cls._fn.apply(ctx, factors, *weights)


def to_device_tables(q, device: int = 0):
    """Upload a workloads.Query's key columns as int32 device tensors."""
    import torch

    return [[torch.from_numpy(np.ascontiguousarray(c)).to(f"cuda:{device}") for c in tb] for tb in q.tables]
