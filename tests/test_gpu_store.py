"""Storing and reloading summaries (gj_summary_save / gj_summary_load): a
reloaded summary gives the same views, materialized tuples, values, paper GFJS
and projected rows as the summary it was saved from (and so as the oracle);
damaged files are refused."""
import os

import numpy as np
import pytest

from conftest import load_fig1
from paper_2206_10435_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gctx():
    from paper_2206_10435_amd import gj

    return gj.Context(0)


def _say(*a):
    print(*a, flush=True)


def _views(s):
    out = []
    for t in range(s.n_tables):
        out.append(s.table(t))
        if t > 0:
            out.append(s.edge(t))
    return out


def _same_views(a, b):
    va, vb = _views(a), _views(b)
    assert len(va) == len(vb)
    for x, y in zip(va, vb):
        assert x.keys() == y.keys()
        for k in x:
            assert np.array_equal(x[k], y[k]), k


def _rows(gctx, s, n, first, count):
    import torch

    out = torch.full((max(count, 1) * n,), -1, dtype=torch.int64, device="cuda:0")
    nw = gctx.desummarize(s, first, count, out)
    return out[: nw * n].view(nw, n).cpu().numpy()


def _vals(gctx, s, first, count):
    import torch

    nc = gctx.result_columns(s)
    out = torch.full((max(count, 1) * nc,), -1, dtype=torch.int32, device="cuda:0")
    nw = gctx.desummarize_projected(s, first, count, out)
    return out[: nw * nc].view(nw, nc).cpu().numpy()


def _queries():
    return [load_fig1(), W.cfg1()] + [W.random_tree_query(900 + i, 2 + i, 150, 20, s=0.7, min_rows=20)
                                      for i in range(5)]


@pytest.mark.parametrize("qi", range(7))
def test_roundtrip_with_rows(gctx, oracle_mod, tmp_path, qi):
    from paper_2206_10435_amd import gj

    q = _queries()[qi]
    o = oracle_mod.Oracle(q)
    tabs = gj.to_device_tables(q)
    s = gctx.summarize(gctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col))
    path = str(tmp_path / f"{q.name}.gjs")
    nb = gctx.save(s, path, with_rows=True)
    assert nb == os.path.getsize(path)
    # the host-only check reads the same file back: header, entry and row counts
    info = gj.summary_file_check(path)
    assert info["bytes"] == nb and info["n_tables"] == q.n_tables and info["with_rows"]
    assert info["join_size"] == s.join_size and not info["projected"]
    assert info["entries"] == [len(s.table(t)["c"]) for t in range(q.n_tables)]
    assert info["rows"] == [q.n_rows(t) for t in range(q.n_tables)]
    r = gctx.load(path)
    _say("case store", q.name, "bytes", nb, "Q", s.join_size)
    assert r.join_size == s.join_size == o.join_size()[0] and r.n_tables == q.n_tables
    _same_views(s, r)
    Q, n = s.join_size, q.n_tables
    ref = o.canonical_result()
    assert np.array_equal(_rows(gctx, r, n, 0, Q), ref)
    if Q > 3:
        assert np.array_equal(_rows(gctx, r, n, Q // 3, Q // 2), ref[Q // 3: Q // 3 + Q // 2])
    assert np.array_equal(_vals(gctx, r, 0, Q), _vals(gctx, s, 0, Q))
    cols = [(t, tabs[t][-1]) for t in range(n)]
    cs, cr = gctx.colset(s, cols), gctx.colset(r, cols)
    import torch

    a = torch.empty(max(Q, 1) * n, dtype=torch.int32, device="cuda:0")
    b = torch.empty(max(Q, 1) * n, dtype=torch.int32, device="cuda:0")
    assert gctx.desummarize_values(s, cs, 0, Q, a) == gctx.desummarize_values(r, cr, 0, Q, b) == Q
    assert torch.equal(a, b)
    if Q <= 200_000:
        ga, gb = gctx.unroll_gfjs(s, 0, Q), gctx.unroll_gfjs(r, 0, Q)
        assert all(np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1]) for x, y in zip(ga, gb))


def test_roundtrip_without_rows_and_projected(gctx, oracle_mod, tmp_path):
    from paper_2206_10435_amd import gj

    q = W.cfg1()
    o = oracle_mod.Oracle(q)
    tabs = gj.to_device_tables(q)
    f = gctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col)
    s = gctx.summarize(f)
    p_full = str(tmp_path / "full.gjs")
    n_small = gctx.save(s, p_full, with_rows=False)
    n_big = gctx.save(s, str(tmp_path / "rows.gjs"), with_rows=True)
    assert n_small < n_big
    r = gctx.load(p_full)
    _same_views(s, r)
    Q = s.join_size
    assert np.array_equal(_vals(gctx, r, 0, Q), _vals(gctx, s, 0, Q))
    out = __import__("torch").empty(64, dtype=__import__("torch").int64, device="cuda:0")
    with pytest.raises(gj.GJError) as ei:
        gctx.desummarize(r, 0, 4, out)
    assert ei.value.status == gj.GJ_E_INVALID
    # projected summary: stored without rows only
    mask = [3, 2, 0]
    ps = gctx.summarize_projected(f, mask)
    with pytest.raises(gj.GJError):
        gctx.save(ps, str(tmp_path / "bad.gjs"), with_rows=True)
    pp = str(tmp_path / "proj.gjs")
    gctx.save(ps, pp, with_rows=False)
    info = gj.summary_file_check(pp)
    assert info["projected"] and not info["with_rows"] and info["n_tables"] == 2
    pr = gctx.load(pp)
    assert pr.n_tables == ps.n_tables == 2
    _same_views(ps, pr)
    assert np.array_equal(_vals(gctx, pr, 0, Q), o.projected_result(mask))


def test_damaged_files_refused(gctx, tmp_path):
    from paper_2206_10435_amd import gj

    q = load_fig1()
    tabs = gj.to_device_tables(q)
    s = gctx.summarize(gctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col))
    path = str(tmp_path / "fig1.gjs")
    gctx.save(s, path, with_rows=True)
    data = open(path, "rb").read()
    cases = {
        "truncated": data[: len(data) // 2],
        "magic": b"X" + data[1:],
        # the last table's last row id beyond the table
        "row id": data[:-4] + np.array([1 << 30], dtype=np.int32).tobytes(),
    }
    cases["trailing"] = data + b"\0"
    for name, blob in cases.items():
        p = str(tmp_path / f"{name}.gjs")
        open(p, "wb").write(blob)
        with pytest.raises(gj.GJError) as ei:
            gctx.load(p)
        assert ei.value.status == gj.GJ_E_INVALID, name
        with pytest.raises(gj.GJError) as ei:
            gj.summary_file_check(p)
        assert ei.value.status == gj.GJ_E_INVALID, name
    with pytest.raises(gj.GJError):
        gctx.load(str(tmp_path / "missing.gjs"))
