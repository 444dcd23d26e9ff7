"""The C ABI's contracts on the GPU: the factor view's count column, error
messages kept per context, summaries of several factor sets with nothing read
back (eagerly and recorded into a HIP graph, checked on every replay against
the oracle), allocation failures reported as GJ_E_OOM without leaking,
batch launches on another stream ordered before reads on the context's
stream, and the autotuner's choices and cache."""
import ctypes as C
import json
import os

import numpy as np
import pytest

from conftest import load_fig1
from paper_2206_10435_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _queries():
    return [load_fig1(), W.cfg1()] + [W.random_tree_query(900 + i, 2 + i % 4, 3000, 400, s=0.8, max_extra_cols=2,
                                                         min_rows=1000) for i in range(4)]


def test_factor_view_count_column(oracle_mod):
    from paper_2206_10435_amd import gj

    ctx = gj.Context(0)
    for q in _queries()[:3]:
        f = ctx.build_factors(gj.to_device_tables(q), q.parent, q.sep_col, q.parent_col)
        o = oracle_mod.Oracle(q)
        for t in range(q.n_tables):
            g, r = f.table(t), o.factor(t)
            assert g["count"].dtype == np.int64
            assert np.array_equal(g["count"], (g["end"] - g["start"]).astype(np.int64))
            assert np.array_equal(g["count"], r["count"])


def test_error_messages_per_context():
    import torch

    from paper_2206_10435_amd import gj

    L = gj.load_library()
    c1, c2 = gj.Context(0), gj.Context(0)
    q = W.cfg1()
    s = c1.summarize(c1.build_factors(gj.to_device_tables(q), q.parent, q.sep_col, q.parent_col))
    out = torch.empty(30, dtype=torch.int32, device="cuda:0")
    with pytest.raises(gj.GJError) as ei:
        c1.desummarize(s, s.join_size + 1, 10, out)
    assert ei.value.status == gj.GJ_E_RANGE
    assert b"beyond the join size" in L.gj_last_error(c1.h)
    assert L.gj_last_error(c2.h) == b""
    # a call without a context records on the thread only
    with pytest.raises(gj.GJError):
        gj.validate([5, 5], [2, 2], [-1, 1], [0, 0], [0, 1])
    assert b"parent" in L.gj_last_error(None)
    assert b"beyond the join size" in L.gj_last_error(c1.h)
    # objects made by a context record on it
    with pytest.raises(gj.GJError):
        s.edge(0)
    assert b"gj_summary_edge" in L.gj_last_error(c1.h)
    assert L.gj_last_error(c2.h) == b""


def _check_summaries(sums, qs, oracles, js, st):
    from paper_2206_10435_amd import gj

    for i, (s, q, o) in enumerate(zip(sums, qs, oracles)):
        Q, ovf = o.join_size()
        assert not ovf
        assert int(js[i]) == Q and int(st[i]) == gj.GJ_OK, i
        assert s.join_size == Q
        for t in range(q.n_tables):
            g, r = s.table(t), o.summary_table(t)
            for k in ("keys", "c", "U", "D", "F"):
                assert np.array_equal(g[k], r[k]), (i, t, k)
            if t:
                ge, re_ = s.edge(t), o.summary_edge(t)
                for k in ("s", "M", "D"):
                    assert np.array_equal(ge[k], re_[k]), (i, t, k)


def test_summarize_batch_eager_in_place_and_graph(oracle_mod):
    """Several factor sets summarized with nothing read back; the same
    summaries recomputed in place; the in-place call recorded into a HIP graph
    and replayed three times, with eager work in between, each replay checked
    against the oracle."""
    import torch

    from paper_2206_10435_amd import gj

    side = torch.cuda.Stream()
    ctx = gj.Context(0, stream=side)
    qs = _queries()
    oracles = [oracle_mod.Oracle(q) for q in qs]
    with torch.cuda.stream(side):
        fs = [ctx.build_factors(gj.to_device_tables(q), q.parent, q.sep_col, q.parent_col) for q in qs]
        js = torch.full((len(qs),), -1, dtype=torch.int64, device="cuda:0")
        st = torch.full((len(qs),), -1, dtype=torch.int32, device="cuda:0")
    sums = ctx.summarize_batch(fs, js, st)
    side.synchronize()
    _check_summaries(sums, qs, oracles, js.cpu().numpy(), st.cpu().numpy())
    _say("summarize_batch: eager ok")
    # in place
    with torch.cuda.stream(side):
        js.fill_(-1)
        st.fill_(-1)
    ctx.summarize_batch(fs, js, st, outs=sums)
    side.synchronize()
    _check_summaries(sums, qs, oracles, js.cpu().numpy(), st.cpu().numpy())
    _say("summarize_batch: in place ok")
    # recorded into a graph: nothing allocated, nothing read back
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        ctx.summarize_batch(fs, js, st, outs=sums)
    for rep in range(3):
        with torch.cuda.stream(side):
            js.fill_(-1)
            st.fill_(-1)
            junk = torch.randn(1 << 20, device="cuda:0").sum()  # eager work between replays
        side.synchronize()
        g.replay()
        side.synchronize()
        for s in sums:
            s.refresh()
        _check_summaries(sums, qs, oracles, js.cpu().numpy(), st.cpu().numpy())
        _say(f"summarize_batch: graph replay {rep} ok")
        del junk
    # and bad arguments are refused before anything runs
    with pytest.raises(gj.GJError) as ei:
        ctx.summarize_batch([fs[0], fs[0]], js, st)
    assert ei.value.status == gj.GJ_E_INVALID
    with pytest.raises(gj.GJError) as ei:
        ctx.summarize_batch(fs[:2], js, st, outs=[sums[1], sums[0]])
    assert ei.value.status == gj.GJ_E_INVALID


def test_allocation_failure_reports_oom_and_frees():
    """An allocator that fails after k allocations: the build or summary
    reports GJ_E_OOM, every block it obtained is returned, and the context
    works afterwards."""
    import torch

    from paper_2206_10435_amd import gj

    state = {"limit": 0, "n": 0, "live": set()}
    stream = torch.cuda.current_stream()

    def alloc(nbytes):
        state["n"] += 1
        if state["n"] > state["limit"]:
            return 0
        p = torch.cuda.caching_allocator_alloc(nbytes, 0, stream)
        state["live"].add(p)
        return p

    def free(p):
        state["live"].discard(p)
        torch.cuda.caching_allocator_delete(p)

    ctx = gj.Context(0, allocator=(alloc, free))
    q = W.cfg1()
    tabs = gj.to_device_tables(q)
    import gc

    seen = set()
    for limit in (0, 1, 5, 12, 20, 30, 40, 60):
        state.update(limit=limit, n=0)
        f = s = None
        try:
            f = ctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col)
            s = ctx.summarize(f)
            seen.add("ok")
        except gj.GJError as e:
            assert e.status == gj.GJ_E_OOM, (limit, e)
            assert b"allocation" in gj.load_library().gj_last_error(ctx.h)
            seen.add("oom")
        f = s = None
        gc.collect()
        assert not state["live"], (limit, len(state["live"]))
    assert seen == {"ok", "oom"}
    state.update(limit=10**9, n=0)
    s = ctx.summarize(ctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col))
    from oracle import oracle as O

    assert s.join_size == O.Oracle(q).join_size()[0]


def test_batch_launch_on_another_stream_orders_reads():
    import torch

    from paper_2206_10435_amd import gj

    ctx = gj.Context(0)
    qs = [W.cfg5_query(i) for i in range(8)]
    qd = [dict(tables=gj.to_device_tables(q), parent=q.parent, sep_col=q.sep_col, parent_col=q.parent_col)
          for q in qs]
    b = ctx.batch_create(qd)
    b.launch(graph=True)
    ref = b.results()
    other = torch.cuda.Stream()
    for graph in (True, False):
        for _ in range(3):
            b.launch(graph=graph, stream=other)
            js, st = b.results()  # read on the context's stream, no host synchronization in between
            assert np.array_equal(js, ref[0]) and np.array_equal(st, ref[1])


def test_autotuner_chooses_caches_and_keeps_results(tmp_path, monkeypatch):
    import torch

    from paper_2206_10435_amd import autotune, gj

    cache = tmp_path / "tune.json"
    monkeypatch.setenv("GJ_TUNE_CACHE", str(cache))
    ctx = gj.Context(0)
    q = W.cfg1()
    tabs = gj.to_device_tables(q)
    s = ctx.summarize(ctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col))
    n = s.join_size
    ref = torch.empty(n * 3, dtype=torch.int64, device="cuda:0")
    ctx.desummarize(s, 0, n, ref)
    out = torch.empty_like(ref)
    dt = autotune.tune_desummarize(ctx, s, out, 0, n)
    assert dt["desum_stage"] in autotune.DESUM_STAGE and dt["desum_rounds"] in autotune.DESUM_ROUNDS
    assert len(dt["trials"]) == len(autotune.DESUM_STAGE) * len(autotune.DESUM_ROUNDS)
    ft = autotune.tune_factors(ctx, tabs, q.parent, q.sep_col, q.parent_col)
    assert ft["sort_items"] in autotune.SORT_ITEMS and ft["radix_bits"] in autotune.RADIX_BITS
    applied = autotune.apply(ctx, ft, dt)
    s2 = ctx.summarize(ctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col))
    out.fill_(-1)
    ctx.desummarize(s2, 0, n, out)
    assert torch.equal(out, ref), applied
    ctx.set_tune()
    qs = [W.cfg5_query(i) for i in range(12)]
    qd = [dict(tables=gj.to_device_tables(x), parent=x.parent, sep_col=x.sep_col, parent_col=x.parent_col)
          for x in qs]
    base = ctx.batch_create(qd)
    base.launch()
    rj, rs = base.results()
    tb = autotune.tune_batch(ctx, qd, reps=1)
    tb["batch"].launch()
    tj, ts = tb["batch"].results()
    assert np.array_equal(tj, rj) and np.array_equal(ts, rs)
    rec = json.loads(cache.read_text())
    kinds = {k.split("|")[1] for k in rec}
    assert kinds == {"desum", "factors", "batch"}, kinds
    # a second call reads the cache instead of measuring
    again = autotune.tune_batch(ctx, qd)
    assert (again["sort_items"], again["radix_bits"]) == (tb["sort_items"], tb["radix_bits"])
