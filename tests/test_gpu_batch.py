"""Many queries in one plan recorded as a HIP graph of one launch per stage:
every query's join size, status and summary against the oracle; replays of
the graph agree with each other and with the same kernels launched one by
one.  The persistent one-kernel form is switched off and refuses to launch."""
import numpy as np
import pytest

from paper_2206_10435_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gctx():
    from paper_2206_10435_amd import gj

    return gj.Context(0)


def _say(*a):
    print(*a, flush=True)


def _queries(seed, nq):
    # the many-query shape (2..6 tables, chain or star, Zipf keys), scaled down
    return W.cfg5(seed, n_queries=nq, min_rows_exp=1.5, max_rows_exp=3.3, min_dom_exp=0.7, max_dom_exp=2.7)


def _qdicts(qs):
    from paper_2206_10435_amd import gj

    return [dict(tables=gj.to_device_tables(q), parent=q.parent, sep_col=q.sep_col, parent_col=q.parent_col)
            for q in qs]


def _check_summary(s, o, q):
    for t in range(q.n_tables):
        g = s.table(t)
        r = o.summary_table(t)
        for k in ("keys", "c", "U", "D", "F"):
            assert np.array_equal(g[k], r[k]), (q.name, t, k)
    for t in range(1, q.n_tables):
        g = s.edge(t)
        r = o.summary_edge(t)
        for k in ("s", "M", "D"):
            assert np.array_equal(g[k], r[k]), (q.name, t, k)


def test_batch_matches_oracle_and_replays(gctx, oracle_mod):
    import torch

    from paper_2206_10435_amd import gj

    qs = _queries(17, 48)
    # two queries whose join size overflows int64 (aligned heavy hitters)
    qs.insert(5, W.chain_query(11, 0, 6, 100_000, 10, 0.0, name="overflow_chain6"))
    qs.append(W.star_query(12, 0, 6, 30_000, 4, 0.0, aligned=True, name="overflow_star6"))
    oracles = [oracle_mod.Oracle(q) for q in qs]
    ref = [o.join_size() for o in oracles]
    _say("case batch", len(qs), "queries,", sum(1 for _, ovf in ref if ovf), "overflow")
    assert sum(1 for _, ovf in ref if ovf) >= 2
    b = gctx.batch_create(_qdicts(qs))
    b.launch(graph=True)
    js, st = b.results()
    for i, ((Q, ovf), q) in enumerate(zip(ref, qs)):
        if ovf:
            assert st[i] == gj.GJ_E_OVERFLOW, i
        else:
            assert st[i] == gj.GJ_OK and js[i] == Q, (i, js[i], Q)
    # full summaries of the non-overflowing queries
    for i, ((Q, ovf), q, o) in enumerate(zip(ref, qs, oracles)):
        if not ovf:
            _check_summary(b.summary(i), o, q)
    # materialize a few from the batch summaries
    for i in [k for k, (Q, ovf) in enumerate(ref) if not ovf and 0 < Q <= 200_000][:6]:
        s = b.summary(i)
        out = torch.empty(ref[i][0] * qs[i].n_tables, dtype=torch.int32, device="cuda:0")
        assert gctx.desummarize(s, 0, ref[i][0], out) == ref[i][0]
        got = out.view(-1, qs[i].n_tables).cpu().numpy()
        assert np.array_equal(got, oracles[i].canonical_result()), i
    # replays: graph, eager, graph again -- identical results every time
    first = (js.copy(), st.copy())
    for mode in ("kernels", "eager", "kernels", "kernels"):
        b.launch(mode=mode)
        torch.cuda.synchronize()
        js2, st2 = b.results()
        assert np.array_equal(js2, first[0]) and np.array_equal(st2, first[1]), mode
    for i in [k for k, (Q, ovf) in enumerate(ref) if not ovf][:5]:
        _check_summary(b.summary(i), oracles[i], qs[i])


def test_batch_equals_single_query_path(gctx, oracle_mod):
    from paper_2206_10435_amd import gj

    qs = _queries(23, 12)
    b = gctx.batch_create(_qdicts(qs))
    b.launch(graph=True)
    js, st = b.results()
    for i, q in enumerate(qs):
        tabs = gj.to_device_tables(q)
        f = gctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col)
        try:
            s = gctx.summarize(f)
        except gj.GJError as e:
            assert e.status == gj.GJ_E_OVERFLOW and st[i] == gj.GJ_E_OVERFLOW
            continue
        assert st[i] == gj.GJ_OK and js[i] == s.join_size
        sb = b.summary(i)
        for t in range(q.n_tables):
            a1, a2 = s.table(t), sb.table(t)
            for k in a1:
                assert np.array_equal(a1[k], a2[k]), (i, t, k)


def test_batch_with_tune(gctx, oracle_mod):
    from paper_2206_10435_amd import gj

    qs = _queries(29, 10)
    ref = [oracle_mod.Oracle(q).join_size() for q in qs]
    b = gctx.batch_create(_qdicts(qs), tune=gj.Tune(8, 6, 4, 2))
    b.launch(graph=True)
    js, st = b.results()
    for i, (Q, ovf) in enumerate(ref):
        assert (st[i] == gj.GJ_E_OVERFLOW) if ovf else (st[i] == gj.GJ_OK and js[i] == Q)


@pytest.mark.skip(reason="the persistent batch kernel is switched off: its first launch on the device did not "
                         "finish within the run's silence limit and the cause has not been shown")
def test_persistent_kernel_every_mode_and_task_size(gctx, oracle_mod):
    """The persistent kernel at task sizes from one tile to whole tables, with
    8- and 16-key sort tiles, against the oracle on every replay (with eager
    work in between), and bit-identical to the launch-per-stage graph."""
    import torch

    from paper_2206_10435_amd import gj

    qs = _queries(31, 36) + [W.cfg5_query(i) for i in (3, 9)]
    qs.insert(7, W.chain_query(11, 0, 6, 100_000, 10, 0.0, name="overflow_chain6"))
    oracles = [oracle_mod.Oracle(q) for q in qs]
    ref = [o.join_size() for o in oracles]
    check = [i for i, (Q, ovf) in enumerate(ref) if not ovf][:: 5] + [len(qs) - 2, len(qs) - 1]
    for si, rows in [(8, 0), (8, 256), (16, 2048), (8, 1 << 20)]:
        b = gctx.batch_create(_qdicts(qs), tune=gj.Tune(si, 8, 0, 4, rows))
        info = b.info()
        _say("case persistent", si, rows, info)
        assert info["tasks"] > 0 and info["grid"] >= 1
        kept = None
        for rep, mode in enumerate(("persistent", "kernels", "persistent", "eager", "persistent")):
            junk = torch.randn(1 << 18, device="cuda:0").sum()  # eager work between launches
            b.launch(mode=mode)
            js, st = b.results()
            for i, (Q, ovf) in enumerate(ref):
                if ovf:
                    assert st[i] == gj.GJ_E_OVERFLOW, (mode, i)
                else:
                    assert st[i] == gj.GJ_OK and js[i] == Q, (mode, i, js[i], Q)
            sums = {i: [b.summary(i).table(t) for t in range(qs[i].n_tables)] for i in check}
            if kept is None:
                kept = sums
                for i in check:
                    _check_summary(b.summary(i), oracles[i], qs[i])
            else:
                for i in check:
                    for t, (x, y) in enumerate(zip(sums[i], kept[i])):
                        for k in x:
                            assert np.array_equal(x[k], y[k]), (mode, rep, i, t, k)
            del junk


def test_persistent_launch_refused_while_switched_off(gctx):
    from paper_2206_10435_amd import gj

    qs = _queries(37, 4)
    b = gctx.batch_create(_qdicts(qs))
    info = b.info()
    assert info["tasks"] > 0 and info["stages"] > 0
    with pytest.raises(gj.GJError) as ei:
        b.launch(mode="persistent")
    assert ei.value.status == gj.GJ_E_INVALID and "switched off" in str(ei.value)
