"""Parity of the HIP path (through the C ABI) with the CPU oracle: factors,
summary, join size and materialized tuples, bit-exact."""
import numpy as np
import pytest

from conftest import load_fig1
from paper_2206_10435_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gctx():
    from paper_2206_10435_amd import gj

    ctx = gj.Context(0)
    yield ctx


def _say(*a):
    print(*a, flush=True)


def _factor_parity(f, o, q):
    for t in range(q.n_tables):
        g = f.table(t)
        r = o.factor(t)
        assert np.array_equal(g["keys"], r["keys"]), f"factor keys t={t}"
        assert np.array_equal(g["count"], r["count"]), f"factor counts t={t}"
        assert np.array_equal(g["start"].astype(np.int64), r["start"]), f"factor starts t={t}"
        assert np.array_equal(g["perm"], r["perm"]), f"factor perm t={t}"


def _summary_parity(s, o, q):
    Q, ovf = o.join_size()
    assert not ovf
    assert s.join_size == Q
    for t in range(q.n_tables):
        g = s.table(t)
        r = o.summary_table(t)
        for k in ("keys", "c", "U", "D", "F"):
            assert np.array_equal(g[k], r[k]), f"summary {k} t={t}"
        # pre: exclusive prefix of c*U inside each separator group (whole table at the root)
        cu = g["c"] * g["U"]
        grp = np.zeros(len(cu), dtype=np.int64) if t == 0 else g["keys"][:, q.sep_col[t]].astype(np.int64)
        exp = np.zeros(len(cu), dtype=np.int64)
        for i in range(1, len(cu)):
            exp[i] = 0 if grp[i] != grp[i - 1] else exp[i - 1] + cu[i - 1]
        assert np.array_equal(g["pre"], exp), f"summary pre t={t}"
    for t in range(1, q.n_tables):
        g = s.edge(t)
        r = o.summary_edge(t)
        for k in ("s", "M", "D"):
            assert np.array_equal(g[k], r[k]), f"edge {k} t={t}"


def _desum(gctx, s, n, first, count, dtype):
    import torch

    out = torch.full((max(count, 1) * n,), -7, dtype=dtype, device="cuda:0")
    nw = gctx.desummarize(s, first, count, out)
    return out[: nw * n].view(nw, n).cpu().numpy().astype(np.int64), nw


def _full(gctx, q, o, check_factors=True, rowid_dtypes=("int32",)):
    import torch

    from paper_2206_10435_amd import gj

    tabs = gj.to_device_tables(q)
    f = gctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col)
    if check_factors:
        _factor_parity(f, o, q)
    s = gctx.summarize(f)
    _summary_parity(s, o, q)
    Q = s.join_size
    assert Q <= 4_000_000, "full materialization is for joins of at most a few million tuples"
    ref = o.canonical_result().astype(np.int64)
    for dt in rowid_dtypes:
        got, nw = _desum(gctx, s, q.n_tables, 0, Q, getattr(torch, dt))
        assert nw == Q
        assert np.array_equal(got, ref), f"tuples ({dt})"
    return f, s, ref


def test_fig1(gctx, oracle_mod):
    _say("case fig1")
    q = load_fig1()
    o = oracle_mod.Oracle(q)
    _full(gctx, q, o, rowid_dtypes=("int32", "int64"))


def _tiny():
    out = []
    for seed in range(14):
        n = 2 + seed % 4
        maxr = {2: 30, 3: 14, 4: 8, 5: 6}[n]
        out.append(W.random_tree_query(seed, n, maxr, domain=2 + seed % 3, s=0.5 * (seed % 3),
                                       allow_empty=(seed % 7 == 6), min_rows=maxr // 2, max_extra_cols=1))
    return out


@pytest.mark.parametrize("q", _tiny(), ids=lambda q: q.name)
def test_tiny_random(gctx, oracle_mod, q):
    _say("case tiny", q.name)
    _full(gctx, q, oracle_mod.Oracle(q))


def _medium():
    # several tiles per table (4096 rows per tile), ragged tails, up to 8 key columns
    specs = [(101, 3, 9000, 300, 0.9), (102, 4, 6000, 1200, 0.6), (103, 5, 5000, 1500, 0.9),
             (104, 6, 4000, 1500, 0.3), (105, 3, 20000, 4000, 1.2), (106, 4, 12000, 3000, 0.0),
             (108, 5, 8000, 2000, 1.0)]
    return [W.random_tree_query(seed, n, rows, dom, s=s, max_extra_cols=3, min_rows=rows // 3)
            for seed, n, rows, dom, s in specs]


@pytest.mark.parametrize("q", _medium(), ids=lambda q: q.name)
def test_medium_random(gctx, oracle_mod, q):
    o = oracle_mod.Oracle(q)
    Q, _ = o.join_size()
    _say("case medium", q.name, "Q =", Q)
    if Q > 3_000_000:
        pytest.skip(f"join size {Q} too large for full materialization on the CPU")
    _full(gctx, q, o)


def test_cfg1_chain3(gctx, oracle_mod):
    q = W.cfg1()
    o = oracle_mod.Oracle(q)
    _say("case cfg1", o.join_size())
    f, s, ref = _full(gctx, q, o)
    # chunked, odd sizes, both widths
    import torch

    Q = s.join_size
    pos = 0
    for i, sz in enumerate([1, 7, 1000, 12345, 99999, 3, 500000]):
        if pos >= Q:
            break
        got, nw = _desum(gctx, s, 3, pos, sz, torch.int64 if i % 2 else torch.int32)
        assert nw == min(sz, Q - pos)
        assert np.array_equal(got, ref[pos:pos + nw])
        pos += nw
    # a range past the end is clipped, beyond it is an error
    got, nw = _desum(gctx, s, 3, Q - 5, 100, torch.int32)
    assert nw == 5 and np.array_equal(got, ref[Q - 5:])
    got, nw = _desum(gctx, s, 3, Q, 100, torch.int32)
    assert nw == 0
    from paper_2206_10435_amd import gj

    with pytest.raises(gj.GJError) as ei:
        _desum(gctx, s, 3, Q + 1, 10, torch.int32)
    assert ei.value.status == gj.GJ_E_RANGE


def test_wide_keys_128bit(gctx, oracle_mod):
    # root with two full-range int32 columns + a join column: > 64 packed bits
    rng = np.random.default_rng(7)
    n0, n1 = 7000, 5000
    a = rng.integers(-2**31, 2**31 - 1, n0, dtype=np.int64).astype(np.int32)
    b = rng.integers(-2**31, 2**31 - 1, n0, dtype=np.int64).astype(np.int32)
    a[:50] = a[50:100]  # some duplicate entries
    b[:50] = b[50:100]
    c = rng.integers(0, 300, n0).astype(np.int32)
    c[:50] = c[50:100]
    d = rng.integers(0, 300, n1).astype(np.int32)
    e = rng.integers(-5, 5, n1).astype(np.int32)
    q = W.Query("wide", [[a, b, c], [d, e]], [-1, 0], [0, 0], [0, 2])
    o = oracle_mod.Oracle(q)
    _say("case wide", o.join_size())
    _full(gctx, q, o)
    try:
        for si, rb in ((8, 5), (16, 7)):  # narrower digits on 128-bit words (more passes)
            gctx.set_tune(si, rb)
            _full(gctx, q, o)
    finally:
        gctx.set_tune()


def _wide_keys_query():
    # four full-range int32 key columns and a join column (more than 128 key
    # bits with the row ids) in the root and in its child, some rows repeated
    rng = np.random.default_rng(11)

    def full(n):
        return rng.integers(-2**31, 2**31 - 1, n, dtype=np.int64).astype(np.int32)

    n0, n1, n2 = 9000, 4000, 2000
    t0 = [full(n0) for _ in range(4)] + [rng.integers(0, 500, n0).astype(np.int32)]
    t1 = [rng.integers(0, 500, n1).astype(np.int32)] + [full(n1) for _ in range(4)] + \
         [rng.integers(0, 40, n1).astype(np.int32)]
    t2 = [rng.integers(0, 40, n2).astype(np.int32), full(n2)]
    for tab in (t0, t1):
        for c in tab:
            c[:150] = c[300:450]  # whole repeated rows: entries of count 2
    t0[1][450:600] = t0[1][600:750]  # repeated values inside a column
    return W.Query("wider_than_128", [t0, t1, t2], [-1, 0, 1], [0, 0, 0], [0, 4, 5])


def test_keys_wider_than_a_sort_word(gctx, oracle_mod):
    """Tables whose key and row-id bits exceed 128: the widest columns are
    ranked for the sort and their values restored in the entries' keys."""
    q = _wide_keys_query()
    o = oracle_mod.Oracle(q)
    _say("case wider than 128 bits", o.join_size())
    _full(gctx, q, o, rowid_dtypes=("int32", "int64"))


def test_degenerate_tables(gctx, oracle_mod):
    import torch

    from paper_2206_10435_amd import gj

    # constant keys (no key bits at all), a single-row table, extreme values
    c0 = np.full(100, 5, np.int32)
    q = W.Query("const", [[c0, np.arange(100, dtype=np.int32)], [np.full(3, 5, np.int32)],
                          [np.array([2**31 - 1], np.int32), np.array([-2**31], np.int32)]],
                [-1, 0, 0], [0, 0, 0], [0, 0, 1])
    q.tables[2] = [np.array([1], np.int32), np.array([-2**31], np.int32)]
    q.tables[0][1][:] = np.arange(100, dtype=np.int32) % 2
    q.tables[0][1][7] = 1
    q = W.Query("const", [[c0, q.tables[0][1]], [np.full(3, 5, np.int32)],
                          [np.array([1, 1], np.int32), np.array([-2**31, 2**31 - 1], np.int32)]],
                [-1, 0, 0], [0, 0, 0], [0, 0, 1])
    o = oracle_mod.Oracle(q)
    _say("case degenerate", o.join_size())
    _full(gctx, q, o)
    # an empty table empties the join
    q2 = W.Query("empty", [[c0, c0.copy()], [np.zeros(0, np.int32)]], [-1, 0], [0, 0], [0, 1])
    o2 = oracle_mod.Oracle(q2)
    tabs = gj.to_device_tables(q2)
    f = gctx.build_factors(tabs, q2.parent, q2.sep_col, q2.parent_col)
    _factor_parity(f, o2, q2)
    s = gctx.summarize(f)
    assert s.join_size == 0
    out = torch.empty(16, dtype=torch.int32, device="cuda:0")
    assert gctx.desummarize(s, 0, 4, out) == 0
    with pytest.raises(gj.GJError):
        gctx.desummarize(s, 1, 4, out)


def test_tune_variants_same_result(gctx, oracle_mod):
    q = W.random_tree_query(201, 4, 9000, 1500, s=0.8, max_extra_cols=3, min_rows=3000)
    o = oracle_mod.Oracle(q)
    _say("case tune", o.join_size())
    try:
        for si, rb, dr, ds in [(8, 4, 1, 4), (16, 6, 3, 2), (8, 8, 17, 8), (16, 7, 5, 2), (16, 8, 1, 8)]:
            gctx.set_tune(si, rb, dr, ds)
            _full(gctx, q, o)
    finally:
        gctx.set_tune()


def _by_table_count():
    # one query per table count, 1..10 (10 runs the kernel built for any count)
    specs = [(1, 300, 50000, 10), (2, 300, 3000, 100), (3, 306, 2000, 500), (4, 300, 1500, 300),
             (5, 303, 800, 300), (6, 300, 800, 300), (7, 300, 800, 300), (8, 300, 800, 300),
             (9, 300, 800, 300), (10, 301, 800, 300)]
    return [W.random_tree_query(seed, n, rows, dom, s=0.7, max_extra_cols=2, min_rows=rows // 2)
            for n, seed, rows, dom in specs]


@pytest.mark.parametrize("q", _by_table_count(), ids=lambda q: f"n{q.n_tables}")
def test_expansion_every_stage_width_table_count(gctx, oracle_mod, q):
    """Every staging depth and row-id width at every table count, whole and
    ragged ranges: covers lane segments that are not whole 16-byte units at
    the requested depth (int32 ids, odd table counts) and the staging layouts."""
    import torch

    from paper_2206_10435_amd import gj

    o = oracle_mod.Oracle(q)
    ref = o.canonical_result().astype(np.int64)
    tabs = gj.to_device_tables(q)
    s = gctx.summarize(gctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col))
    Q = s.join_size
    assert Q == len(ref) and Q > 0
    n = q.n_tables
    _say("case stages", q.name, "n =", n, "Q =", Q)
    first = Q // 3 + 1
    cnt = min(Q - first, 4097 + 13 * n)
    try:
        for stage in (2, 4, 8):
            for rounds in (1, 7):
                # the general kernel (a two-table summary would take the keyed-lookup one)
                gctx.set_tune(16, 8, rounds, stage, desum_general=1)
                assert gctx.desum_kernel(s) == "general"
                for dt in (torch.int32, torch.int64):
                    got, nw = _desum(gctx, s, n, 0, Q, dt)
                    assert nw == Q and np.array_equal(got, ref), (stage, rounds, dt)
                    got, nw = _desum(gctx, s, n, first, cnt, dt)
                    assert nw == cnt and np.array_equal(got, ref[first:first + cnt]), (stage, rounds, dt, "window")
    finally:
        gctx.set_tune()


def test_overflow_reported(gctx, oracle_mod):
    from paper_2206_10435_amd import gj

    q = W.chain_query(11, 0, 6, 100_000, 10, 0.0)
    o = oracle_mod.Oracle(q)
    assert o.join_size()[1]
    _say("case overflow")
    tabs = gj.to_device_tables(q)
    f = gctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col)
    with pytest.raises(gj.GJError) as ei:
        gctx.summarize(f)
    assert ei.value.status == gj.GJ_E_OVERFLOW


def test_unroll_gfjs_fig1_and_ranges(gctx, oracle_mod):
    from conftest import load_fig2
    from paper_2206_10435_amd import gj

    q = load_fig1()
    o = oracle_mod.Oracle(q)
    tabs = gj.to_device_tables(q)
    s = gctx.summarize(gctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col))
    runs = gctx.unroll_gfjs(s, 0, 32)
    gfjs, _, _ = load_fig2()
    for col, (vals, freqs) in zip("ABCD", runs):
        assert list(zip(vals.tolist(), freqs.tolist())) == gfjs[col], col
    # ranges of a larger join against the oracle's runs over the same rows
    q = W.random_tree_query(102, 4, 6000, 1200, s=0.6, max_extra_cols=3, min_rows=2000)
    o = oracle_mod.Oracle(q)
    ref = o.canonical_result()
    s = gctx.summarize(gctx.build_factors(gj.to_device_tables(q), q.parent, q.sep_col, q.parent_col))
    Q = s.join_size
    for first, cnt in [(0, Q), (1, 5000), (Q // 3, 70001), (Q - 10, 50)]:
        got = gctx.unroll_gfjs(s, first, cnt)
        exp = o.gfjs(ref[first:first + cnt])
        assert len(got) == len(exp)
        for (gv, gf), (ev, ef) in zip(got, exp):
            assert np.array_equal(gv, ev) and np.array_equal(gf, ef), (first, cnt)
            assert int(gf.sum()) == min(cnt, Q - first)


def _bucketed_queries():
    # parents with at least 4x their children's rows take the downward pass by
    # buckets (child groups summed per bucket in LDS), the others the atomic
    # scatter: star leaves of both kinds, small and large group counts (one
    # group per bucket, and many), and a chain where a bucketed child's parent
    # is itself a child (its downward message enters the items)
    star = W.star_query(401, 0, 6, [60000, 200, 5000, 15000, 30000, 9000], 4000, 0.7, name="star_mixed")
    skew = W.star_query(402, 0, 4, [70000, 3000, 17000, 1000], 600, 1.1, name="star_skewed")
    chain = W.chain_query(403, 0, 4, [90000, 20000, 4000, 900], 3000, 0.5, name="chain_shrinking")
    return [star, skew, chain]


@pytest.mark.parametrize("q", _bucketed_queries(), ids=lambda q: q.name)
def test_downward_pass_by_buckets(gctx, oracle_mod, q):
    from paper_2206_10435_amd import gj

    o = oracle_mod.Oracle(q)
    Q, ovf = o.join_size()
    _say("case bucketed down", q.name, "Q =", Q, "overflow", ovf)
    assert not ovf
    f = gctx.build_factors(gj.to_device_tables(q), q.parent, q.sep_col, q.parent_col)
    s = gctx.summarize(f)
    _summary_parity(s, o, q)
    # the same summary from a batch of the query twice (one plan, both paths)
    b = gctx.batch_create([dict(tables=gj.to_device_tables(q), parent=q.parent, sep_col=q.sep_col,
                                parent_col=q.parent_col)] * 2)
    b.launch(graph=True)
    js, st = b.results()
    assert list(js) == [Q, Q] and list(st) == [gj.GJ_OK, gj.GJ_OK]
    _summary_parity(b.summary(1), o, q)
