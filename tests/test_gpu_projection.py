"""Early projections on the GPU (gj_summarize_projected +
gj_desummarize_projected) against the oracle's projection: the projected
result element by element, and every kept table's projected entries and
edges, bit-exact."""
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


def _expand(gctx, s, first, count):
    import torch

    nc = gctx.result_columns(s)
    out = torch.full((max(count, 1) * nc,), -7, dtype=torch.int32, device="cuda:0")
    nw = gctx.desummarize_projected(s, first, count, out)
    return out[: nw * nc].view(nw, nc).cpu().numpy(), nw


def _check(gctx, oracle_mod, q, mask, windows=True):
    from paper_2206_10435_amd import gj

    o = oracle_mod.Oracle(q)
    ok, mn, kept = o.projection(mask)
    assert ok
    tabs = gj.to_device_tables(q)
    f = gctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col)
    s = gctx.summarize_projected(f, mask)
    Q, _ = o.join_size()
    _say("case projection", q.name, "mask", [int(x) for x in mask], "Q", Q)
    assert s.join_size == Q
    src = [t for t in range(q.n_tables) if kept[t]]
    assert s.n_tables == len(src)
    for i, t in enumerate(src):
        g, r = s.table(i), o.projected_table(mask, t)
        for k in ("keys", "c", "U", "D", "F"):
            assert np.array_equal(g[k], r[k]), (t, k)
        if i > 0:
            ge, re = s.edge(i), o.summary_edge(t)
            for k in ("s", "M", "D"):
                assert np.array_equal(ge[k], re[k]), (t, "edge", k)
    ref = o.projected_result(mask)
    got, nw = _expand(gctx, s, 0, Q + 3)
    assert nw == Q and np.array_equal(got, ref)
    if windows and Q > 2:
        for first, cnt in ((1, Q - 2), (Q // 2, min(Q - Q // 2, 999)), (Q - 1, 5)):
            got, nw = _expand(gctx, s, first, cnt)
            exp = ref[first:first + cnt]
            assert nw == len(exp) and np.array_equal(got, exp), (first, cnt)
    return s


FIG1_MASKS = {"A": [1, 0, 0], "AB": [3, 0, 0], "ABC": [3, 2, 0], "ABCD": [3, 2, 2], "BC": [2, 2, 0]}


@pytest.mark.parametrize("name", sorted(FIG1_MASKS))
def test_fig1(gctx, oracle_mod, name):
    _check(gctx, oracle_mod, load_fig1(), FIG1_MASKS[name])


def test_fig1_unsupported(gctx):
    from paper_2206_10435_amd import gj

    q = load_fig1()
    tabs = gj.to_device_tables(q)
    f = gctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col)
    for mask, code in (([0, 0, 2], gj.GJ_E_GRAPH), ([1, 0, 2], gj.GJ_E_GRAPH), ([0, 2, 0], gj.GJ_E_GRAPH),
                       ([3, 1, 2], gj.GJ_E_GRAPH),
                       ([0, 0, 0], gj.GJ_E_INVALID), ([4, 0, 0], gj.GJ_E_INVALID)):
        with pytest.raises(gj.GJError) as ei:
            gctx.summarize_projected(f, mask)
        assert ei.value.status == code, mask


def test_random_trees(gctx, oracle_mod):
    done = 0
    for seed in range(10):
        n = 2 + seed % 5
        q = W.random_tree_query(700 + seed, n, 300 if n <= 3 else 80, 40 if n <= 3 else 12, s=0.8,
                                min_rows=30, max_extra_cols=2)
        o = oracle_mod.Oracle(q)
        rng = np.random.Generator(np.random.PCG64(seed))
        tried = 0
        for _ in range(60):
            mask = [int(rng.integers(0, 1 << len(tb))) for tb in q.tables]
            if not o.projection(mask)[0] or len(o.projected_columns(mask)) > 16:
                continue
            _check(gctx, oracle_mod, q, mask)
            tried += 1
            done += 1
            if tried == 3:
                break
    assert done >= 15


def test_cfg1_chain3(gctx, oracle_mod):
    q = W.cfg1()
    for mask in ([3, 0, 0], [1, 0, 0], [3, 2, 0], [3, 3, 3]):
        _check(gctx, oracle_mod, q, mask, windows=(mask == [3, 2, 0]))


@pytest.mark.parametrize("n,rows,mask", [(2, 3000, [1, 0]), (2, 3000, [3, 0]), (2, 3000, [3, 2]),
                                         (3, 300, [3, 2, 2]), (4, 80, [3, 2, 2, 2])],
                         ids=["A", "AB", "ABC", "ABCD", "ABCDE"])
def test_long_runs(gctx, oracle_mod, n, rows, mask):
    """Chains over two key values: the projected result is a handful of runs
    of 1e5 to 1e6 identical tuples, so whole waves of the run expansion lie
    inside one run (1 to 5 columns per tuple), whole and from unaligned
    offsets."""
    q = W.chain_query(31, 9, n, rows, 2, 0.0, name=f"long_runs{n}")
    _check(gctx, oracle_mod, q, mask)


def test_projected_entry_grouping_many_full_entries(gctx, oracle_mod):
    """Keeping only A of T0(A, B): each of the 3 A values groups about a
    thousand full (A, B) entries, so a projected frequency is summed over
    many waves."""
    q = W.chain_query(32, 9, 2, [40000, 4000], 2000, 0.0, name="wide_groups")
    q.tables[0][0] = (q.tables[0][0] % 3).astype(np.int32)
    _check(gctx, oracle_mod, q, [1, 0])
    _check(gctx, oracle_mod, q, [3, 0])


def test_values_of_unprojected_summary(gctx, oracle_mod):
    """On a full summary, run expansion writes every attribute of every result
    row: the oracle's sorted result mapped to its values."""
    from paper_2206_10435_amd import gj

    for q in (load_fig1(), W.random_tree_query(801, 4, 60, 10, s=0.5, min_rows=10)):
        o = oracle_mod.Oracle(q)
        rows = o.canonical_result()
        cols = [(t, c) for t in range(q.n_tables) for c in range(len(q.tables[t]))
                if t == 0 or c != q.sep_col[t]]
        ref = np.stack([q.tables[t][c][rows[:, t]] for t, c in cols], axis=1)
        tabs = gj.to_device_tables(q)
        s = gctx.summarize(gctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col))
        assert gctx.result_columns(s) == len(cols)
        got, nw = _expand(gctx, s, 0, s.join_size)
        assert nw == len(ref) and np.array_equal(got, ref)


def test_projected_summary_rejects_row_id_calls(gctx):
    import torch

    from paper_2206_10435_amd import gj

    q = load_fig1()
    tabs = gj.to_device_tables(q)
    s = gctx.summarize_projected(gctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col), [3, 0, 0])
    out = torch.empty(256, dtype=torch.int64, device="cuda:0")
    with pytest.raises(gj.GJError) as ei:
        gctx.desummarize(s, 0, 4, out)
    assert ei.value.status == gj.GJ_E_INVALID
    with pytest.raises(gj.GJError) as ei:
        gctx.colset(s, [(0, tabs[0][0])])
    assert ei.value.status == gj.GJ_E_INVALID
    with pytest.raises(gj.GJError) as ei:
        gctx.unroll_gfjs(s, 0, 4)
    assert ei.value.status == gj.GJ_E_INVALID
    o32 = torch.empty(256, dtype=torch.int32, device="cuda:0")
    with pytest.raises(gj.GJError) as ei:
        gctx.desummarize_projected(s, s.join_size + 1, 4, o32)
    assert ei.value.status == gj.GJ_E_RANGE
