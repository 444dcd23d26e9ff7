"""Payload gather: materializing attribute and payload values through the
expansion kernel (gj_colset_create + gj_desummarize_values), compared element
by element with the oracle's sorted result, whose row ids index the host
copies of the same columns."""
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


def _payload(q, seed, per_table=2):
    """Seeded int32 payload columns (full int32 range) for every table."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 77])))
    return [[rng.integers(-2**31, 2**31 - 1, size=q.n_rows(t), dtype=np.int64).astype(np.int32)
             for _ in range(per_table)] for t in range(q.n_tables)]


def _values(gctx, s, cs, first, count):
    import torch

    nc = cs.n_cols
    out = torch.full((max(count, 1) * nc,), -7, dtype=torch.int32, device="cuda:0")
    nw = gctx.desummarize_values(s, cs, first, count, out)
    return out[: nw * nc].view(nw, nc).cpu().numpy(), nw


def _check_query(gctx, oracle_mod, q, seed, picks, windows=True):
    """picks: list of (table, source, index) with source 'key' or 'pay'."""
    import torch

    from paper_2206_10435_amd import gj

    o = oracle_mod.Oracle(q)
    ref_rows = o.canonical_result()
    pay = _payload(q, seed)
    host_cols, dev_cols = [], []
    for t, src, i in picks:
        h = q.tables[t][i] if src == "key" else pay[t][i]
        host_cols.append((t, np.ascontiguousarray(h, dtype=np.int32)))
        dev_cols.append((t, torch.from_numpy(host_cols[-1][1]).to("cuda:0")))
    ref = np.stack([c[ref_rows[:, t]] for t, c in host_cols], axis=1) if len(ref_rows) else \
        np.zeros((0, len(picks)), np.int32)
    tabs = gj.to_device_tables(q)
    s = gctx.summarize(gctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col))
    Q = s.join_size
    assert Q == len(ref_rows)
    cs = gctx.colset(s, dev_cols)
    _say("case values", q.name, "tables", q.n_tables, "cols", len(picks), "Q", Q)
    got, nw = _values(gctx, s, cs, 0, Q + 5)
    assert nw == Q and np.array_equal(got, ref)
    if windows and Q > 2:
        for first, cnt in ((1, Q - 2), (Q // 2, min(Q - Q // 2, 1001)), (Q - 1, 7)):
            got, nw = _values(gctx, s, cs, first, cnt)
            exp = ref[first:first + cnt]
            assert nw == len(exp) and np.array_equal(got, exp), (first, cnt)
    return s, cs


def test_fig1_all_attributes(gctx, oracle_mod):
    q = load_fig1()
    picks = [(t, "key", c) for t in range(q.n_tables) for c in range(len(q.tables[t]))]
    _check_query(gctx, oracle_mod, q, 1, picks)


def test_cfg1_chain3_payload(gctx, oracle_mod):
    q = W.cfg1()
    picks = [(0, "pay", 0), (1, "pay", 1), (2, "pay", 0), (0, "key", 0), (2, "key", 1)]
    _check_query(gctx, oracle_mod, q, 2, picks, windows=True)


@pytest.mark.parametrize("n,ncols", [(1, 1), (2, 3), (3, 4), (4, 8), (5, 5), (6, 9), (8, 16), (10, 12)])
def test_random_trees(gctx, oracle_mod, n, ncols):
    q = W.random_tree_query(500 + n, n, 400 if n <= 4 else 120, 60 if n <= 4 else 25, s=0.8,
                            max_extra_cols=2, min_rows=20)
    rng = np.random.Generator(np.random.PCG64(900 + n))
    picks = []
    for _ in range(ncols):
        t = int(rng.integers(0, n))
        if rng.random() < 0.5:
            picks.append((t, "key", int(rng.integers(0, len(q.tables[t])))))
        else:
            picks.append((t, "pay", int(rng.integers(0, 2))))
    _check_query(gctx, oracle_mod, q, 3, picks)


def test_errors(gctx, oracle_mod):
    import torch

    from paper_2206_10435_amd import gj

    q = load_fig1()
    tabs = gj.to_device_tables(q)
    s = gctx.summarize(gctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col))
    s2 = gctx.summarize(gctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col))
    col = tabs[0][0]
    with pytest.raises(gj.GJError) as ei:
        gctx.colset(s, [(3, col)])
    assert ei.value.status == gj.GJ_E_INVALID
    with pytest.raises(gj.GJError):
        gctx.colset(s, [(0, col)] * 17)
    cs = gctx.colset(s, [(0, col)])
    out = torch.empty(64, dtype=torch.int32, device="cuda:0")
    with pytest.raises(gj.GJError) as ei:
        gctx.desummarize_values(s2, cs, 0, 4, out)  # set made for other factors
    assert ei.value.status == gj.GJ_E_INVALID
    with pytest.raises(gj.GJError) as ei:
        gctx.desummarize_values(s, cs, s.join_size + 1, 4, out)
    assert ei.value.status == gj.GJ_E_RANGE
    assert gctx.desummarize_values(s, cs, s.join_size, 4, out) == 0
