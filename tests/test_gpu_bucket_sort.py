"""The factor build's bucket sort for tables with 128-bit sort words (Sec. 3.2,
potentials from one group-by): global passes over the two top digits, then each
run of equal top bits sorted in LDS.  Forced onto small tables with
sort_local_rows = 1 and checked against the oracle -- entries (keys, counts,
starts), the row order inside every entry, and the summary -- on spread keys,
repeated rows, separator groups of a child table, every edge of the block
ranges (tables of 1 to a few tiles), and tables with a bucket longer than a
block holds, which must take the full per-digit sort instead."""
import numpy as np
import pytest

from paper_2206_10435_amd import workloads as W

pytestmark = pytest.mark.gpu

TILE = 704  # positions per block of the LDS sort
CAP = 1920  # longest range a block sorts


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def gctx():
    from paper_2206_10435_amd import gj

    ctx = gj.Context(0)
    ctx.set_tune(sort_local_rows=1)
    yield ctx
    ctx.set_tune()


def _spread(rng, n, bits=(20, 17, 19, 19)):
    return [rng.integers(0, 1 << b, n).astype(np.int32) for b in bits]


def _root_and_child(rng, cols0, n1):
    """Root with the given columns; a child joined on root column 0."""
    lo, hi = int(cols0[0].min()), int(cols0[0].max())
    c = [rng.integers(lo, hi + 1, n1).astype(np.int32), rng.integers(-3, 4, n1).astype(np.int32)]
    return W.Query("bucket", [cols0, c], [-1, 0], [0, 0], [0, 0])


def _cases():
    rng = np.random.default_rng(2026)
    out = []
    # spread keys: about five rows per bucket
    out.append(("spread_300k", _root_and_child(rng, _spread(rng, 300_000), 20_000)))
    # rows drawn from a pool of 3000 wide tuples: entries of many rows
    pool = np.stack(_spread(rng, 3000), axis=1)
    rows = pool[rng.integers(0, 3000, 60_000)]
    out.append(("repeated_rows", _root_and_child(rng, [rows[:, c].copy() for c in range(4)], 5_000)))
    # one top-bit run longer than a block holds (a value of the first column on
    # 12000 rows) among spread keys: the table is sorted again in full
    cols = _spread(rng, 80_000)
    cols[0][rng.permutation(80_000)[:12_000]] = 777
    out.append(("long_bucket", _root_and_child(rng, cols, 4_000)))
    # a run of about CAP - TILE rows: the longest that fits wherever it starts
    # (and more than LS_SMALL words share its top varying digit: the LSD passes)
    cols = _spread(rng, 40_000)
    cols[0][rng.permutation(40_000)[:CAP - TILE - 48]] = 4242
    out.append(("bucket_near_cap", _root_and_child(rng, cols, 3_000)))
    # a child whose key is 128 bits wide: separator groups
    n1 = 50_000
    child = [rng.integers(0, 900, n1).astype(np.int32)] + _spread(rng, n1, (20, 20, 18))
    root = [rng.integers(0, 900, 2_000).astype(np.int32), rng.integers(0, 5, 2_000).astype(np.int32)]
    out.append(("wide_child", W.Query("wide_child", [root, child], [-1, 0], [0, 0], [0, 0])))
    # block-range edges: tables of 1 row up to a few tiles
    for n in (1, 2, TILE - 1, TILE, TILE + 1, 2 * TILE + 7, CAP + 1, 3 * TILE):
        out.append((f"n{n}", _root_and_child(rng, _spread(rng, n, (31, 31, 20)), 50)))
    return out


def _factor_parity(f, o, q, name):
    for t in range(q.n_tables):
        g, r = f.table(t), o.factor(t)
        for k in ("keys", "count", "perm"):
            assert np.array_equal(g[k], r[k]), (name, t, k)
        assert np.array_equal(g["start"].astype(np.int64), r["start"]), (name, t, "start")


@pytest.mark.parametrize("idx", range(13))
def test_bucket_sort_matches_oracle(gctx, oracle_mod, idx):
    from paper_2206_10435_amd import gj

    name, q = _cases()[idx]
    _say("case", name, [q.n_rows(t) for t in range(q.n_tables)])
    o = oracle_mod.Oracle(q)
    tabs = gj.to_device_tables(q)
    f = gctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col)
    kinds = [f.sort_kind(t) for t in range(q.n_tables)]
    _say("  sort", kinds)
    wide = 0 if name != "wide_child" else 1
    if name == "long_bucket":
        assert kinds[wide] == "buckets_redone"
    elif q.n_rows(wide) > 1:
        assert kinds[wide] == "buckets"
    _factor_parity(f, o, q, name)
    s = gctx.summarize(f)
    Q, ovf = o.join_size()
    assert not ovf and s.join_size == Q
    for t in range(q.n_tables):
        g, r = s.table(t), o.summary_table(t)
        for k in ("keys", "c", "U", "D", "F"):
            assert np.array_equal(g[k], r[k]), (name, t, k)


def test_same_factors_as_the_per_digit_sort(gctx):
    """Both sorts on the same tables give identical factor arrays."""
    from paper_2206_10435_amd import gj

    name, q = _cases()[0]
    tabs = gj.to_device_tables(q)
    f1 = gctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col)
    assert f1.sort_kind(0) == "buckets"
    ref = [f1.table(t) for t in range(q.n_tables)]
    try:
        gctx.set_tune(sort_local_rows=0)
        f0 = gctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col)
        assert f0.sort_kind(0) == "digits"
        for t in range(q.n_tables):
            g = f0.table(t)
            for k in ("keys", "count", "start", "end", "perm"):
                assert np.array_equal(g[k], ref[t][k]), (t, k)
    finally:
        gctx.set_tune(sort_local_rows=1)


def test_bad_arguments_refused(gctx):
    """sort_local_rows < 0 and a table index outside the factor set are refused
    with GJ_E_INVALID, and the context keeps its setting."""
    from paper_2206_10435_amd import gj

    with pytest.raises(gj.GJError) as ei:
        gctx.set_tune(sort_local_rows=-1)
    assert ei.value.status == gj.GJ_E_INVALID
    assert b"sort_local_rows" in gj.load_library().gj_last_error(gctx.h)
    name, q = _cases()[5]  # two tables of 1 and 50 rows
    f = gctx.build_factors(gj.to_device_tables(q), q.parent, q.sep_col, q.parent_col)
    for t in (-1, q.n_tables):
        with pytest.raises(gj.GJError) as ei:
            f.sort_kind(t)
        assert ei.value.status == gj.GJ_E_INVALID
    assert f.sort_kind(1) == "digits"
