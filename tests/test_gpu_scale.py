"""Full-size workloads on the GPU, checked against the oracle where it can
compute one answer at a time and by properties that fix the answer otherwise:

* join size: the oracle's row-level count;
* factors: counts sum to the rows, entries strictly increasing, perm a
  permutation whose rows carry their entry's keys;
* summary: every row's fan-out (U*D of its entry) equals the oracle's, and
  the run lengths of every table sum to the join size;
* tuples: windows of 2^20 consecutive result rows (at the start, at offsets
  beyond 2^32, at the end) are valid join tuples, strictly increasing in the
  result order, and the oracle's rank of the first and last tuple of each
  window equals its position -- so each window is exactly those ranks of the
  result; plus the oracle's unrank at sampled positions.
"""
import numpy as np
import pytest

from paper_2206_10435_amd import workloads as W

pytestmark = pytest.mark.gpu

WIN = 1 << 20


@pytest.fixture(scope="module")
def gctx():
    from paper_2206_10435_amd import gj

    return gj.Context(0)


def _say(*a):
    print(*a, flush=True)


def _sort_columns(q, tup):
    """attribute values of every result column, then the row ids (int64)."""
    cols = []
    for t in range(q.n_tables):
        for c in range(len(q.tables[t])):
            if t == 0 or c != q.sep_col[t]:
                cols.append(q.tables[t][c][tup[:, t]].astype(np.int64))
    for t in range(q.n_tables):
        cols.append(tup[:, t].astype(np.int64))
    return np.stack(cols, axis=1)


def _strictly_increasing(m):
    d = np.diff(m, axis=0)
    nz = d != 0
    first = np.argmax(nz, axis=1)
    any_nz = nz.any(axis=1)
    return bool(any_nz.all() and (d[np.arange(len(d)), first] > 0).all())


def _check_window(gctx, s, q, o, first, cnt):
    import torch

    n = q.n_tables
    out = torch.empty(cnt * n, dtype=torch.int64, device="cuda:0")
    nw = gctx.desummarize(s, first, cnt, out)
    assert nw == min(cnt, s.join_size - first)
    tup = out[: nw * n].view(nw, n).cpu().numpy()
    for t in range(1, n):
        p = q.parent[t]
        assert np.array_equal(q.tables[t][q.sep_col[t]][tup[:, t]], q.tables[p][q.parent_col[t]][tup[:, p]]), t
    assert _strictly_increasing(_sort_columns(q, tup))
    _say("  window", first, "valid and increasing; ranking with the oracle")
    assert o.rank(tup[0]) == first
    assert o.rank(tup[-1]) == first + nw - 1
    for pos in (0, nw // 3, nw - 1):
        assert np.array_equal(o.unrank(first + pos), tup[pos])


def _factor_properties(f, q):
    for t in range(q.n_tables):
        g = f.table(t)
        N = q.n_rows(t)
        assert int(g["count"].sum()) == N
        assert np.array_equal(np.sort(g["perm"]), np.arange(N, dtype=np.int32))
        # entries strictly increasing in their sort order (separator first for t >= 1)
        order = ([q.sep_col[t]] if t else []) + [c for c in range(len(q.tables[t])) if t == 0 or c != q.sep_col[t]]
        keys = g["keys"][:, order].astype(np.int64)
        assert _strictly_increasing(keys)
        # every row carries its entry's keys; rows inside an entry ascend
        ent = np.repeat(np.arange(len(g["count"])), g["count"])
        for c in range(len(q.tables[t])):
            assert np.array_equal(q.tables[t][c][g["perm"]], g["keys"][ent, c])
        same = ent[1:] == ent[:-1]
        assert (g["perm"][1:][same] > g["perm"][:-1][same]).all()


def _fanout_parity(f, s, q, o):
    for t in range(q.n_tables):
        fac = f.table(t)
        sm = s.table(t)
        assert int(sm["F"].sum()) == s.join_size
        # map every row to its surviving entry (by key tuple) and compare U*D
        k = len(q.tables[t])
        fan = np.zeros(q.n_rows(t), dtype=np.int64)
        if len(sm["c"]):
            fk = fac["keys"].astype(np.int64)
            sk = sm["keys"].astype(np.int64)
            # entries are sorted; surviving ones are a subsequence: locate them
            fk_view = np.ascontiguousarray(fk).view([("", np.int64)] * k).ravel()
            sk_view = np.ascontiguousarray(sk).view([("", np.int64)] * k).ravel()
            idx = np.searchsorted(fk_view, sk_view) if t == 0 else None
            if idx is None:
                order = [q.sep_col[t]] + [c for c in range(k) if c != q.sep_col[t]]
                fk_o = np.ascontiguousarray(fk[:, order]).view([("", np.int64)] * k).ravel()
                sk_o = np.ascontiguousarray(sk[:, order]).view([("", np.int64)] * k).ravel()
                idx = np.searchsorted(fk_o, sk_o)
            per_entry = np.zeros(len(fac["count"]), dtype=np.int64)
            per_entry[idx] = sm["U"] * sm["D"]
            ent = np.repeat(np.arange(len(fac["count"])), fac["count"])
            fan[fac["perm"]] = per_entry[ent]
        assert np.array_equal(fan, o.fanouts(t)), t


def _run_workload(gctx, oracle_mod, q, windows):
    from paper_2206_10435_amd import gj

    o = oracle_mod.Oracle(q)
    Q, ovf = o.join_size()
    _say(q.name, "join size", Q)
    assert not ovf
    tabs = gj.to_device_tables(q)
    f = gctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col)
    _factor_properties(f, q)
    _say("factors ok")
    s = gctx.summarize(f)
    assert s.join_size == Q
    _fanout_parity(f, s, q, o)
    _say("summary ok")
    for first in windows(Q):
        _check_window(gctx, s, q, o, first, WIN)
        _say("window", first, "ok")


def test_chain4_full_size(gctx, oracle_mod):
    q = W.cfg2(payload=False)
    rng = np.random.default_rng(3)
    _run_workload(gctx, oracle_mod, q,
                  lambda Q: [0, 5 * (1 << 28) + 12345, int(rng.integers(1 << 33, Q - WIN)), Q - WIN // 2])


def test_star_full_size(gctx):
    """Star plus chain at full size (fact 5e7 rows, 128-bit sort words).  Every
    fact row matches exactly one row of each dimension (foreign keys into
    primary keys), so with cntB = number of bridge rows per j value:
      join size        = sum over fact rows f of cntB[j(k1_f)]
      fan-out of f     = cntB[j(k1_f)], of a dimension row = the summed fan-outs
                         of the fact rows that reference it, of a bridge row =
                         the number of fact rows reaching its j through D1;
      rank of a tuple  = (tuples of the fact rows before r0 in (k1..k4, row id)
                         order) + (position of r5 among the bridge rows with
                         the same j, by row id),
    all computed with numpy, independent of both the GPU path and the oracle."""
    import torch

    from paper_2206_10435_amd import gj

    q = W.cfg3()
    F, D1, B = q.tables[0], q.tables[1], q.tables[5]
    nf = q.n_rows(0)
    cntB = np.bincount(B[0], minlength=1_000_000).astype(np.int64)
    d1row = np.empty(q.n_rows(1), dtype=np.int64)
    d1row[D1[0]] = np.arange(q.n_rows(1))
    fan_f = cntB[D1[1][d1row[F[0]]]]
    Q = int(fan_f.sum())
    _say("star join size (closed form)", Q)
    tabs = gj.to_device_tables(q)
    f = gctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col)
    # the fact table's 75 key bits take the bucket sort (top two digits
    # globally, each run of equal top bits in LDS), the dimensions one pass a digit
    assert [f.sort_kind(t) for t in range(q.n_tables)] == ["buckets"] + ["digits"] * 5
    _factor_properties(f, q)
    _say("factors ok")
    s = gctx.summarize(f)
    assert s.join_size == Q
    # per-row fan-outs of every table
    fan = {0: fan_f}
    cnt_k1 = np.bincount(F[0], minlength=q.n_rows(1)).astype(np.int64)
    fan[1] = cnt_k1[D1[0]] * cntB[D1[1]]
    for i in (2, 3, 4):
        fi = np.bincount(F[i - 1], weights=fan_f.astype(np.float64), minlength=q.n_rows(i))
        fan[i] = np.rint(fi).astype(np.int64)[q.tables[i][0]]
    reach = np.rint(np.bincount(D1[1], weights=cnt_k1[D1[0]].astype(np.float64), minlength=1_000_000))
    fan[5] = reach.astype(np.int64)[B[0]]
    for t in range(6):
        fac, sm = f.table(t), s.table(t)
        assert int(sm["F"].sum()) == Q
        per_entry = np.zeros(len(fac["count"]), dtype=np.int64)
        k = len(q.tables[t])
        order = ([q.sep_col[t]] if t else []) + [c for c in range(k) if t == 0 or c != q.sep_col[t]]
        fk = np.ascontiguousarray(fac["keys"][:, order].astype(np.int64)).view([("", np.int64)] * k).ravel()
        sk = np.ascontiguousarray(sm["keys"][:, order].astype(np.int64)).view([("", np.int64)] * k).ravel()
        per_entry[np.searchsorted(fk, sk)] = sm["U"] * sm["D"]
        got = np.zeros(q.n_rows(t), dtype=np.int64)
        got[fac["perm"]] = per_entry[np.repeat(np.arange(len(fac["count"])), fac["count"])]
        assert np.array_equal(got, fan[t]), t
    _say("summary ok (all per-row fan-outs)")
    # rank of every tuple of a window, in closed form
    order = np.lexsort((np.arange(nf), F[3], F[2], F[1], F[0]))
    start = np.empty(nf, dtype=np.int64)
    start[order] = np.concatenate([[0], np.cumsum(fan_f[order])[:-1]])
    ordB = np.argsort(B[0], kind="stable")
    gstart = np.searchsorted(B[0][ordB], np.arange(1_000_000))
    pos_in_j = np.empty(q.n_rows(5), dtype=np.int64)
    pos_in_j[ordB] = np.arange(q.n_rows(5)) - gstart[B[0][ordB]]
    rng = np.random.default_rng(4)
    for first in [0, int(rng.integers(WIN, Q - WIN)), Q - WIN + 7]:
        out = torch.empty(WIN * 6, dtype=torch.int64, device="cuda:0")
        nw = gctx.desummarize(s, first, WIN, out)
        assert nw == min(WIN, Q - first)
        tup = out[: nw * 6].view(nw, 6).cpu().numpy()
        for t in range(1, 6):
            p = q.parent[t]
            assert np.array_equal(q.tables[t][q.sep_col[t]][tup[:, t]], q.tables[p][q.parent_col[t]][tup[:, p]])
        assert np.array_equal(start[tup[:, 0]] + pos_in_j[tup[:, 5]], first + np.arange(nw))
        _say("window", first, "ok")


def test_star_scaled_against_oracle(gctx, oracle_mod):
    """The same star shape at 1/100 of the size, every tuple against the oracle."""
    import torch

    from paper_2206_10435_amd import gj

    q = W.cfg3(fact_rows=500_000, dim_rows=(10_000, 1_000, 3_000, 5_000), bridge_rows=100_000,
               bridge_domain=10_000)
    o = oracle_mod.Oracle(q)
    Q, _ = o.join_size()
    _say("scaled star", Q)
    f = gctx.build_factors(gj.to_device_tables(q), q.parent, q.sep_col, q.parent_col)
    s = gctx.summarize(f)
    assert s.join_size == Q
    for t in range(6):
        g, r = s.table(t), o.summary_table(t)
        for k in ("keys", "c", "U", "D", "F"):
            assert np.array_equal(g[k], r[k]), (t, k)
    out = torch.empty(Q * 6, dtype=torch.int64, device="cuda:0")
    assert gctx.desummarize(s, 0, Q, out) == Q
    assert np.array_equal(out.view(Q, 6).cpu().numpy(), o.canonical_result())


def test_chain4_values_and_projection_full_size(gctx):
    """The 4-table chain at full size with its payload: windows far into the
    result (beyond 2^32 rows) of (a) the 8 payload columns equal the payload
    at the row ids the row-id expansion writes for the same window, and (b)
    the projection onto (A, B, C) equals the (A, B, C) values of the same
    window of the full result (sorting by all columns and keeping a prefix
    of them keeps the order and the multiplicities)."""
    import torch

    from paper_2206_10435_amd import gj

    q = W.cfg2()
    tabs = gj.to_device_tables(q)
    f = gctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col)
    s = gctx.summarize(f)
    Q = s.join_size
    n = q.n_tables
    pay = [[torch.from_numpy(c).to("cuda:0") for c in p] for p in q.payload]
    cols = [(t, pay[t][i]) for t in range(n) for i in range(len(pay[t]))]
    cs = gctx.colset(s, cols)
    ps = gctx.summarize_projected(f, [3, 2, 0, 0])
    assert ps.join_size == Q
    rng = np.random.default_rng(5)
    for first in (0, 3 * (1 << 28) + 99, int(rng.integers(1 << 33, Q - WIN)), Q - WIN // 3):
        cnt = min(WIN, Q - first)
        rid = torch.empty(cnt * n, dtype=torch.int64, device="cuda:0")
        assert gctx.desummarize(s, first, cnt, rid) == cnt
        tup = rid.view(cnt, n).cpu().numpy()
        val = torch.empty(cnt * len(cols), dtype=torch.int32, device="cuda:0")
        assert gctx.desummarize_values(s, cs, first, cnt, val) == cnt
        got = val.view(cnt, len(cols)).cpu().numpy()
        exp = np.stack([q.payload[t][i][tup[:, t]] for t in range(n) for i in range(len(q.payload[t]))], axis=1)
        assert np.array_equal(got, exp), first
        pv = torch.empty(cnt * 3, dtype=torch.int32, device="cuda:0")
        assert gctx.desummarize_projected(ps, first, cnt, pv) == cnt
        pexp = np.stack([q.tables[0][0][tup[:, 0]], q.tables[0][1][tup[:, 0]], q.tables[1][1][tup[:, 1]]], axis=1)
        assert np.array_equal(pv.view(cnt, 3).cpu().numpy(), pexp), first
        _say("values and projection window", first, "ok")
