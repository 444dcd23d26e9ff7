"""Full-size parity with the CPU oracle, element by element where the oracle
can compute the whole answer:

* the 4-table chain (4 x 1e7 rows, Zipf(1.1) over 1e5): every surviving entry
  (keys, c, U, D, F, block offset) and every edge (s, M, D) of the summary;
  the whole first 2^28-tuple chunk and a whole seeded chunk beyond 2^33 --
  every tuple a join tuple, strictly increasing in the result order, and the
  oracle's rank of both ends equal to their positions;
* the star plus chain (fact table 5e7 rows, 128-bit sort words): the whole
  summary, and the whole result (both chunks, 4.5e8 tuples) valid and
  strictly increasing with exactly the oracle's join size of tuples, i.e. the
  sorted result itself;
* the weighted chain (4 x 1e6 rows): gradients of 1,000 seeded rows (250 per
  table) against central finite differences of W evaluated in __float128;
* the 256-query batch at its full sizes: every join size and status against
  the oracle's (stored by tests/golden/make_batch_queries.py), and the whole
  summaries of the largest queries and of a seeded sample; a batch of
  overflowing and ordinary queries reports each query's status.
"""
import concurrent.futures as cf
import os

import numpy as np
import pytest

from paper_2206_10435_amd import workloads as W

pytestmark = pytest.mark.gpu

CHUNK = 1 << 28
THREADS = max(1, min(16, os.cpu_count() or 1))
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def gctx():
    from paper_2206_10435_amd import gj

    return gj.Context(0)


def _pre_expected(keys_sep, c, U):
    """Exclusive prefix of c*U inside each run of equal separator values."""
    cu = c * U
    if len(cu) == 0:
        return cu
    heads = np.r_[True, keys_sep[1:] != keys_sep[:-1]]
    incl = np.cumsum(cu)
    gidx = np.cumsum(heads) - 1
    base = (incl - cu)[heads][gidx]
    return incl - cu - base


def _compare_summary(s, o, q):
    """Every table's surviving entries and every edge, element by element."""
    n = q.n_tables

    def ref_table(t):
        return t, o.summary_table(t), (o.summary_edge(t) if t else None)

    with cf.ThreadPoolExecutor(max_workers=min(n, THREADS)) as ex:
        refs = {t: (r, e) for t, r, e in ex.map(ref_table, range(n))}
    for t in range(n):
        g, (r, re_) = s.table(t), refs[t]
        for k in ("keys", "c", "U", "D", "F"):
            assert np.array_equal(g[k], r[k]), f"summary {k} t={t}"
        sep = np.zeros(len(g["c"]), np.int64) if t == 0 else g["keys"][:, q.sep_col[t]].astype(np.int64)
        assert np.array_equal(g["pre"], _pre_expected(sep, g["c"], g["U"])), f"summary pre t={t}"
        if t:
            ge = s.edge(t)
            for k in ("s", "M", "D"):
                assert np.array_equal(ge[k], re_[k]), f"edge {k} t={t}"
        _say(f"  table {t}: {len(g['c'])} entries identical")


def _chunk(gctx, s, n, first, count):
    import torch

    out = torch.empty(count * n, dtype=torch.int64, device="cuda:0")
    nw = gctx.desummarize(s, first, count, out)
    assert nw == min(count, s.join_size - first)
    host = out[: nw * n].view(nw, n).cpu().numpy()
    del out
    torch.cuda.empty_cache()
    return host


def test_chain4_summary_and_whole_chunks(gctx, oracle_mod):
    from paper_2206_10435_amd import gj

    q = W.cfg2(payload=False)
    _say("chain4: oracle counting")
    o = oracle_mod.Oracle(q)
    Q, ovf = o.join_size()
    assert not ovf
    f = gctx.build_factors(gj.to_device_tables(q), q.parent, q.sep_col, q.parent_col)
    s = gctx.summarize(f)
    assert s.join_size == Q
    _say("chain4: join size", Q, "; comparing the whole summary")
    _compare_summary(s, o, q)
    n = q.n_tables
    rng = np.random.default_rng(20220621)
    deep = int(rng.integers(1 << 33, Q - CHUNK)) // CHUNK * CHUNK
    for first in (0, deep):
        _say(f"chain4: chunk at {first}: expanding {CHUNK} tuples")
        tup = _chunk(gctx, s, n, first, CHUNK)
        assert len(tup) == CHUNK
        _say("  checking every tuple with the oracle")
        assert o.check_tuples(tup, THREADS) == -1, first
        _say("  ranking both ends")
        assert o.rank(tup[0].astype(np.int32)) == first
        assert o.rank(tup[-1].astype(np.int32)) == first + CHUNK - 1
        del tup
        _say(f"  chunk at {first} ok")


def test_star_summary_and_whole_result(gctx, oracle_mod):
    from paper_2206_10435_amd import gj

    q = W.cfg3()
    _say("star: oracle counting")
    o = oracle_mod.Oracle(q)
    Q, ovf = o.join_size()
    assert not ovf
    f = gctx.build_factors(gj.to_device_tables(q), q.parent, q.sep_col, q.parent_col)
    s = gctx.summarize(f)
    assert s.join_size == Q
    _say("star: join size", Q, "; comparing the whole summary")
    _compare_summary(s, o, q)
    n = q.n_tables
    prev_last = None
    total = 0
    for first in range(0, Q, CHUNK):
        _say(f"star: chunk at {first}")
        tup = _chunk(gctx, s, n, first, CHUNK)
        assert o.check_tuples(tup, THREADS) == -1, first
        if prev_last is not None:
            assert o.check_tuples(np.stack([prev_last, tup[0]]), 1) == -1, "chunk boundary"
        else:
            assert o.rank(tup[0].astype(np.int32)) == 0
        prev_last = tup[-1].copy()
        total += len(tup)
        del tup
    assert total == Q
    _say("star: whole result ok,", total, "tuples")


def test_weighted_gradients_1000_rows_against_fd(gctx, oracle_mod):
    """dW/dw for 250 seeded rows of every table against central finite
    differences of W in __float128 (W is multilinear in each weight, so the
    difference quotient is exact up to the float128 rounding): relative error
    at most 1e-12, and exactly 0 where the row's fan-out is 0."""
    import torch

    from paper_2206_10435_amd import gj

    q, w64, _ = W.cfg4()
    o = oracle_mod.Oracle(q)
    dev = "cuda:0"
    f = gctx.build_factors(gj.to_device_tables(q), q.parent, q.sep_col, q.parent_col)
    ws = [torch.from_numpy(w).to(dev) for w in w64]
    Wv, st = gctx.weighted_forward(f, ws)
    grads = [torch.empty_like(w) for w in ws]
    gctx.weighted_backward(st, torch.ones((), dtype=torch.float64, device=dev), grads)
    rng = np.random.default_rng(1000)
    worst = 0.0
    zeros = 0
    for t in range(q.n_tables):
        rows = np.sort(rng.choice(q.n_rows(t), 250, replace=False))
        _say(f"weighted: table {t}: finite differences of 250 rows on {THREADS} threads")
        fd = o.weighted_fd(w64, t, rows, hfrac=0.25, threads=THREADS)
        g = grads[t].cpu().numpy()[rows]
        nz = fd != 0
        zeros += int((~nz).sum())
        assert (g[~nz] == 0).all(), t
        rel = np.abs(g[nz] - fd[nz]) / np.abs(fd[nz])
        worst = max(worst, float(rel.max()) if nz.any() else 0.0)
        assert (rel <= 1e-12).all(), (t, float(rel.max()))
    _say(f"weighted: 1000 rows, worst relative error {worst:.3e}, {zeros} zero fan-outs")


def _kept_queries():
    kept, rejected = {}, 0
    with open(os.path.join(GOLDEN, "batch_queries.txt")) as fh:
        for line in fh:
            p = line.split()
            if not p or p[0].startswith("#"):
                continue
            if p[0] == "kept":
                kept[int(p[1])] = (int(p[2]), int(p[3]))
            elif p[0] == "rejected":
                rejected += 1
    return kept, rejected


def test_batch_256_queries_full_size(gctx, oracle_mod):
    from paper_2206_10435_amd import gj

    kept, rejected = _kept_queries()
    assert len(kept) == 256
    _say(f"batch: 256 queries ({rejected} draws rejected for join sizes >= 2^62)")
    qs = W.cfg5(attempts=[kept[i][0] for i in range(256)])
    qd = [dict(tables=gj.to_device_tables(q), parent=q.parent, sep_col=q.sep_col,
               parent_col=q.parent_col) for q in qs]
    b = gctx.batch_create(qd)
    for rep in range(3):
        b.launch(graph=True)
        js, stt = b.results()
        assert (stt == gj.GJ_OK).all(), rep
        assert js.tolist() == [kept[i][1] for i in range(256)], rep
    _say("batch: every join size and status equals the oracle's (3 replays)")
    rows = [q.total_rows() for q in qs]
    largest = list(np.argsort(rows)[-6:])
    sample = sorted(set(largest) | set(np.random.default_rng(5).choice(256, 10, replace=False).tolist()))
    for i in sample:
        q = qs[i]
        _say(f"batch: query {i} ({q.name}, {rows[i]} rows): whole summary")
        o = oracle_mod.Oracle(q)
        _compare_summary(b.summary(i), o, q)
        o.close()


def test_batch_overflow_set(gctx, oracle_mod):
    """Queries whose join size overflows 2^63-1 among ordinary ones: each
    query's status and join size as the oracle says, in one graph."""
    from paper_2206_10435_amd import gj

    qs = []
    for k in range(6):
        if k % 2 == 0:
            qs.append(W.chain_query(11 + k, 0, 6, 100_000, 10, 0.0, name=f"ovf{k}"))
        else:
            qs.append(W.cfg5_query(k))
    qd = [dict(tables=gj.to_device_tables(q), parent=q.parent, sep_col=q.sep_col, parent_col=q.parent_col)
          for q in qs]
    b = gctx.batch_create(qd)
    b.launch(graph=True)
    js, stt = b.results()
    for i, q in enumerate(qs):
        Q, ovf = oracle_mod.Oracle(q).join_size()
        if ovf:
            assert stt[i] == gj.GJ_E_OVERFLOW, i
            with pytest.raises(gj.GJError) as ei:
                b.summary(i)
            assert ei.value.status == gj.GJ_E_OVERFLOW
        else:
            assert stt[i] == gj.GJ_OK and js[i] == Q, i
    assert sum(stt == gj.GJ_E_OVERFLOW) == 3
