"""Pins for the CPU oracle: values the paper prints, brute force, closed forms,
invariants and metamorphic relations.  None of these re-types the oracle's own
formulas; each would fail on a plausible mistake (dropped term, wrong index,
transposed operand, wrong order)."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

from conftest import load_fig1, load_fig2
from paper_2206_10435_amd import workloads as W


# ---------------------------------------------------------------------------
# Figure 1 / Figure 2 (printed by the paper)
# ---------------------------------------------------------------------------

def test_fig1_join_size_and_gfjs(oracle_mod):
    q = load_fig1()
    o = oracle_mod.Oracle(q)
    gfjs, rows, facts = load_fig2()
    Q, ovf = o.join_size()
    assert not ovf
    assert Q == sum(f for _, f in gfjs["A"]) == facts["a3_in_result"] == 32
    res = o.canonical_result()
    assert res.shape == (32, 3)
    # values of the sorted result, columns (A, B, C, D)
    A = q.tables[0][0][res[:, 0]]
    B = q.tables[0][1][res[:, 0]]
    C = q.tables[1][1][res[:, 1]]
    D = q.tables[2][1][res[:, 2]]
    for first, last, a, b, c, d in rows:
        sl = slice(first, last + 1)
        assert (A[sl] == a).all() and (B[sl] == b).all() and (C[sl] == c).all() and (D[sl] == d).all()
    runs = o.gfjs(res)
    for col, (vals, freqs) in zip("ABCD", runs):
        assert list(zip(vals.tolist(), freqs.tolist())) == gfjs[col], col


def test_fig1_uir_and_redundancy(oracle_mod):
    q = load_fig1()
    _, _, facts = load_fig2()
    t1b, t2b = q.tables[0][1], q.tables[1][0]
    # T1 join T2 on b0/b1: intermediate tuples that never reach the result
    uir = sum(int((t1b == b).sum()) * int((t2b == b).sum()) for b in (0, 1))
    assert uir == facts["uir"]
    assert int((q.tables[0][0] == 3).sum()) == facts["a3_in_T1"]
    o = oracle_mod.Oracle(q)
    res = o.materialize()
    # no result tuple uses the b0/b1 rows of T1 (rows 0..5)
    assert (res[:, 0] >= 6).all()


# ---------------------------------------------------------------------------
# Brute force on tiny random acyclic queries
# ---------------------------------------------------------------------------

def _tiny_queries():
    out = []
    for seed in range(14):
        n = 2 + seed % 4
        maxr = {2: 30, 3: 14, 4: 8, 5: 6}[n]
        out.append(W.random_tree_query(seed, n, maxr, domain=2 + seed % 3, s=0.5 * (seed % 3),
                                       allow_empty=(seed % 7 == 6), min_rows=maxr // 2,
                                       max_extra_cols=1))
    return out


def _subtree(q, t):
    ch = [[] for _ in range(q.n_tables)]
    for j in range(1, q.n_tables):
        ch[q.parent[j]].append(j)
    out, st = [], [t]
    while st:
        x = st.pop()
        out.append(x)
        st.extend(ch[x])
    return sorted(out)


@pytest.mark.parametrize("q", _tiny_queries(), ids=lambda q: q.name)
def test_bruteforce_matches_materialize_and_counts(oracle_mod, q):
    o = oracle_mod.Oracle(q)
    bf = o.brute_force()
    mat = o.materialize()
    Q, ovf = o.join_size()
    assert not ovf
    assert Q == len(bf) == len(mat)
    # both enumerate in lexicographic row-id order
    assert np.array_equal(bf, mat)
    n = q.n_tables
    for t in range(n):
        fan = o.fanouts(t)
        expect = np.bincount(bf[:, t], minlength=q.n_rows(t)) if len(bf) else np.zeros(q.n_rows(t), int)
        assert np.array_equal(fan, expect)
    # entry-level U, D, F by projection counting: tuples through row r factor
    # into (completions of r's subtree) x (completions of the rest)
    for t in range(n):
        sub = _subtree(q, t)
        rest = [j for j in range(n) if j not in sub]
        summ = o.summary_table(t)
        fac = o.factor(t)
        k = len(q.tables[t])
        keys_by_row = np.stack([q.tables[t][c] for c in range(k)], axis=1) if q.n_rows(t) else None
        for e in range(len(summ["c"])):
            rows_e = np.nonzero((keys_by_row == summ["keys"][e]).all(axis=1))[0]
            assert len(rows_e) == summ["c"][e]
            r0 = rows_e[0]
            sel = bf[bf[:, t] == r0]
            below = {tuple(x) for x in sel[:, sub]}
            outside = {tuple(x) for x in sel[:, rest]} if rest else {()}
            assert summ["U"][e] == len(below)
            assert summ["D"][e] == len(outside)
            assert summ["F"][e] == int(np.isin(bf[:, t], rows_e).sum())
        # surviving entries are exactly the factor entries used by the result
        used = set(bf[:, t].tolist())
        n_used_groups = sum(1 for e in range(len(fac["count"]))
                            if used & set(fac["perm"][fac["start"][e]:fac["start"][e] + fac["count"][e]].tolist()))
        assert n_used_groups == len(summ["c"])
    # edges: M(s)*D(s) = number of result tuples whose t-row carries s
    for t in range(1, n):
        ed = o.summary_edge(t)
        sepv = q.tables[t][q.sep_col[t]]
        sub = _subtree(q, t)
        rest = [j for j in range(n) if j not in sub]
        vals_in_res = sepv[bf[:, t]] if len(bf) else np.array([], np.int32)
        assert sorted(set(vals_in_res.tolist())) == ed["s"].tolist()
        for s, M, D in zip(ed["s"], ed["M"], ed["D"]):
            sel = bf[vals_in_res == s]
            assert M == len({tuple(x) for x in sel[:, sub]})
            assert D == len({tuple(x) for x in sel[:, rest]})
            assert M * D == len(sel)


@pytest.mark.parametrize("q", _tiny_queries(), ids=lambda q: q.name)
def test_canonical_order_unrank_rank(oracle_mod, q):
    o = oracle_mod.Oracle(q)
    res = o.canonical_result()
    n = q.n_tables
    # sorted by attribute values (signed), then row ids
    cols = []
    for t in range(n):
        for c in range(len(q.tables[t])):
            if t == 0 or c != q.sep_col[t]:
                cols.append(q.tables[t][c][res[:, t]].astype(np.int64))
    keyrows = [tuple(int(col[i]) for col in cols) + tuple(int(x) for x in res[i]) for i in range(len(res))]
    assert keyrows == sorted(keyrows)
    assert len(set(keyrows)) == len(keyrows)
    for R in range(len(res)):
        assert np.array_equal(o.unrank(R), res[R])
        assert o.rank(res[R]) == R
    with pytest.raises(IndexError):
        o.unrank(len(res))
    # GFJS invariant: every column's frequencies sum to the join size
    for vals, freqs in o.gfjs(res):
        assert int(freqs.sum()) == len(res)


# ---------------------------------------------------------------------------
# Closed forms (textbook linear algebra, independent of the oracle)
# ---------------------------------------------------------------------------

def _count_matrix(x, y, dom, off):
    C = np.zeros((dom, dom), dtype=np.int64)
    np.add.at(C, (x.astype(np.int64) + off, y.astype(np.int64) + off), 1)
    return C


@pytest.mark.parametrize("n,N,dom", [(2, 3000, 50), (3, 2000, 40), (4, 1500, 30)])
def test_chain_closed_form(oracle_mod, n, N, dom):
    q = W.chain_query(7 + n, 0, n, N, dom, 0.7)
    o = oracle_mod.Oracle(q)
    Cs = [_count_matrix(q.tables[t][0], q.tables[t][1], dom, 0) for t in range(n)]
    one = np.ones(dom, dtype=np.int64)
    left = [one]
    for t in range(n):
        left.append(left[-1] @ Cs[t])
    right = [one]
    for t in reversed(range(n)):
        right.append(Cs[t] @ right[-1])
    right = right[::-1]  # right[t] = C_t ... C_{n-1} 1
    Q, _ = o.join_size()
    assert Q == int(left[n].sum())
    # F_t(x, y) = (1^T C_0..C_{t-1})[x] * C_t[x,y] * (C_{t+1}..C_{n-1} 1)[y]
    for t in range(n):
        s = o.summary_table(t)
        for (x, y), F, c in zip(s["keys"], s["F"], s["c"]):
            assert F == left[t][x] * Cs[t][x, y] * right[t + 1][y]
            assert c == Cs[t][x, y]
        nz = (left[t][:, None] * Cs[t] * right[t + 1][None, :]) > 0
        assert int(nz.sum()) == len(s["F"])


def test_two_table_closed_form(oracle_mod):
    q = W.chain_query(3, 0, 2, [5000, 7000], 300, 1.1)
    o = oracle_mod.Oracle(q)
    b1 = np.bincount(q.tables[0][1], minlength=300)
    b2 = np.bincount(q.tables[1][0], minlength=300)
    assert o.join_size()[0] == int(b1 @ b2)


def test_star_closed_form(oracle_mod):
    q = W.star_query(5, 0, 4, [4000, 900, 800, 700], 60, 0.8)
    o = oracle_mod.Oracle(q)
    hs = [np.bincount(q.tables[i][0], minlength=60) for i in range(1, 4)]
    centre = q.tables[0]
    expect = sum(int(hs[0][centre[0][r]]) * int(hs[1][centre[1][r]]) * int(hs[2][centre[2][r]])
                 for r in range(len(centre[0])))
    assert o.join_size()[0] == expect


# ---------------------------------------------------------------------------
# Metamorphic relations
# ---------------------------------------------------------------------------

def _summary(o, q):
    return [o.summary_table(t) for t in range(q.n_tables)], [o.summary_edge(t) for t in range(1, q.n_tables)]


def _eq_summ(a, b):
    for x, y in zip(a[0], b[0]):
        for k in x:
            assert np.array_equal(x[k], y[k]), k
    for x, y in zip(a[1], b[1]):
        for k in x:
            assert np.array_equal(x[k], y[k]), k


def test_row_shuffle_invariance(oracle_mod):
    q = W.random_tree_query(21, 4, 200, 12, s=0.8)
    o = oracle_mod.Oracle(q)
    rng = np.random.default_rng(1)
    perms = [rng.permutation(q.n_rows(t)) for t in range(q.n_tables)]
    q2 = W.Query("shuf", [[c[p] for c in tb] for tb, p in zip(q.tables, perms)], q.parent, q.sep_col, q.parent_col)
    o2 = oracle_mod.Oracle(q2)
    _eq_summ(_summary(o, q), _summary(o2, q2))
    # row ids map through the permutations
    for t in range(q.n_tables):
        f1, f2 = o.fanouts(t), o2.fanouts(t)
        assert np.array_equal(f2, f1[perms[t]])


def test_duplicate_rows_doubles(oracle_mod):
    q = W.random_tree_query(22, 4, 150, 10, s=0.5)
    o = oracle_mod.Oracle(q)
    t = 2
    q2 = W.Query("dup", [[np.concatenate([c, c]) if i == t else c for c in tb] for i, tb in enumerate(q.tables)],
                 q.parent, q.sep_col, q.parent_col)
    o2 = oracle_mod.Oracle(q2)
    assert o2.join_size()[0] == 2 * o.join_size()[0]
    s1, s2 = o.summary_table(t), o2.summary_table(t)
    assert np.array_equal(s2["c"], 2 * s1["c"])
    assert np.array_equal(s2["F"], 2 * s1["F"])


def test_dangling_rows_leave_summary(oracle_mod):
    q = W.random_tree_query(23, 4, 150, 10, s=0.5)
    o = oracle_mod.Oracle(q)
    # rows whose keys are outside every domain value never join
    q2 = W.Query("dangle", [[np.concatenate([c, np.full(37, 10**6 + 7 * i + j, np.int32)])
                             for j, c in enumerate(tb)] for i, tb in enumerate(q.tables)],
                 q.parent, q.sep_col, q.parent_col)
    o2 = oracle_mod.Oracle(q2)
    _eq_summ(_summary(o, q), _summary(o2, q2))


def test_overflow_aligned(oracle_mod):
    # 6-chain of 1e5 rows over 10 values: about 1e25 tuples, beyond int64
    q = W.chain_query(11, 0, 6, 100_000, 10, 0.0)
    o = oracle_mod.Oracle(q)
    _, ovf = o.join_size()
    assert ovf
    q = W.chain_query(11, 0, 3, 1000, 10, 0.0)
    assert not oracle_mod.Oracle(q).join_size()[1]


# ---------------------------------------------------------------------------
# Weighted join size (exact rational arithmetic on the brute-force result)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_weighted_against_exact_rationals(oracle_mod, seed):
    q = W.random_tree_query(30 + seed, 3 + seed % 2, 10, 4, s=0.6)
    o = oracle_mod.Oracle(q)
    rng = np.random.default_rng(seed)
    w = [rng.uniform(0.5, 2.0, q.n_rows(t)) for t in range(q.n_tables)]
    bf = o.brute_force()
    Wexact = Fraction(0)
    grads = [[Fraction(0)] * q.n_rows(t) for t in range(q.n_tables)]
    for tup in bf:
        ws = [Fraction(float(w[t][r])) for t, r in enumerate(tup)]
        prod = Fraction(1)
        for x in ws:
            prod *= x
        Wexact += prod
        for t, r in enumerate(tup):
            grads[t][r] += prod / ws[t]
    Wo, go = o.weighted(w)
    assert abs(Fraction(Wo) - Wexact) <= abs(Wexact) * Fraction(1, 10**15)
    for t in range(q.n_tables):
        for r in range(q.n_rows(t)):
            assert abs(Fraction(float(go[t][r])) - grads[t][r]) <= abs(grads[t][r]) * Fraction(1, 10**15)
    # unit weights give the join size
    assert o.weighted(None)[0] == float(len(bf))


def test_weighted_invariants_and_fd(oracle_mod):
    q = W.chain_query(41, 0, 4, 2000, 60, 1.0)
    o = oracle_mod.Oracle(q)
    rng = np.random.default_rng(5)
    w = [rng.uniform(0.5, 2.0, q.n_rows(t)) for t in range(4)]
    Wv, g = o.weighted(w)
    # Euler: W is linear in each table's weights, so sum_r w_r dW/dw_r = W
    for t in range(4):
        assert abs(float(np.dot(w[t], g[t])) - Wv) <= 1e-12 * Wv
    # scaling one table's weights by 2^k scales W by 2^k exactly
    w2 = [x.copy() for x in w]
    w2[1] *= 8.0
    assert o.weighted(w2, grads=False)[0] == 8.0 * Wv
    # central finite differences have no truncation error (multilinear)
    rows = rng.choice(q.n_rows(2), 25, replace=False)
    fd = o.weighted_fd(w, 2, rows, threads=4)
    ref = g[2][rows]
    nz = ref != 0
    assert np.all(np.abs(fd[nz] - ref[nz]) <= 1e-13 * np.abs(ref[nz]))
    assert np.all(fd[~nz] == 0)


def test_star_plus_chain_closed_forms(oracle_mod):
    """Foreign keys into primary keys plus a many-to-many bridge: join size,
    every row's fan-out and the rank of every result tuple in closed form."""
    q = W.cfg3(fact_rows=60_000, dim_rows=(2_000, 300, 500, 700), bridge_rows=20_000, bridge_domain=1_500)
    o = oracle_mod.Oracle(q)
    res = o.canonical_result()
    F, D1, B = q.tables[0], q.tables[1], q.tables[5]
    nf, dom = q.n_rows(0), 1_500
    cntB = np.bincount(B[0], minlength=dom).astype(np.int64)
    d1row = np.empty(q.n_rows(1), dtype=np.int64)
    d1row[D1[0]] = np.arange(q.n_rows(1))
    fan_f = cntB[D1[1][d1row[F[0]]]]
    assert o.join_size()[0] == int(fan_f.sum()) == len(res)
    order = np.lexsort((np.arange(nf), F[3], F[2], F[1], F[0]))
    start = np.empty(nf, dtype=np.int64)
    start[order] = np.concatenate([[0], np.cumsum(fan_f[order])[:-1]])
    ordB = np.argsort(B[0], kind="stable")
    gstart = np.searchsorted(B[0][ordB], np.arange(dom))
    pos = np.empty(q.n_rows(5), dtype=np.int64)
    pos[ordB] = np.arange(q.n_rows(5)) - gstart[B[0][ordB]]
    assert np.array_equal(start[res[:, 0]] + pos[res[:, 5]], np.arange(len(res)))
    cnt_k1 = np.bincount(F[0], minlength=q.n_rows(1)).astype(np.int64)
    assert np.array_equal(o.fanouts(0), fan_f)
    assert np.array_equal(o.fanouts(1), cnt_k1[D1[0]] * cntB[D1[1]])
    for i in (2, 3, 4):
        fi = np.rint(np.bincount(F[i - 1], weights=fan_f.astype(float), minlength=q.n_rows(i))).astype(np.int64)
        assert np.array_equal(o.fanouts(i), fi[q.tables[i][0]])


def test_reroot_invariance(oracle_mod):
    """Any table can be the root: join size, weighted size and every row's
    gradient are unchanged (only the result order changes)."""
    q = W.random_tree_query(41, 5, 400, 30, s=0.7, max_extra_cols=1, min_rows=200)
    rng = np.random.default_rng(2)
    w = [rng.uniform(0.5, 2.0, q.n_rows(t)) for t in range(q.n_tables)]
    o = oracle_mod.Oracle(q)
    W0, g0 = o.weighted(w)
    for r in range(q.n_tables):
        qr, order = W.reroot(q, r)
        orr = oracle_mod.Oracle(qr)
        assert orr.join_size() == o.join_size()
        Wr, gr = orr.weighted([w[t] for t in order])
        assert abs(Wr - W0) <= 1e-13 * W0
        for k, t in enumerate(order):
            assert np.allclose(gr[k], g0[t], rtol=1e-13, atol=0)
            assert np.array_equal(orr.fanouts(k), o.fanouts(t))


def test_check_tuples_accepts_sorted_result_and_rejects_corruptions(oracle_mod):
    """The chunk checker (every tuple a join tuple, strictly increasing in the
    result order) accepts the brute-force result sorted by (values, row ids)
    in Python, and names the first bad tuple of a swapped pair, a duplicate,
    a row id out of range and a tuple that breaks a join edge."""
    checked = 0
    for q in [load_fig1()] + _tiny_queries():
        o = oracle_mod.Oracle(q)
        bf = o.brute_force().astype(np.int64)
        if len(bf) < 4:
            continue
        n = q.n_tables
        cols = [(t, c) for t in range(n) for c in range(len(q.tables[t])) if t == 0 or c != q.sep_col[t]]
        key = lambda r: tuple(int(q.tables[t][c][r[t]]) for t, c in cols) + tuple(int(x) for x in r)
        ref = np.array(sorted(bf.tolist(), key=key), dtype=np.int64)
        for threads in (1, 3):
            assert o.check_tuples(ref, threads) == -1
        sw = ref.copy()
        sw[[1, 2]] = sw[[2, 1]]
        assert o.check_tuples(sw, 2) == 2
        dup = ref.copy()
        dup[3] = dup[2]
        assert o.check_tuples(dup, 2) == 3
        oob = ref.copy()
        oob[1, n - 1] = q.n_rows(n - 1)
        assert o.check_tuples(oob, 2) == 1
        # a row of the last table whose separator value differs from the one its tuple needs
        t = n - 1
        if n > 1:
            need = q.tables[q.parent[t]][q.parent_col[t]][ref[2, q.parent[t]]]
            other = np.nonzero(q.tables[t][q.sep_col[t]] != need)[0]
            if len(other):
                brk = ref.copy()
                brk[2, t] = other[0]
                assert o.check_tuples(brk, 2) == 2
        checked += 1
    assert checked >= 8


@pytest.mark.parametrize("q", _tiny_queries()[:8], ids=lambda q: q.name)
def test_materialize_ranges_partition_the_brute_force_result(oracle_mod, q):
    """The range DFS (the threaded CPU baseline) against brute force: the
    tuples of root rows [lo, hi) are exactly the brute-force tuples whose
    root row lies there, and cut points in any place split the result."""
    o = oracle_mod.Oracle(q)
    bf = o.brute_force()
    n0 = q.n_rows(0)
    for cuts in ([0, n0], [0, n0 // 2, n0], [0, 1, n0 // 3, n0 - 1, n0]):
        cuts = sorted(set(max(0, min(n0, c)) for c in cuts))
        parts = [o.materialize_range(a, b, 10**6) for a, b in zip(cuts, cuts[1:])]
        for (a, b), p in zip(zip(cuts, cuts[1:]), parts):
            assert np.array_equal(p, bf[(bf[:, 0] >= a) & (bf[:, 0] < b)]) if len(bf) else len(p) == 0
    for T in (1, 3):
        got = o.materialize_threads(10**6 * T, T)
        assert np.array_equal(np.concatenate(got) if got else bf[:0], bf)
    # the limit cuts each range's output in DFS order
    if len(bf) > 2:
        p = o.materialize_range(0, n0, 2)
        assert np.array_equal(p, bf[:2])
