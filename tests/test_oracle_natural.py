"""Pins for the oracle's natural joins over named attributes (cyclic queries):
the worked triangle of Sec. 3.2.1, trace closed forms for triangles and
4-cycles, brute force, and agreement with the tree oracle on acyclic queries."""
import numpy as np
import pytest

from paper_2206_10435_amd import workloads as W


def _rng(seed):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 31])))


def _table(rng, n, doms):
    return [rng.integers(0, d, size=n).astype(np.int32) for d in doms]


def _count_matrix(x, y, dx, dy):
    m = np.zeros((dx, dy), dtype=np.int64)
    np.add.at(m, (x, y), 1)
    return m


def test_sec321_triangle_example(oracle_mod):
    """Sec. 3.2.1: entries (a1, b1) x5, (b1, c1) x10, (c1, a1) x20 of T1(A, B),
    T2(B, C), T3(C, A) give the joint entry (a1, b1, c1) with frequency 1000."""
    one = lambda k: np.full(k, 1, np.int32)  # noqa: E731
    T1 = [np.concatenate([one(5), [2, 3]]).astype(np.int32), np.concatenate([one(5), [1, 1]]).astype(np.int32)]
    T2 = [np.concatenate([one(10), [1]]).astype(np.int32), np.concatenate([one(10), [2]]).astype(np.int32)]
    T3 = [one(20), one(20)]
    o = oracle_mod.NaturalOracle([T1, T2, T3], [[0, 1], [1, 2], [2, 0]])
    keys, counts = o.potential([0, 1, 2], [0, 1, 2])
    assert keys.tolist() == [[1, 1, 1]] and counts.tolist() == [1000]
    assert o.join_size() == 1000


@pytest.mark.parametrize("seed", range(6))
def test_triangle_trace(oracle_mod, seed):
    rng = _rng(seed)
    d = 3 + seed
    R, S, T = (_table(rng, 40 + 10 * seed, [d, d]) for _ in range(3))
    o = oracle_mod.NaturalOracle([R, S, T], [[0, 1], [1, 2], [2, 0]])
    mR, mS, mT = (_count_matrix(x[0], x[1], d, d) for x in (R, S, T))
    assert o.join_size() == int(np.trace(mR @ mS @ mT))
    # and the joint potential is the elementwise product R[a,b] S[b,c] T[c,a]
    keys, counts = o.potential([0, 1, 2], [0, 1, 2])
    exp = {(a, b, c): int(mR[a, b] * mS[b, c] * mT[c, a]) for a in range(d) for b in range(d) for c in range(d)
           if mR[a, b] * mS[b, c] * mT[c, a] > 0}
    assert {tuple(k): int(v) for k, v in zip(keys.tolist(), counts.tolist())} == exp


@pytest.mark.parametrize("seed", range(4))
def test_four_cycle_trace(oracle_mod, seed):
    rng = _rng(100 + seed)
    d = 4
    tabs = [_table(rng, 25, [d, d]) for _ in range(4)]
    o = oracle_mod.NaturalOracle(tabs, [[0, 1], [1, 2], [2, 3], [3, 0]])
    m = [_count_matrix(t[0], t[1], d, d) for t in tabs]
    assert o.join_size() == int(np.trace(m[0] @ m[1] @ m[2] @ m[3]))


def test_brute_force(oracle_mod):
    for seed in range(10):
        rng = _rng(200 + seed)
        n = 3 + seed % 3
        nattr = 3 + seed % 3
        tabs, attrs = [], []
        for t in range(n):
            k = 2 + int(rng.integers(0, 2))
            a = [int(x) for x in rng.choice(nattr, size=k, replace=False)]
            attrs.append(a)
            tabs.append(_table(rng, 6, [3] * k))
        o = oracle_mod.NaturalOracle(tabs, attrs)
        bf = o.brute_force()
        mt = o.materialize()
        assert len(bf) == len(mt) == o.join_size()
        assert sorted(map(tuple, bf.tolist())) == sorted(map(tuple, mt.tolist()))


def test_acyclic_agrees_with_tree_oracle(oracle_mod):
    for seed in range(6):
        q = W.random_tree_query(300 + seed, 2 + seed % 4, 30, 5, s=0.5, min_rows=10, max_extra_cols=1)
        # attribute ids: a column joined to its parent shares the parent's attribute
        attrs, nxt = [], 0
        for t in range(q.n_tables):
            a = []
            for c in range(len(q.tables[t])):
                if t > 0 and c == q.sep_col[t]:
                    a.append(attrs[q.parent[t]][q.parent_col[t]])
                else:
                    a.append(nxt)
                    nxt += 1
            attrs.append(a)
        if any(len(set(a)) != len(a) for a in attrs):
            continue
        nat = oracle_mod.NaturalOracle(q.tables, attrs)
        tree = oracle_mod.Oracle(q)
        assert nat.join_size() == tree.join_size()[0]
        order = [a for t in range(q.n_tables) for c, a in enumerate(attrs[t])
                 if t == 0 or c != q.sep_col[t]]
        rows = tree.canonical_result()
        vals = nat.attribute_values(rows, order)
        assert np.array_equal(nat.sorted_values(order), vals)
