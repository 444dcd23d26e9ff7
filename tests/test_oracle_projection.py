"""Pins for the oracle's early projections (Sec. 3.7): the projected result is
every join result tuple restricted to the output attributes, multiplicities
kept, sorted by all of them.  Pinned by the paper's Figure 2 (its leading GFJS
columns are the GFJS of the projections onto those leading attributes), brute
force on tiny random queries, the identity projection and re-rooting."""
import collections

import numpy as np
import pytest

from conftest import load_fig1, load_fig2
from paper_2206_10435_amd import workloads as W


def _runs(vals):
    """Definition 1 per prefix: for column i, one (value, length) run per
    maximal block of rows with equal columns 0..i."""
    out = []
    for i in range(vals.shape[1]):
        runs = []
        for r in range(vals.shape[0]):
            if r > 0 and (vals[r, : i + 1] == vals[r - 1, : i + 1]).all():
                runs[-1][1] += 1
            else:
                runs.append([int(vals[r, i]), 1])
        out.append([tuple(x) for x in runs])
    return out


def _all_mask(q):
    return [(1 << len(tb)) - 1 for tb in q.tables]


@pytest.mark.parametrize("cols", ["AB", "ABC", "ABCD", "A"])
def test_fig2_leading_columns(oracle_mod, cols):
    """Projecting Figure 1's join onto A, (A, B), (A, B, C) keeps the leading
    GFJS columns Figure 2 prints (the runs of a column depend only on the
    columns before it); with A alone, one run of 32."""
    q = load_fig1()
    o = oracle_mod.Oracle(q)
    gfjs, _, _ = load_fig2()
    # A = T1.0, B = T1.1 (= T2.0), C = T2.1 (= T3.0), D = T3.1
    bits = {"A": (0, 0), "B": (0, 1), "C": (1, 1), "D": (2, 1)}
    mask = [0, 0, 0]
    for ch in cols:
        t, c = bits[ch]
        mask[t] |= 1 << c
    ok, _, _ = o.projection(mask)
    assert ok
    res = o.projected_result(mask)
    assert res.shape == (32, len(cols))
    runs = _runs(res)
    for i, ch in enumerate(cols):
        assert runs[i] == gfjs[ch], ch


def test_fig1_projected_tables(oracle_mod):
    """(A, B): T2 and T3 are deleted, T1's entries carry their completions:
    c(a3, b3) = 2 rows x 4, c(a3, b4) = 4 rows x 6 (the B messages derived by
    hand from Figure 1)."""
    q = load_fig1()
    o = oracle_mod.Oracle(q)
    ok, m, kept = o.projection([3, 0, 0])
    assert ok and kept.tolist() == [True, False, False]
    r = o.projected_table([3, 0, 0], 0)
    assert r["keys"].tolist() == [[3, 3], [3, 4]]
    assert r["c"].tolist() == [8, 24] and r["F"].tolist() == [8, 24]
    assert r["U"].tolist() == [1, 1] and r["D"].tolist() == [1, 1]


def test_unsupported(oracle_mod):
    q = load_fig1()
    o = oracle_mod.Oracle(q)
    assert not o.projection([0, 0, 0])[0]      # nothing to output
    assert not o.projection([0, 0, 2])[0]      # D alone: T3 kept, its separator C summed out
    assert not o.projection([1, 0, 2])[0]      # A and D: T1 - T3 linked through B, C
    assert not o.projection([0, 2, 0])[0]      # C alone: T2 kept, its separator B summed out
    assert o.projection([2, 2, 0])[0]          # B and C: T1 (B) - T2 (C) on output B


def test_identity_projection(oracle_mod):
    """Every attribute output: the projected summary is the summary, except
    that a table whose only column is its separator adds no column and is
    folded into its parent (c * U unchanged, so F is unchanged)."""
    full_kept = folded = 0
    for seed in range(16):
        q = W.random_tree_query(40 + seed, 2 + seed % 4, 12, 3, s=0.5, min_rows=5, max_extra_cols=1)
        o = oracle_mod.Oracle(q)
        mask = _all_mask(q)
        ok, _, kept = o.projection(mask)
        assert ok
        full_kept += bool(kept.all())
        for t in range(q.n_tables):
            if not kept[t]:
                assert len(q.tables[t]) == 1
                folded += 1
                continue
            a, b = o.projected_table(mask, t), o.summary_table(t)
            for k in ("keys", "D", "F"):
                assert np.array_equal(a[k], b[k]), (seed, t, k)
            assert np.array_equal(a["c"] * a["U"], b["c"] * b["U"]), (seed, t)
            if all(kept[j] for j in range(1, q.n_tables) if q.parent[j] == t):
                assert np.array_equal(a["c"], b["c"]) and np.array_equal(a["U"], b["U"]), (seed, t)
    assert full_kept >= 3 and folded >= 1


def _random_masks(q, rng, count):
    out = []
    for _ in range(count * 6):
        m = [int(rng.integers(0, 1 << len(tb))) for tb in q.tables]
        out.append(m)
    return out


def test_brute_force(oracle_mod):
    """Projected result and per-entry run lengths against the projected
    brute-force result; c * U * D = F; run lengths sum to the join size."""
    checked = 0
    for seed in range(12):
        n = 2 + seed % 4
        q = W.random_tree_query(60 + seed, n, {2: 20, 3: 10, 4: 7, 5: 5}[n], 2 + seed % 3, s=0.5,
                                min_rows=3, max_extra_cols=1)
        o = oracle_mod.Oracle(q)
        bf = o.brute_force()
        Q, _ = o.join_size()
        rng = np.random.Generator(np.random.PCG64(seed))
        for mask in _random_masks(q, rng, 4):
            ok, mn, kept = o.projection(mask)
            if not ok:
                continue
            cols = o.projected_columns(mask)
            exp = collections.Counter(tuple(int(q.tables[t][c][r[t]]) for t, c in cols) for r in bf)
            res = o.projected_result(mask)
            assert collections.Counter(map(tuple, res.tolist())) == exp
            assert all(tuple(res[i]) <= tuple(res[i + 1]) for i in range(len(res) - 1))
            for t in range(n):
                if not kept[t]:
                    continue
                r = o.projected_table(mask, t)
                assert np.array_equal(r["c"] * r["U"] * r["D"], r["F"])
                assert int(r["F"].sum()) == Q
                ocols = [c for c in range(len(q.tables[t])) if (int(mn[t]) >> c) & 1]
                cnt = collections.Counter(tuple(int(q.tables[t][c][row[t]]) for c in ocols) for row in bf)
                got = {tuple(k): int(f) for k, f in zip(r["keys"].tolist(), r["F"].tolist())}
                assert got == dict(cnt), (seed, mask, t)
            checked += 1
    assert checked >= 20


def test_reroot_makes_projection_supported(oracle_mod):
    """(C, D) cannot be projected with T1 as the root (T3's separator C links
    it to T1 through B); rooted at T3 it can, and the result is the same bag."""
    q = load_fig1()
    o = oracle_mod.Oracle(q)
    assert not o.projection([0, 0, 2])[0]
    qr, order = W.reroot(q, 2)
    orr = oracle_mod.Oracle(qr)
    pos = {t: i for i, t in enumerate(order)}
    mask = [0] * 3
    mask[pos[2]] = 3  # C and D of T3
    ok, _, _ = orr.projection(mask)
    assert ok
    res = orr.projected_result(mask)
    full = o.canonical_result()
    exp = sorted(zip(q.tables[2][0][full[:, 2]].tolist(), q.tables[2][1][full[:, 2]].tolist()))
    assert sorted(map(tuple, res.tolist())) == exp
