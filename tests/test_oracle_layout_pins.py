"""Pins for the layout of two oracle outputs that go beyond plain values.

* The factor of a table (Sec. 3.2: every distinct key tuple with its
  frequency) together with the grouped row ids: entries strictly increasing
  in (separator, then the other columns in declared order) -- the root in
  declared order --, counts summing to the rows, starts the prefix sums of the
  counts, the row list a permutation whose rows carry their entry's keys and
  ascend inside an entry.
* The frequency split of a kept table's projected entries under early
  projections (Sec. 3.7): c' counts the distinct combinations of one of the
  entry's rows with a completion of its deleted children's subtrees, U the
  distinct completions of its kept children's subtrees, D those outside its
  subtree -- each counted separately, by brute force over the join result.

A mutation test plants plausible mistakes in scratch copies of the oracle
source (separator not first, rows descending inside an entry, starts that
are entry indexes, key columns written in sort order instead of declared
order, deleted completions moved into U, a deleted child's outside message
taken for its subtree's) and checks that these pins catch every one of them.
"""
import collections
import concurrent.futures as cf
import os
import shutil
import subprocess

import numpy as np
import pytest

from conftest import load_fig1
from paper_2206_10435_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


# ---------------------------------------------------------------------------
# Factor layout against its definition
# ---------------------------------------------------------------------------

def factor_layout_failures(q, t, fac):
    """Every way the factor of table t departs from its definition (empty if none)."""
    bad = []
    N = q.n_rows(t)
    k = len(q.tables[t])
    keys, cnt, start, perm = fac["keys"], fac["count"], fac["start"], fac["perm"]
    M = len(cnt)
    if not (cnt > 0).all() or int(cnt.sum()) != N:
        bad.append("counts are not positive or do not sum to the rows")
    if not np.array_equal(start, np.concatenate([[0], np.cumsum(cnt)[:-1]]).astype(np.int64)[:M]):
        bad.append("starts are not the exclusive prefix sums of the counts")
    if not np.array_equal(np.sort(perm), np.arange(N, dtype=np.int32)):
        bad.append("row list is not a permutation")
        return bad
    ent = np.repeat(np.arange(M), cnt) if int(cnt.sum()) == N else None
    if ent is not None:
        for c in range(k):
            if not np.array_equal(q.tables[t][c][perm], keys[ent, c]):
                bad.append(f"rows do not carry their entry's key column {c}")
        same = ent[1:] == ent[:-1]
        if not (perm[1:][same] > perm[:-1][same]).all():
            bad.append("rows do not ascend inside an entry")
    order = ([q.sep_col[t]] if t else []) + [c for c in range(k) if t == 0 or c != q.sep_col[t]]
    tup = [tuple(int(keys[e, c]) for c in order) for e in range(M)]
    if any(not (tup[i] < tup[i + 1]) for i in range(M - 1)):
        bad.append("entries are not strictly increasing in (separator, other columns)")
    distinct = {tuple(int(q.tables[t][c][r]) for c in range(k)) for r in range(N)}
    if M != len(distinct):
        bad.append("entry count differs from the number of distinct key tuples")
    return bad


def _layout_queries():
    qs = [load_fig1()]
    for seed in range(10):
        n = 2 + seed % 4
        qs.append(W.random_tree_query(500 + seed, n, 60, 3 + seed % 4, s=0.7, max_extra_cols=3, min_rows=20))
    return qs


def _all_layout_failures(oracle_mod, L=None):
    out = []
    for q in _layout_queries():
        o = oracle_mod.Oracle(q, L)
        for t in range(q.n_tables):
            out += [f"{q.name} t={t}: {m}" for m in factor_layout_failures(q, t, o.factor(t))]
        o.close()
    return out


def test_factor_layout(oracle_mod):
    assert _all_layout_failures(oracle_mod) == []


def test_factor_layout_fig1_values(oracle_mod):
    """Figure 1's factors read off the printed tables: T1 (a, b) with counts
    3, 2, 1, 2, 4; T2 (b, c) with 2, 3, 3, 1, 2, 1; T3 (c, d) with 4, 4, 2, 2
    (the tables are printed sorted, so every row list is the identity)."""
    q = load_fig1()
    o = oracle_mod.Oracle(q)
    exp = {0: ([(0, 0), (1, 1), (2, 1), (3, 3), (3, 4)], [3, 2, 1, 2, 4]),
           1: ([(0, 0), (1, 0), (2, 1), (3, 2), (4, 3), (4, 4)], [2, 3, 3, 1, 2, 1]),
           2: ([(1, 0), (2, 2), (3, 3), (4, 4)], [4, 4, 2, 2])}
    for t, (keys, counts) in exp.items():
        f = o.factor(t)
        assert [tuple(k) for k in f["keys"].tolist()] == keys, t
        assert f["count"].tolist() == counts, t
        assert f["start"].tolist() == np.concatenate([[0], np.cumsum(counts)[:-1]]).tolist(), t
        assert f["perm"].tolist() == list(range(q.n_rows(t))), t


# ---------------------------------------------------------------------------
# Projected c' / U / D split by brute force
# ---------------------------------------------------------------------------

def _children(q):
    ch = [[] for _ in range(q.n_tables)]
    for j in range(1, q.n_tables):
        ch[q.parent[j]].append(j)
    return ch


def _subtree(ch, t):
    out, st = [], [t]
    while st:
        x = st.pop()
        out.append(x)
        st.extend(ch[x])
    return sorted(out)


def projected_split_failures(q, o, bf, mask):
    """Compare every kept table's projected (keys, c', U, D, F) with distinct
    counts over the brute-force result."""
    bad = []
    ok, mn, kept = o.projection(mask)
    if not ok:
        return bad
    ch = _children(q)
    n = q.n_tables
    for t in range(n):
        if not kept[t]:
            continue
        ocols = [c for c in range(len(q.tables[t])) if (int(mn[t]) >> c) & 1]
        dele = sorted(x for c in ch[t] if not kept[c] for x in _subtree(ch, c))
        keep = sorted(x for c in ch[t] if kept[c] for x in _subtree(ch, c))
        inside = set(_subtree(ch, t))
        outside = [x for x in range(n) if x not in inside]
        sets = collections.defaultdict(lambda: (set(), set(), set()))
        F = collections.Counter()
        for row in bf:
            key = tuple(int(q.tables[t][c][row[t]]) for c in ocols)
            a, b, d = sets[key]
            a.add((int(row[t]),) + tuple(int(row[x]) for x in dele))
            b.add(tuple(int(row[x]) for x in keep))
            d.add(tuple(int(row[x]) for x in outside))
            F[key] += 1
        r = o.projected_table(mask, t)
        got = {tuple(k): (int(c), int(u), int(dd), int(f))
               for k, c, u, dd, f in zip(r["keys"].tolist(), r["c"], r["U"], r["D"], r["F"])}
        exp = {k: (len(sets[k][0]), len(sets[k][1]), len(sets[k][2]), F[k]) for k in F}
        if got != exp:
            diff = [k for k in set(got) | set(exp) if got.get(k) != exp.get(k)][:3]
            bad.append(f"{q.name} mask={list(mask)} t={t}: " +
                       "; ".join(f"{k}: got {got.get(k)} expected {exp.get(k)}" for k in diff))
    return bad


def _split_cases():
    cases = []
    for seed in range(14):
        n = 3 + seed % 3
        q = W.random_tree_query(700 + seed, n, {3: 9, 4: 7, 5: 5}[n], 2 + seed % 3, s=0.5, min_rows=3,
                                max_extra_cols=2)
        rng = np.random.Generator(np.random.PCG64(seed))
        masks = [[int(rng.integers(0, 1 << len(tb))) for tb in q.tables] for _ in range(40)]
        cases.append((q, masks))
    return cases


def _all_split_failures(oracle_mod, L=None):
    out, checked, with_deleted = [], 0, 0
    for q, masks in _split_cases():
        o = oracle_mod.Oracle(q, L)
        bf = o.brute_force()
        if len(bf) == 0:
            o.close()
            continue
        for m in masks:
            ok, _, kept = o.projection(m)
            if not ok:
                continue
            checked += 1
            with_deleted += int(not kept.all())
            out += projected_split_failures(q, o, bf, m)
        o.close()
    return out, checked, with_deleted


def test_projected_split_brute_force(oracle_mod):
    bad, checked, with_deleted = _all_split_failures(oracle_mod)
    assert bad == []
    assert checked >= 40 and with_deleted >= 20, (checked, with_deleted)


# ---------------------------------------------------------------------------
# Planted mistakes in scratch copies of the oracle
# ---------------------------------------------------------------------------

MUTANTS = {
    "separator_not_first": [(
        "    if (t > 0) v.push_back(sep[t]);\n    for (int c = 0; c < K[t]; ++c)\n"
        "      if (t == 0 || c != sep[t]) v.push_back(c);\n    return v;",
        "    for (int c = 0; c < K[t]; ++c) v.push_back(c);\n    return v;")],
    "rows_descending": [(
        "return less_key(a, b) || (!less_key(b, a) && a < b);",
        "return less_key(a, b) || (!less_key(b, a) && a > b);")],
    "starts_are_indexes": [("if (start) start[e] = g.start[e];", "if (start) start[e] = e;")],
    "keys_in_sort_order": [(
        "      for (int c = 0; c < s.K[t]; ++c) keys[e * s.K[t] + c] = s.key(t, c, r0);",
        "      for (int c = 0; c < s.K[t]; ++c) keys[e * s.K[t] + c] = s.key(t, s.canon_cols(t)[c], r0);")],
    "deleted_weight_in_U": [
        ("      if (!kept[ch]) w = smul(w, lookup(s.sumdown[ch], s.key(t, s.pcol[ch], r)));",
         "      if (false) w = smul(w, lookup(s.sumdown[ch], s.key(t, s.pcol[ch], r)));"),
        ("      if (kept[ch]) u = smul(u, lookup(", "      u = smul(u, lookup(")],
    "deleted_child_wrong_message": [(
        "if (!kept[ch]) w = smul(w, lookup(s.sumdown[ch], s.key(t, s.pcol[ch], r)));",
        "if (!kept[ch]) w = smul(w, lookup(s.upval[ch], s.key(t, s.pcol[ch], r)));")],
}

FACTOR_MUTANTS = ("separator_not_first", "rows_descending", "starts_are_indexes", "keys_in_sort_order")
SPLIT_MUTANTS = ("deleted_weight_in_U", "deleted_child_wrong_message")


@pytest.fixture(scope="module")
def mutant_libs(tmp_path_factory, oracle_mod):
    src_dir = os.path.join(ROOT, "oracle")
    text = open(os.path.join(src_dir, "gj_oracle.cpp")).read()
    base = tmp_path_factory.mktemp("mutants")

    def build(name):
        s = text
        for find, repl in MUTANTS[name]:
            assert s.count(find) == 1, f"mutant {name}: the planted spot is gone from the oracle source"
            s = s.replace(find, repl)
        d = base / name
        d.mkdir()
        (d / "gj_oracle.cpp").write_text(s)
        shutil.copy(os.path.join(src_dir, "gj_natural.cpp"), d / "gj_natural.cpp")
        lib = str(d / "liboracle_mutant.so")
        subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-pthread",
                               str(d / "gj_oracle.cpp"), str(d / "gj_natural.cpp"), "-o", lib])
        return name, lib

    with cf.ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        return dict(ex.map(build, MUTANTS))


@pytest.mark.parametrize("name", FACTOR_MUTANTS)
def test_layout_pin_catches(oracle_mod, mutant_libs, name):
    L = oracle_mod.load_at(mutant_libs[name])
    assert _all_layout_failures(oracle_mod, L), f"planted mistake {name} not caught"


@pytest.mark.parametrize("name", SPLIT_MUTANTS)
def test_split_pin_catches(oracle_mod, mutant_libs, name):
    L = oracle_mod.load_at(mutant_libs[name])
    bad, _, _ = _all_split_failures(oracle_mod, L)
    assert bad, f"planted mistake {name} not caught"
