"""Run inside a process that preloads the address sanitizer: exercises every
oracle entry point with a sanitizer build of the oracle (path in argv[1])
and compares its results with the regular build's.  Any out-of-bounds
access, use after free or undefined behaviour aborts the process."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

from conftest import load_fig1  # noqa: E402
from oracle import oracle as O  # noqa: E402
from paper_2206_10435_amd import workloads as W  # noqa: E402


def run(o, q):
    out = {}
    out["js"] = o.join_size()
    Q, ovf = out["js"]
    for t in range(q.n_tables):
        out[f"factor{t}"] = o.factor(t)
        out[f"summ{t}"] = o.summary_table(t)
        out[f"fan{t}"] = o.fanouts(t)
        if t > 0:
            out[f"edge{t}"] = o.summary_edge(t)
    if not ovf and Q <= 5000:
        mat = o.materialize()
        out["mat"] = mat
        out["bf"] = o.brute_force()
        out["canon"] = o.canonical_result()
        out["ranges"] = o.materialize_threads(Q, 3)
        out["range"] = o.materialize_range(0, q.n_rows(0) // 2, Q)
        if Q:
            tup = out["canon"].astype(np.int64)
            out["check"] = o.check_tuples(tup, threads=2)
            bad = tup.copy()
            bad[0, 0] = -1
            out["check_bad"] = o.check_tuples(bad, threads=2)
            out["unrank"] = [o.unrank(r) for r in range(0, Q, max(1, Q // 7))]
            out["rank"] = [o.rank(tuple(int(v) for v in out["canon"][r])) for r in range(0, Q, max(1, Q // 7))]
            out["gfjs"] = o.gfjs(out["canon"])
        w = [np.linspace(0.5, 2.0, q.n_rows(t)) for t in range(q.n_tables)]
        out["weighted"] = o.weighted(w)
        out["fd"] = o.weighted_fd(w, 0, np.arange(min(3, q.n_rows(0)), dtype=np.int64))
        mask = [(1 << len(q.tables[t])) - 1 if t % 2 == 0 else 0 for t in range(q.n_tables)]
        mask[0] = 1
        out["proj"] = o.projection(mask)
        ok, mn, kept = out["proj"]
        if ok:
            for t in range(q.n_tables):
                if kept[t]:
                    out[f"ptab{t}"] = o.projected_table(mask, t)
            out["pres"] = o.projected_result(mask)
    return out


def same(a, b):
    if isinstance(a, dict):
        return a.keys() == b.keys() and all(same(a[k], b[k]) for k in a)
    if isinstance(a, (list, tuple)):
        return len(a) == len(b) and all(same(x, y) for x, y in zip(a, b))
    if isinstance(a, np.ndarray):
        return np.array_equal(a, b)
    return a == b


def main():
    San = O.load_at(sys.argv[1])
    Reg = O.lib()
    qs = [load_fig1()]
    for seed in range(10):
        n = 2 + seed % 4
        qs.append(W.random_tree_query(seed, n, {2: 30, 3: 14, 4: 8, 5: 6}[n], domain=2 + seed % 3, s=0.5 * (seed % 3),
                                      allow_empty=(seed % 7 == 6), min_rows=2, max_extra_cols=1))
    qs.append(W.chain_query(11, 0, 6, 200, 3, 0.0, name="overflow_chain6"))
    for q in qs:
        a = run(O.Oracle(q, L=San), q)
        b = run(O.Oracle(q, L=Reg), q)
        assert same(a, b), q.name
    # natural joins (cyclic): the sanitizer build through the module's library
    O._lib = San
    tri = [[np.array([0, 1, 1, 2], np.int32), np.array([1, 2, 0, 0], np.int32)],
           [np.array([1, 2, 0, 0], np.int32), np.array([2, 0, 2, 1], np.int32)],
           [np.array([0, 1, 2, 2], np.int32), np.array([2, 0, 1, 0], np.int32)]]
    attrs = [[0, 1], [1, 2], [0, 2]]
    nat = O.NaturalOracle(tri, attrs)
    n_nat = nat.join_size()
    rows = nat.materialize()
    assert len(rows) == n_nat
    nat.sorted_values([0, 1, 2])
    nat.potential([0, 1], [0, 1])
    nat.brute_force()
    print("sanitized oracle ok", len(qs), "queries", flush=True)


if __name__ == "__main__":
    main()
