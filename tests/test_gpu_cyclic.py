"""Cyclic queries on the GPU: POTENTIAL-JOIN (Algorithm 1) against the
oracle's joint potential, and the junction-tree summary of natural joins
(triangles, 4-cycles with a composite separator, a lastFM_cyc-shaped query,
random cyclic graphs, acyclic chains) against the oracle's sorted result."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gctx():
    from paper_2206_10435_amd import gj

    return gj.Context(0)


def _say(*a):
    print(*a, flush=True)


def _rng(seed):
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 47])))


def _zipf_col(rng, n, dom, s):
    if s == 0:
        return rng.integers(0, dom, size=n).astype(np.int32)
    p = 1.0 / np.arange(1, dom + 1) ** s
    p /= p.sum()
    perm = rng.permutation(dom)
    return perm[rng.choice(dom, size=n, p=p)].astype(np.int32)


def _tables(rng, attrs, n, dom, s=0.0):
    return [[_zipf_col(rng, n, dom, s) for _ in a] for a in attrs]


def _dev(tables):
    import torch

    return [[torch.from_numpy(c).to("cuda:0") for c in tb] for tb in tables]


def _check_potential(gctx, oracle_mod, tables, attrs):
    got = gctx.potential_join(_dev(tables), attrs)
    o = oracle_mod.NaturalOracle(tables, attrs)
    order = sorted({a for at in attrs for a in at})
    keys, counts = o.potential(list(range(len(tables))), order)
    _say("case potential", attrs, "entries", len(counts))
    assert got["attrs"] == order
    assert np.array_equal(got["keys"], keys) and np.array_equal(got["freq"], counts)


def test_potential_sec321_example(gctx, oracle_mod):
    one = lambda k: np.full(k, 1, np.int32)  # noqa: E731
    T1 = [np.concatenate([one(5), [2, 3]]).astype(np.int32), np.concatenate([one(5), [1, 1]]).astype(np.int32)]
    T2 = [np.concatenate([one(10), [1]]).astype(np.int32), np.concatenate([one(10), [2]]).astype(np.int32)]
    T3 = [one(20), one(20)]
    got = gctx.potential_join(_dev([T1, T2, T3]), [[0, 1], [1, 2], [2, 0]])
    assert got["keys"].tolist() == [[1, 1, 1]] and got["freq"].tolist() == [1000]


@pytest.mark.parametrize("case", range(8))
def test_potential_random(gctx, oracle_mod, case):
    rng = _rng(case)
    shapes = [
        [[0, 1], [1, 2], [2, 0]],
        [[0, 1], [1, 2], [2, 0]],
        [[0, 1, 2], [1, 2], [0, 2]],
        [[0, 1], [0, 2], [0, 3], [1, 2], [1, 3], [2, 3]],
        [[3, 1], [1, 2], [2, 3]],
        [[0, 1]],
        [[0, 1], [1, 2]],
        [[5, 2], [2, 9], [9, 5], [5, 7]],
    ]
    attrs = shapes[case]
    # rows and domain keep the oracle's row-level join below ~1e7 tuples
    rows, dom = [(300, 6), (400, 7), (300, 8), (40, 6), (500, 10), (700, 12), (500, 30), (200, 8)][case]
    tables = _tables(rng, attrs, rows, dom, s=0.6 * (case % 2))
    _check_potential(gctx, oracle_mod, tables, attrs)


def test_potential_empty(gctx, oracle_mod):
    rng = _rng(99)
    tables = [[np.zeros(10, np.int32), np.zeros(10, np.int32)], [np.ones(10, np.int32), rng.integers(0, 3, 10).astype(np.int32)]]
    got = gctx.potential_join(_dev(tables), [[0, 1], [1, 2]])
    assert len(got["freq"]) == 0


def _check_cyclic(gctx, oracle_mod, tables, attrs, windows=True):
    import torch

    s = gctx.summarize_cyclic(_dev(tables), attrs)
    o = oracle_mod.NaturalOracle(tables, attrs)
    Q = o.join_size()
    _say("case cyclic", attrs, "Q", Q, "cliques", s.n_tables)
    assert s.join_size == Q
    ra = gctx.result_attributes(s)
    assert sorted(ra) == sorted({a for at in attrs for a in at})
    ref = o.sorted_values(ra)
    nc = len(ra)
    out = torch.full((max(Q, 1) * nc + 64,), -7, dtype=torch.int32, device="cuda:0")
    nw = gctx.desummarize_projected(s, 0, Q + 3, out)
    got = out[: nw * nc].view(nw, nc).cpu().numpy()
    assert nw == Q and np.array_equal(got, ref)
    if windows and Q > 2:
        for first, cnt in ((1, Q - 2), (Q // 2, min(Q - Q // 2, 777))):
            nw = gctx.desummarize_projected(s, first, cnt, out)
            got = out[: nw * nc].view(nw, nc).cpu().numpy()
            assert nw == cnt and np.array_equal(got, ref[first:first + cnt])
    return s


def test_triangle(gctx, oracle_mod):
    rng = _rng(1)
    attrs = [[0, 1], [1, 2], [2, 0]]
    _check_cyclic(gctx, oracle_mod, _tables(rng, attrs, 400, 12, s=0.8), attrs)


def test_four_cycle_composite_separator(gctx, oracle_mod):
    rng = _rng(2)
    attrs = [[0, 1], [1, 2], [2, 3], [3, 0]]
    s = _check_cyclic(gctx, oracle_mod, _tables(rng, attrs, 300, 8, s=0.5), attrs)
    assert s.n_tables == 2


def test_lastfm_shaped(gctx, oracle_mod):
    rng = _rng(3)
    attrs = [[1, 2], [2, 3], [3, 4], [4, 1], [0, 1], [0, 4]]
    _check_cyclic(gctx, oracle_mod, _tables(rng, attrs, 90, 6, s=0.7), attrs)


def test_acyclic_chain_matches(gctx, oracle_mod):
    rng = _rng(4)
    attrs = [[0, 1], [1, 2], [2, 3], [3, 4]]
    _check_cyclic(gctx, oracle_mod, _tables(rng, attrs, 500, 30, s=1.0), attrs)


def test_random_cyclic(gctx, oracle_mod):
    done = 0
    for seed in range(40):
        rng = _rng(1000 + seed)
        na = int(rng.integers(3, 7))
        nt = int(rng.integers(3, 7))
        attrs = []
        for _ in range(nt):
            k = int(rng.integers(2, 4))
            attrs.append([int(x) for x in rng.choice(na, size=min(k, na), replace=False)])
        used = sorted({a for t in attrs for a in t})
        # connect: a table per consecutive pair of attributes not yet linked
        adj = {a: set() for a in used}
        for t in attrs:
            for x in t:
                adj[x] |= set(t) - {x}
        comp, st = {used[0]}, [used[0]]
        while st:
            x = st.pop()
            for y in adj[x] - comp:
                comp.add(y)
                st.append(y)
        if comp != set(used) or len(attrs) > 8:
            continue
        from paper_2206_10435_amd import gj

        jt = gj.junction_tree(attrs)
        if jt["n_fill"] == 0 and all(len(c) <= 2 for c in jt["cliques"]):
            continue  # acyclic and binary: covered elsewhere
        tables = _tables(rng, attrs, 60, 4, s=0.5)
        o = oracle_mod.NaturalOracle(tables, attrs)
        if o.join_size() > 2_000_000:
            continue
        _check_cyclic(gctx, oracle_mod, tables, attrs, windows=False)
        done += 1
        if done == 12:
            break
    assert done >= 8
