"""The junction-tree planner (host only): min fill-in triangulation, maxcliques
and a maximal spanning tree, checked against the definitions of Sec. 2.2.1 --
every table inside its clique, running intersection, chordal fill-in with a
minimum-fill choice at every step, maximal cliques, maximum total separator
weight (brute force over all spanning trees of small clique graphs)."""
import itertools

import numpy as np
import pytest

from paper_2206_10435_amd import gj


def _graph(attrs):
    adj = {}
    for a in attrs:
        for x in a:
            adj.setdefault(x, set())
        for x, y in itertools.combinations(a, 2):
            adj[x].add(y)
            adj[y].add(x)
    return adj


def _check(attrs):
    jt = gj.junction_tree(attrs)
    cl = [set(c) for c in jt["cliques"]]
    k = len(cl)
    par = jt["parent"]
    assert par[0] == -1 and all(0 <= par[i] < i for i in range(1, k))
    # tables inside their clique, and no earlier clique holds them
    for t, a in enumerate(attrs):
        c = jt["table_clique"][t]
        assert set(a) <= cl[c] and not any(set(a) <= cl[j] for j in range(c))
    # replay the elimination: each step's node has the minimum fill among the rest
    adj = {x: set(v) for x, v in _graph(attrs).items()}
    left = set(adj)
    fill_total = 0
    recorded = []
    for v in jt["elim_order"]:
        def fill(u):
            nb = adj[u] & left
            return sum(1 for x, y in itertools.combinations(sorted(nb), 2) if y not in adj[x])
        assert fill(v) == min(fill(u) for u in left)
        nb = adj[v] & left
        fill_total += fill(v)
        for x, y in itertools.combinations(nb, 2):
            adj[x].add(y)
            adj[y].add(x)
        recorded.append((nb | {v}) - set())
        left.remove(v)
    assert fill_total == jt["n_fill"]
    # cliques: the maximal recorded cliques, each a clique of the triangulated graph
    maximal = {frozenset(c) for c in recorded if not any(c < d for d in recorded)}
    assert {frozenset(c) for c in cl} == maximal and len(cl) == len(maximal)
    for c in cl:
        assert all(y in adj[x] for x, y in itertools.combinations(c, 2))
    # running intersection: the cliques holding an attribute form a subtree
    for a in jt["attr_ids"]:
        holders = [i for i in range(k) if a in cl[i]]
        roots = [i for i in holders if par[i] < 0 or a not in cl[par[i]]]
        assert len(roots) == 1, (a, holders)
    # maximum weight among all spanning trees (small clique graphs)
    w = sum(len(cl[i] & cl[par[i]]) for i in range(1, k))
    if k <= 6:
        best = 0
        for ps in itertools.product(*[range(k)] * (k - 1)):
            p = [-1] + list(ps)
            ok = True
            for i in range(1, k):
                seen, x = set(), i
                while x > 0 and ok:
                    if x in seen:
                        ok = False
                    seen.add(x)
                    x = p[x]
                if p[i] == i:
                    ok = False
            if ok:
                best = max(best, sum(len(cl[i] & cl[p[i]]) for i in range(1, k)))
        assert w == best
    return jt


def test_chain_tree_needs_no_fill():
    jt = _check([[0, 1], [1, 2], [2, 3]])
    assert jt["n_fill"] == 0 and jt["cliques"] == [[0, 1], [1, 2], [2, 3]]


def test_triangle_is_one_clique():
    jt = _check([[0, 1], [1, 2], [2, 0]])
    assert jt["n_fill"] == 0 and jt["cliques"] == [[0, 1, 2]] and jt["table_clique"] == [0, 0, 0]


def test_four_cycle_gets_one_chord():
    jt = _check([[0, 1], [1, 2], [2, 3], [3, 0]])
    assert jt["n_fill"] == 1 and len(jt["cliques"]) == 2
    assert all(len(c) == 3 for c in jt["cliques"])


def test_lastfm_like_cycle():
    """A 5-node cyclic query shaped like the paper's lastFM_cyc (users U1..U4
    in a cycle plus an artist joined to two of them)."""
    attrs = [[1, 2], [2, 3], [3, 4], [4, 1], [0, 1], [0, 4]]
    jt = _check(attrs)
    assert max(len(c) for c in jt["cliques"]) == 3


@pytest.mark.parametrize("seed", range(40))
def test_random_graphs(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    na = int(rng.integers(3, 9))
    nt = int(rng.integers(2, 9))
    attrs = []
    for _ in range(nt):
        k = int(rng.integers(1, 4))
        attrs.append([int(x) for x in rng.choice(na, size=min(k, na), replace=False)])
    # keep the query connected: chain the attributes' first tables if needed
    used = sorted({a for t in attrs for a in t})
    for x, y in zip(used, used[1:]):
        attrs.append([x, y]) if rng.random() < 0.3 else None
    adj = _graph(attrs)
    comp, st = {used[0]}, [used[0]]
    while st:
        x = st.pop()
        for y in adj[x] - comp:
            comp.add(y)
            st.append(y)
    if comp != set(adj):
        with pytest.raises(gj.GJError) as ei:
            gj.junction_tree(attrs)
        assert ei.value.status == gj.GJ_E_GRAPH
        return
    _check(attrs)


def test_errors():
    with pytest.raises(gj.GJError):
        gj.junction_tree([[0, -1]])
    with pytest.raises(gj.GJError):
        gj.junction_tree([list(range(i * 8, i * 8 + 8)) for i in range(9)])  # 72 attributes
