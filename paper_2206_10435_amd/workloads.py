"""Seeded synthetic join workloads (input data only).

This module draws tables and join graphs; it computes nothing about the join
itself (no counts, no messages, no order).  Both the HIP path and the CPU
oracle consume its output, which is why it lives on its own and imports
neither.

Generator rule.  Every column is drawn from
``np.random.Generator(PCG64(SeedSequence([seed, cfg, table, col])))``:

* a Zipf(s, D) rank k in [0, D) with P(k) proportional to (k+1)^-s, sampled by
  inverse CDF (s = 0 gives the uniform distribution);
* mapped through a permutation of [0, D) drawn from the same generator, so that
  the heavy hitters of two columns that meet in an equi-join are *not* forced
  onto the same value.  ``aligned=True`` instead draws one permutation per join
  attribute, which lines the heavy hitters up across an edge (the overflow
  stress case).

A join graph is a rooted tree over the tables: ``parent[t] < t`` (table 0 is
the root), and table t joins its parent on ``key[t][sep_col[t]] ==
key[parent[t]][parent_col[t]]`` (the natural equi-join of Sec. 1.1 restricted
to acyclic queries, Sec. 3.3).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

BASE_SEED = 20220621


@dataclass
class Query:
    """A set of tables (int32 key columns, SoA) plus an acyclic join graph."""

    name: str
    tables: List[List[np.ndarray]]
    parent: List[int]
    sep_col: List[int]
    parent_col: List[int]
    payload: List[List[np.ndarray]] = field(default_factory=list)

    @property
    def n_tables(self) -> int:
        return len(self.tables)

    def n_rows(self, t: int) -> int:
        return int(self.tables[t][0].shape[0]) if self.tables[t] else 0

    def total_rows(self) -> int:
        return sum(self.n_rows(t) for t in range(self.n_tables))


def _rng(seed: int, cfg: int, table: int, col: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, cfg, table, col])))


def zipf_ranks(rng: np.random.Generator, s: float, domain: int, n: int) -> np.ndarray:
    """Ranks in [0, domain) with P(k) proportional to (k+1)^-s (inverse CDF)."""
    if s == 0.0:
        return rng.integers(0, domain, size=n, dtype=np.int64)
    k = np.arange(1, domain + 1, dtype=np.float64)
    cdf = np.cumsum(k ** (-float(s)))
    cdf /= cdf[-1]
    u = rng.random(n)
    r = np.searchsorted(cdf, u, side="right")
    return np.minimum(r, domain - 1)


def zipf_column(seed: int, cfg: int, table: int, col: int, s: float, domain: int, n: int,
                perm_stream: Optional[int] = None) -> np.ndarray:
    """One int32 key column: a Zipf rank pushed through a seeded permutation.

    ``perm_stream`` (if given) names the stream that draws the permutation, so
    two columns with the same ``perm_stream`` share their heavy hitters.
    """
    rng = _rng(seed, cfg, table, col)
    if perm_stream is None:
        perm = rng.permutation(domain)
    else:
        perm = _rng(seed, cfg, 1_000_000 + perm_stream, 0).permutation(domain)
    ranks = zipf_ranks(rng, s, domain, n)
    return perm[ranks].astype(np.int32)


def chain_graph(n: int):
    """T_i(X_i, X_{i+1}); T_i joins T_{i-1} on X_i (its column 0 = parent's column 1)."""
    parent = [-1] + list(range(n - 1))
    sep = [0] * n
    pcol = [0] + [1] * (n - 1)
    sep[0] = 0
    return parent, sep, pcol


def chain_query(seed: int, cfg: int, n_tables: int, n_rows, domain: int, s: float,
                aligned: bool = False, payload_cols: int = 0, name: str = "chain") -> Query:
    """A chain T_0(X_0,X_1) join T_1(X_1,X_2) join ... with Zipf keys."""
    if isinstance(n_rows, int):
        n_rows = [n_rows] * n_tables
    tables, payload = [], []
    for t in range(n_tables):
        cols = []
        for c in range(2):
            attr = t + c
            cols.append(zipf_column(seed, cfg, t, c, s, domain, n_rows[t],
                                    perm_stream=attr if aligned else None))
        tables.append(cols)
        if payload_cols:
            rng = _rng(seed, cfg, t, 100)
            payload.append([rng.integers(-2**31, 2**31 - 1, size=n_rows[t], dtype=np.int64)
                            .astype(np.int32) for _ in range(payload_cols)])
    parent, sep, pcol = chain_graph(n_tables)
    return Query(name, tables, parent, sep, pcol, payload)


def star_query(seed: int, cfg: int, n_tables: int, n_rows, domain: int, s: float,
               aligned: bool = False, name: str = "star") -> Query:
    """Centre T_0(X_1..X_{n-1}) with leaves T_i(X_i, Y_i) joined on X_i."""
    if isinstance(n_rows, int):
        n_rows = [n_rows] * n_tables
    tables = []
    centre = [zipf_column(seed, cfg, 0, c, s, domain, n_rows[0],
                          perm_stream=(c + 1) if aligned else None) for c in range(n_tables - 1)]
    tables.append(centre)
    for t in range(1, n_tables):
        x = zipf_column(seed, cfg, t, 0, s, domain, n_rows[t], perm_stream=t if aligned else None)
        y = zipf_column(seed, cfg, t, 1, s, domain, n_rows[t], perm_stream=None)
        tables.append([x, y])
    parent = [-1] + [0] * (n_tables - 1)
    sep = [0] * n_tables
    pcol = [0] + [t - 1 for t in range(1, n_tables)]
    return Query(name, tables, parent, sep, pcol)


def reroot(q: Query, r: int):
    """The same query with table r as the root: tables reordered breadth-first
    from r so that every parent precedes its children.  Returns the query and
    the old index of every new table."""
    n = q.n_tables
    adj = [[] for _ in range(n)]  # (neighbour, my column, its column)
    for t in range(1, n):
        p = q.parent[t]
        adj[t].append((p, q.sep_col[t], q.parent_col[t]))
        adj[p].append((t, q.parent_col[t], q.sep_col[t]))
    order, par = [r], {r: (-1, 0, 0)}
    i = 0
    while i < len(order):
        u = order[i]
        i += 1
        for v, ucol, vcol in adj[u]:
            if v not in par:
                par[v] = (u, vcol, ucol)
                order.append(v)
    pos = {t: k for k, t in enumerate(order)}
    parent = [-1 if par[t][0] < 0 else pos[par[t][0]] for t in order]
    sep_col = [par[t][1] for t in order]
    parent_col = [par[t][2] for t in order]
    return Query(q.name + f"_root{r}", [q.tables[t] for t in order], parent, sep_col, parent_col), order


# ---------------------------------------------------------------------------
# The five workload shapes.
# ---------------------------------------------------------------------------

def cfg1(seed: int = BASE_SEED, n_rows: int = 10_000, domain: int = 1000) -> Query:
    """3-table chain T1(A,B) T2(B,C) T3(C,D), uniform int32 keys over [0, 1000)."""
    return chain_query(seed, 1, 3, n_rows, domain, 0.0, name=f"chain3_N{n_rows}_D{domain}_uniform")


def cfg2(seed: int = BASE_SEED, n_rows: int = 10_000_000, domain: int = 100_000, s: float = 1.1,
         aligned: bool = False, payload: bool = True) -> Query:
    """4-table chain, Zipf(1.1) keys over [0, 1e5), two int32 payload columns per table.

    With independent per-column permutations the join size is about 1e13; the
    aligned variant (heavy hitters lined up) overflows int64.
    """
    q = chain_query(seed, 2, 4, n_rows, domain, s, aligned=aligned, payload_cols=2 if payload else 0,
                    name=f"chain4_N{n_rows}_D{domain}_zipf{s}" + ("_aligned" if aligned else ""))
    return q


def cfg3(seed: int = BASE_SEED, fact_rows: int = 50_000_000,
         dim_rows=(1_000_000, 100_000, 300_000, 500_000), bridge_rows: int = 10_000_000,
         bridge_domain: int = 1_000_000, s: float = 0.9) -> Query:
    """Star plus chain: fact F(k1..k4) with FKs uniform into D1(pk, j), D2(pk), D3(pk), D4(pk);
    D1.j and a bridge B(j) are Zipf(0.9) over 1e6 values.  Tree: F root, D1..D4 its
    children (joined on pk = k_i), B child of D1 (joined on j)."""
    cfg = 3
    tables = []
    fact = []
    for i, nd in enumerate(dim_rows):
        rng = _rng(seed, cfg, 0, i)
        fact.append(rng.integers(0, nd, size=fact_rows, dtype=np.int64).astype(np.int32))
    tables.append(fact)
    for i, nd in enumerate(dim_rows):
        rng = _rng(seed, cfg, i + 1, 0)
        pk = rng.permutation(nd).astype(np.int32)
        cols = [pk]
        if i == 0:
            cols.append(zipf_column(seed, cfg, 1, 1, s, bridge_domain, nd))
        tables.append(cols)
    tables.append([zipf_column(seed, cfg, 5, 0, s, bridge_domain, bridge_rows)])
    parent = [-1, 0, 0, 0, 0, 1]
    sep = [0, 0, 0, 0, 0, 0]
    pcol = [0, 0, 1, 2, 3, 1]
    return Query(f"star_plus_chain_F{fact_rows}", tables, parent, sep, pcol)


def cfg4(seed: int = BASE_SEED, n_rows: int = 1_000_000, domain: int = 10_000, s: float = 1.2):
    """Weighted 4-table chain, Zipf(1.2) over [0, 1e4), weights U(0.5, 2) (f64 and its f32 rounding)."""
    q = chain_query(seed, 4, 4, n_rows, domain, s, name=f"wchain4_N{n_rows}_D{domain}_zipf{s}")
    w64 = []
    for t in range(4):
        rng = _rng(seed, 4, t, 200)
        w64.append(rng.uniform(0.5, 2.0, size=q.n_rows(t)))
    w32 = [w.astype(np.float32) for w in w64]
    return q, w64, w32


def cfg5_query(qi: int, attempt: int = 0, seed: int = BASE_SEED, min_rows_exp: float = 3.0,
               max_rows_exp: float = 6.0, min_dom_exp: float = 2.0, max_dom_exp: float = 5.0,
               max_tables: int = 6) -> Query:
    """Query qi of the many-query batch: 2..6 tables, chain or star, log-uniform
    sizes and domains, Zipf exponent uniform in [0, 1.5].  `attempt` > 0 draws
    a fresh query from its own streams (the batch replaces a query whose join
    size is too large by a later attempt; which attempt is kept is decided
    outside this module)."""
    rng = _rng(seed, 5, qi, 999) if attempt == 0 else _rng(seed, 5, qi, 999 + 1000 * attempt)
    n = int(rng.integers(2, max_tables + 1))
    shape = "chain" if rng.random() < 0.5 else "star"
    sizes = [int(round(10 ** rng.uniform(min_rows_exp, max_rows_exp))) for _ in range(n)]
    s = float(rng.uniform(0.0, 1.5))
    dom = int(round(10 ** rng.uniform(min_dom_exp, max_dom_exp)))
    sub = seed * 1000 + qi + attempt * 1_000_000
    suffix = "" if attempt == 0 else f"_a{attempt}"
    if shape == "chain" or n == 2:
        return chain_query(sub, 5, n, sizes, dom, s, name=f"q{qi}_chain{n}{suffix}")
    return star_query(sub, 5, n, sizes, dom, s, name=f"q{qi}_star{n}{suffix}")


def cfg5(seed: int = BASE_SEED, n_queries: int = 256, attempts=None, **kw) -> List[Query]:
    """Many independent queries (see cfg5_query); attempts[qi] (default 0)
    picks which draw of query qi is used."""
    return [cfg5_query(qi, 0 if attempts is None else int(attempts[qi]), seed=seed, **kw)
            for qi in range(n_queries)]


def random_tree_query(seed: int, n_tables: int, max_rows: int, domain: int, s: float = 0.0,
                      max_extra_cols: int = 2, allow_empty: bool = False,
                      min_rows: int = 1) -> Query:
    """Small random acyclic query for tests: random tree, random column counts,
    random separator / parent columns, ragged row counts."""
    rng = _rng(seed, 9, 0, 0)
    parent = [-1]
    for t in range(1, n_tables):
        parent.append(int(rng.integers(0, t)))
    children = [[] for _ in range(n_tables)]
    for t in range(1, n_tables):
        children[parent[t]].append(t)
    # every table needs a column per incident edge plus some private ones
    ncols = []
    for t in range(n_tables):
        need = len(children[t]) + (1 if t > 0 else 0)
        ncols.append(max(1, min(8, need + int(rng.integers(0, max_extra_cols + 1)))))
    sep = [0] * n_tables
    pcol = [0] * n_tables
    used = [set() for _ in range(n_tables)]
    for t in range(1, n_tables):
        c = int(rng.integers(0, ncols[t]))
        sep[t] = c
        used[t].add(c)
    for t in range(1, n_tables):
        p = parent[t]
        free = [c for c in range(ncols[p]) if c not in used[p]]
        c = int(rng.choice(free)) if free else int(rng.integers(0, ncols[p]))
        pcol[t] = c
        used[p].add(c)
    tables = []
    lo = 0 if allow_empty else max(1, min_rows)
    for t in range(n_tables):
        n = int(rng.integers(lo, max_rows + 1))
        cols = []
        for c in range(ncols[t]):
            vals = zipf_column(seed, 9, t + 1, c, s, domain, n)
            # shift some values negative so signed order is exercised
            cols.append((vals - domain // 3).astype(np.int32))
        tables.append(cols)
    return Query(f"rand{seed}", tables, parent, sep, pcol)


def cycle_query(seed: int = BASE_SEED, length: int = 3, n_rows: int = 1_000_000, domain: int = 10_000,
                s: float = 1.0):
    """A cyclic natural join T_i(X_i, X_{i+1 mod length}), Zipf(s) keys over
    [0, domain) with an independent permutation per (table, column): the
    triangle (length 3) and 4-cycle shapes of cyclic queries.  Returns the
    tables and their attribute ids."""
    cfg = 6
    tables, attrs = [], []
    for t in range(length):
        tables.append([zipf_column(seed, cfg, t, c, s, domain, n_rows) for c in range(2)])
        attrs.append([t, (t + 1) % length])
    return tables, attrs
