"""The keyed-lookup expansion -- row-id desummarization of summaries whose
tables between the root and the innermost table hold one entry per group --
against the oracle's canonical result (Definition 1's order) and against the
general expansion kernel on the same summary, bit-exact: stars of dimensions
joined on their keys with a bridge below one of them (the star-plus-chain
shape at small sizes), repeated fact rows (root counts above 1), duplicated
dimension rows (middle counts above 1), innermost groups of several entries,
chains with a keyed middle table, two-table joins, and one-tuple root blocks
(every window of 64 ranks spans 64 root entries), alone and next to long
blocks; int32 and int64 row ids, whole results and ragged windows.  Whole
results of the larger cases take the record pass (root-entry records written
first); the one-tuple case and the short windows decode records in place."""
import numpy as np
import pytest

from paper_2206_10435_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gctx():
    from paper_2206_10435_amd import gj

    return gj.Context(0)


def _say(*a):
    print(*a, flush=True)


def _star(seed, fact, dims, bridge_rows, bridge_dom, s, dup_fact=0, dup_dim=0, bridge_extra=0, bridge=True):
    """Fact F(k1..kd) uniform into dimensions D_i(pk[, j]) (pk a permutation);
    D1.j and a bridge B(j[, x]) Zipf(s) over bridge_dom, B a child of D1.
    dup_fact repeats fact rows (root entries of count 2), dup_dim repeats rows
    of the last dimension (its single entries get count 2), bridge_extra > 0
    adds a bridge column x over that many values (several entries per group)."""
    rng = np.random.default_rng(seed)
    fcols = [rng.integers(0, nd, size=fact).astype(np.int32) for nd in dims]
    if dup_fact:
        idx = rng.integers(0, fact, size=dup_fact)
        fcols = [np.concatenate([c, c[idx]]) for c in fcols]
    tables = [fcols]
    for i, nd in enumerate(dims):
        pk = rng.permutation(nd).astype(np.int32)
        cols = [pk]
        if i == 0 and bridge:
            cols.append(W.zipf_ranks(rng, s, bridge_dom, nd).astype(np.int32))
        if i == len(dims) - 1 and dup_dim:
            idx = rng.integers(0, nd, size=dup_dim)
            cols = [np.concatenate([c, c[idx]]) for c in cols]
        tables.append(cols)
    parent = [-1] + [0] * len(dims)
    sep = [0] * (len(dims) + 1)
    pcol = [0] + list(range(len(dims)))
    if bridge:
        bcols = [W.zipf_ranks(rng, s, bridge_dom, bridge_rows).astype(np.int32)]
        if bridge_extra:
            bcols.append(rng.integers(0, bridge_extra, size=bridge_rows).astype(np.int32))
        tables.append(bcols)
        parent.append(1)
        sep.append(0)
        pcol.append(1)
    name = f"star{len(dims)}_s{seed}" + ("_bridge" if bridge else "")
    return W.Query(name, tables, parent, sep, pcol)


def _chain_keyed_middle(seed, n_a, n_b, n_c, dom_c, s):
    """A(x, y) -> B(y, z) with y a key of B -> C(z, w): B's groups hold one entry."""
    rng = np.random.default_rng(seed)
    a = [rng.integers(0, 50, size=n_a).astype(np.int32), rng.integers(0, n_b, size=n_a).astype(np.int32)]
    b = [rng.permutation(n_b).astype(np.int32), W.zipf_ranks(rng, s, dom_c, n_b).astype(np.int32)]
    c = [W.zipf_ranks(rng, s, dom_c, n_c).astype(np.int32), rng.integers(0, 7, size=n_c).astype(np.int32)]
    return W.Query(f"chain3_keyed_s{seed}", [a, b, c], [-1, 0, 1], [0, 0, 0], [0, 1, 1])


def _one_tuple_blocks(seed, n):
    """R(a) -> S(a), both permutations: every root entry expands to one tuple."""
    rng = np.random.default_rng(seed)
    r = [rng.permutation(n).astype(np.int32)]
    t = [rng.permutation(n).astype(np.int32), rng.integers(0, 3, size=n).astype(np.int32)]
    return W.Query(f"pair_unit_blocks_{n}", [r, t], [-1, 0], [0, 0], [0, 0])


def _mixed_blocks(seed, n):
    """R(a) -> S(a): the first half of R's keys match one row of S, the rest 40
    rows each; the records of R's entries stay small against the output, so
    the expansion takes them from the record pass while runs of 64 one-tuple
    entries fill whole windows."""
    rng = np.random.default_rng(seed)
    r = [rng.permutation(n).astype(np.int32)]
    half = n // 2
    keys = np.concatenate([np.arange(half), np.repeat(np.arange(half, n), 40)])
    rng.shuffle(keys)
    t = [keys.astype(np.int32), rng.integers(0, 1000, size=len(keys)).astype(np.int32)]
    return W.Query(f"pair_mixed_blocks_{n}", [r, t], [-1, 0], [0, 0], [0, 0])


def _two_table(seed, n_r, n_s, dom, s):
    rng = np.random.default_rng(seed)
    r = [W.zipf_ranks(rng, s, dom, n_r).astype(np.int32), rng.integers(0, 5, size=n_r).astype(np.int32)]
    t = [W.zipf_ranks(rng, s, dom, n_s).astype(np.int32), rng.integers(0, 9, size=n_s).astype(np.int32)]
    return W.Query(f"pair_zipf_s{seed}", [r, t], [-1, 0], [0, 0], [0, 0])


def _cases():
    return [
        _star(1, 20000, (400, 60, 150, 250), 3000, 400, 0.9),
        _star(2, 15000, (300, 40, 90, 120), 2500, 300, 0.9, dup_fact=3000),
        _star(3, 12000, (300, 40, 90, 120), 2000, 300, 0.7, dup_dim=40),
        _star(4, 12000, (300, 40, 90, 120), 2500, 300, 0.9, bridge_extra=6),
        _star(5, 9000, (200, 30, 80, 100), 2000, 200, 0.9, dup_fact=2000, dup_dim=30, bridge_extra=4),
        _star(6, 30000, (500, 70, 200), 0, 0, 0.0, bridge=False),
        _chain_keyed_middle(7, 6000, 900, 4000, 300, 0.8),
        _one_tuple_blocks(8, 70001),
        _mixed_blocks(10, 10000),
        _two_table(9, 5000, 4000, 600, 1.0),
        # eight tables (the largest exact instance) and nine (the instance for any count)
        _star(12, 8000, (100, 30, 40, 50, 60, 70), 1500, 100, 0.8, bridge_extra=3),
        _star(13, 8000, (100, 30, 40, 50, 60, 70, 80), 1500, 100, 0.8),
    ]


def _desum(gctx, s, n, first, count, dtype):
    import torch

    out = torch.full((max(count, 1) * n,), -7, dtype=dtype, device="cuda:0")
    nw = gctx.desummarize(s, first, count, out)
    assert nw == count
    return out[: nw * n].view(nw, n).cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("q", _cases(), ids=lambda q: q.name)
def test_keyed_lookup_expansion_matches_oracle(gctx, oracle_mod, q):
    import torch

    from paper_2206_10435_amd import gj

    o = oracle_mod.Oracle(q)
    Q, ovf = o.join_size()
    assert not ovf and 0 < Q <= 4_000_000, Q
    _say("case unit", q.name, "Q =", Q)
    ref = o.canonical_result().astype(np.int64)
    s = gctx.summarize(gctx.build_factors(gj.to_device_tables(q), q.parent, q.sep_col, q.parent_col))
    assert s.join_size == Q
    n = q.n_tables
    assert gctx.desum_kernel(s) == "unit"
    windows = [(0, Q), (1, min(63, Q - 1)), (64, min(65, Q - 64)), (Q // 3 + 5, min(4097 + 7, Q - Q // 3 - 5)),
               (Q - 100, 100), (Q - 1, 1), (Q, 0)]
    for dt in (torch.int32, torch.int64):
        for first, cnt in windows:
            got = _desum(gctx, s, n, first, cnt, dt)
            assert np.array_equal(got, ref[first:first + cnt]), (dt, first, cnt)
    # the general kernel on the same summary: the same tuples
    try:
        gctx.set_tune(desum_general=1)
        assert gctx.desum_kernel(s) == "general"
        got = _desum(gctx, s, n, 0, Q, torch.int64)
        assert np.array_equal(got, ref)
    finally:
        gctx.set_tune()
    assert gctx.desum_kernel(s) == "unit"


def test_kernel_choice_follows_the_middle_tables(gctx, oracle_mod):
    """A chain whose middle table has groups of several entries takes the
    general kernel; a one-table query too (no innermost table below a root)."""
    from paper_2206_10435_amd import gj

    q = W.chain_query(31, 0, 3, 3000, 200, 0.8, name="chain3_general")
    s = gctx.summarize(gctx.build_factors(gj.to_device_tables(q), q.parent, q.sep_col, q.parent_col))
    mc = s.table(1)["keys"].shape[0]
    groups = len(np.unique(s.table(1)["keys"][:, q.sep_col[1]]))
    assert mc > groups  # some group of the middle table holds several entries
    assert gctx.desum_kernel(s) == "general"
    q1 = W.Query("single", [[np.arange(100, dtype=np.int32) % 7]], [-1], [0], [0])
    s1 = gctx.summarize(gctx.build_factors(gj.to_device_tables(q1), q1.parent, q1.sep_col, q1.parent_col))
    assert gctx.desum_kernel(s1) == "general"


def test_records_decoded_in_place_when_scratch_is_refused(oracle_mod):
    """The record pass takes scratch from the context's allocator; when the
    allocator refuses it, the expansion decodes the records in place and the
    result is the same, with nothing left allocated."""
    import gc

    import torch

    from paper_2206_10435_amd import gj

    state = {"refuse": False, "live": set(), "refused": 0}
    stream = torch.cuda.current_stream()

    def alloc(nbytes):
        if state["refuse"]:
            state["refused"] += 1
            return 0
        p = torch.cuda.caching_allocator_alloc(nbytes, 0, stream)
        state["live"].add(p)
        return p

    def free(p):
        state["live"].discard(p)
        torch.cuda.caching_allocator_delete(p)

    ctx = gj.Context(0, allocator=(alloc, free))
    q = _star(11, 20000, (400, 60, 150, 250), 3000, 400, 0.9)
    o = oracle_mod.Oracle(q)
    ref = o.canonical_result().astype(np.int64)
    s = ctx.summarize(ctx.build_factors(gj.to_device_tables(q), q.parent, q.sep_col, q.parent_col))
    Q = s.join_size
    assert Q == len(ref) and ctx.desum_kernel(s) == "unit"
    _say("case refused scratch", q.name, "Q =", Q)
    live_before = set(state["live"])
    for refuse in (False, True):
        state["refuse"] = refuse
        out = torch.full((Q * q.n_tables,), -7, dtype=torch.int64, device="cuda:0")
        assert ctx.desummarize(s, 0, Q, out) == Q
        got = out.view(Q, q.n_tables).cpu().numpy()
        assert np.array_equal(got, ref), refuse
        assert state["live"] == live_before, refuse  # the scratch went back
    assert state["refused"] >= 1  # the record pass asked and was refused
    state["refuse"] = False
    del s
    gc.collect()
    torch.cuda.synchronize()
    assert not state["live"]


def _payload(q, seed):
    """One seeded int32 payload column (full int32 range) per table."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 91])))
    return [rng.integers(-2**31, 2**31 - 1, size=q.n_rows(t), dtype=np.int64).astype(np.int32)
            for t in range(q.n_tables)]


def _value_cases():
    # (query, picks): picks are (table, "key"/"pay", column); the column counts
    # reach the 4-, 8- and 16-column instances
    star1 = _star(1, 20000, (400, 60, 150, 250), 3000, 400, 0.9)
    star2 = _star(2, 15000, (300, 40, 90, 120), 2500, 300, 0.9, dup_fact=3000)
    star3 = _star(3, 12000, (300, 40, 90, 120), 2000, 300, 0.7, dup_dim=40)
    star4 = _star(4, 12000, (300, 40, 90, 120), 2500, 300, 0.9, bridge_extra=6)
    chain = _chain_keyed_middle(7, 6000, 900, 4000, 300, 0.8)
    one = _one_tuple_blocks(8, 70001)
    star9 = _star(13, 8000, (100, 30, 40, 50, 60, 70, 80), 1500, 100, 0.8)
    every = lambda q: [(t, "pay", 0) for t in range(q.n_tables)]  # noqa: E731
    return [
        (star1, every(star1) + [(1, "key", 1), (5, "key", 0)]),
        (star2, [(0, "pay", 0), (0, "key", 2), (3, "pay", 0), (5, "pay", 0)]),
        (star3, every(star3) + [(4, "key", 0)]),
        (star4, every(star4) + [(5, "key", 1), (0, "key", 0)]),
        (chain, [(1, "pay", 0), (2, "key", 1), (0, "key", 0)]),
        (one, [(1, "key", 1), (0, "pay", 0), (1, "pay", 0)]),
        (star9, every(star9) + [(0, "key", 3), (1, "key", 1)]),
    ]


@pytest.mark.parametrize("case", _value_cases(), ids=lambda c: f"{c[0].name}_{len(c[1])}cols")
def test_keyed_lookup_values_match_oracle(gctx, oracle_mod, case):
    """Value columns (payload gather) through the keyed-lookup expansion:
    every value equals the host column at the oracle's row id, whole and in
    ragged windows, and the general kernel gives the same values."""
    import torch

    from paper_2206_10435_amd import gj

    q, picks = case
    o = oracle_mod.Oracle(q)
    ref_rows = o.canonical_result()
    pay = _payload(q, 5)
    host = [np.ascontiguousarray(q.tables[t][i] if src == "key" else pay[t], dtype=np.int32) for t, src, i in picks]
    ref = np.stack([h[ref_rows[:, t]] for (t, _, _), h in zip(picks, host)], axis=1)
    s = gctx.summarize(gctx.build_factors(gj.to_device_tables(q), q.parent, q.sep_col, q.parent_col))
    Q = s.join_size
    assert Q == len(ref) and gctx.desum_kernel(s) == "unit"
    cs = gctx.colset(s, [(t, torch.from_numpy(h).to("cuda:0")) for (t, _, _), h in zip(picks, host)])
    nc = len(picks)
    _say("case unit values", q.name, "cols", nc, "Q", Q)

    def values(first, count):
        out = torch.full((max(count, 1) * nc,), -7, dtype=torch.int32, device="cuda:0")
        nw = gctx.desummarize_values(s, cs, first, count, out)
        assert nw == count
        return out[: nw * nc].view(nw, nc).cpu().numpy()

    for first, cnt in [(0, Q), (1, min(63, Q - 1)), (Q // 3 + 5, min(4104, Q - Q // 3 - 5)), (Q - 100, 100)]:
        assert np.array_equal(values(first, cnt), ref[first:first + cnt]), (first, cnt)
    try:
        gctx.set_tune(desum_general=1)
        assert np.array_equal(values(0, Q), ref)
    finally:
        gctx.set_tune()


def test_reloaded_summary_takes_the_keyed_lookup_expansion(gctx, oracle_mod, tmp_path):
    """A star summary written to a file and loaded back carries the counts the
    kernel choice reads: the reloaded summary takes the keyed-lookup expansion
    and gives the oracle's tuples and values."""
    import torch

    from paper_2206_10435_amd import gj

    q = _star(14, 12000, (300, 40, 90, 120), 2500, 300, 0.9, dup_fact=1500)
    o = oracle_mod.Oracle(q)
    ref = o.canonical_result().astype(np.int64)
    s = gctx.summarize(gctx.build_factors(gj.to_device_tables(q), q.parent, q.sep_col, q.parent_col))
    path = str(tmp_path / "star.gjs")
    gctx.save(s, path, with_rows=True)
    r = gctx.load(path)
    Q = r.join_size
    assert Q == len(ref) and gctx.desum_kernel(r) == "unit"
    _say("case reloaded star", q.name, "Q =", Q)
    for dt in (torch.int32, torch.int64):
        assert np.array_equal(_desum(gctx, r, q.n_tables, 0, Q, dt), ref), dt
    pay = _payload(q, 9)
    cs = gctx.colset(r, [(t, torch.from_numpy(pay[t]).to("cuda:0")) for t in range(q.n_tables)])
    out = torch.full((Q * q.n_tables,), -7, dtype=torch.int32, device="cuda:0")
    assert gctx.desummarize_values(r, cs, 0, Q, out) == Q
    exp = np.stack([pay[t][ref[:, t]] for t in range(q.n_tables)], axis=1)
    assert np.array_equal(out.view(Q, q.n_tables).cpu().numpy(), exp)


def test_block_offsets_beyond_32_bits(gctx, oracle_mod):
    """One key shared by 1e5 rows on each side, the child's rows split over two
    entries: the root entry's block holds 1e10 tuples and each child entry's
    5e9, so offsets inside a block pass 2^32 (the 64-bit split, with the search
    inside the innermost group).  Short windows (records decoded in place) are
    compared tuple by tuple with the oracle's unrank; a 1e6-tuple window across
    2^32 (records written first) is checked whole by the oracle's checker, with
    the oracle's rank of its ends.  Both kernels."""
    import torch

    from paper_2206_10435_amd import gj

    rng = np.random.default_rng(22)
    n = 100_000
    ra = np.concatenate([np.zeros(n, np.int64), rng.integers(1, 50, size=1000)])
    sa = np.concatenate([np.zeros(n, np.int64), rng.integers(1, 50, size=1000)])
    sx = np.concatenate([rng.integers(0, 2, size=n), rng.integers(0, 5, size=1000)])
    p1, p2 = rng.permutation(len(ra)), rng.permutation(len(sa))
    q = W.Query("pair_huge_block", [[ra[p1].astype(np.int32)], [sa[p2].astype(np.int32), sx[p2].astype(np.int32)]],
                [-1, 0], [0, 0], [0, 0])
    o = oracle_mod.Oracle(q)
    Q, ovf = o.join_size()
    assert not ovf and Q > 10**10
    s = gctx.summarize(gctx.build_factors(gj.to_device_tables(q), q.parent, q.sep_col, q.parent_col))
    assert s.join_size == Q and gctx.desum_kernel(s) == "unit"
    _say("case huge block, Q =", Q)
    short = [(2**32 - 3, 7), (5 * 10**9 + 2**32 + 11, 9), (Q - 10, 10)]
    try:
        for general in (0, 1):
            gctx.set_tune(desum_general=general)
            for first, cnt in short:
                got = _desum(gctx, s, 2, first, cnt, torch.int64)
                exp = np.stack([o.unrank(first + i) for i in range(cnt)]).astype(np.int64)
                assert np.array_equal(got, exp), (general, first)
            first, cnt = 2**32 - 500_000, 1_000_000
            got = _desum(gctx, s, 2, first, cnt, torch.int64)
            assert o.check_tuples(got) == -1, general
            assert o.rank(got[0].astype(np.int32)) == first and o.rank(got[-1].astype(np.int32)) == first + cnt - 1
            for i in (0, 499_999, 500_000, 500_001, cnt - 1):
                assert np.array_equal(got[i], o.unrank(first + i)), (general, i)
    finally:
        gctx.set_tune()


def _unique_leaves(seed, fact, dims, all_referenced):
    """Fact F(k1..kd) into dimensions D_i(pk), pk a permutation (one row per
    group): every dimension row referenced, or only the first half of each
    dimension's keys."""
    rng = np.random.default_rng(seed)
    fcols = []
    for nd in dims:
        if all_referenced:
            c = np.concatenate([np.arange(nd), rng.integers(0, nd, size=fact - nd)])
            rng.shuffle(c)
        else:
            c = rng.integers(0, nd // 2, size=fact)
        fcols.append(c.astype(np.int32))
    tables = [fcols] + [[rng.permutation(nd).astype(np.int32)] for nd in dims]
    n = len(dims)
    name = "unique_leaves_" + ("all" if all_referenced else "half")
    return W.Query(name, tables, [-1] + [0] * n, [0] * (n + 1), [0] + list(range(n)))


@pytest.mark.parametrize("all_referenced", [True, False], ids=["all_rows_referenced", "half_unreferenced"])
def test_unique_key_leaves(gctx, oracle_mod, all_referenced):
    """Leaves keyed by a unique column send 1 from every group (the upward pass
    gathers no message from them) and, when every row survives, get their child
    records without a gather; with unreferenced rows the records are gathered.
    The summary and every tuple, by both expansion kernels, against the oracle."""
    import torch

    from paper_2206_10435_amd import gj

    q = _unique_leaves(31, 20_000, (700, 1500, 3000), all_referenced)
    o = oracle_mod.Oracle(q)
    Q, ovf = o.join_size()
    assert not ovf and Q == 20_000
    _say("case", q.name, "Q =", Q)
    s = gctx.summarize(gctx.build_factors(gj.to_device_tables(q), q.parent, q.sep_col, q.parent_col))
    assert s.join_size == Q
    for t in range(q.n_tables):
        g, r = s.table(t), o.summary_table(t)
        for k in ("keys", "c", "U", "D", "F"):
            assert np.array_equal(g[k], r[k]), (t, k)
    ref = o.canonical_result().astype(np.int64)
    try:
        for general in (0, 1):
            gctx.set_tune(desum_general=general)
            got = _desum(gctx, s, q.n_tables, 0, Q, torch.int64)
            assert np.array_equal(got, ref), general
            got = _desum(gctx, s, q.n_tables, 777, 5000, torch.int32)
            assert np.array_equal(got, ref[777:5777]), general
    finally:
        gctx.set_tune()
