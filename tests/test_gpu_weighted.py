"""Weighted join size and its adjoint (the downward pass) against the oracle's
__float128 definitions: exact at unit weights, 1e-12 relative otherwise, and
central finite differences at the full 4-table 1e6-row workload."""
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


def _run(gctx, q, weights, dtype):
    import torch

    from paper_2206_10435_amd import gj

    tabs = gj.to_device_tables(q)
    f = gctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col)
    ws = [torch.from_numpy(np.ascontiguousarray(w)).to(dtype).to("cuda:0") for w in weights]
    Wt, st = gctx.weighted_forward(f, ws)
    grads = [torch.empty_like(w) for w in ws]
    gW = torch.ones((), dtype=torch.float64, device="cuda:0")
    gctx.weighted_backward(st, gW, grads)
    return float(Wt.item()), [g.cpu().numpy().astype(np.float64) for g in grads]


def _queries():
    return [W.random_tree_query(seed, n, rows, dom, s=s, max_extra_cols=2, min_rows=rows // 3)
            for seed, n, rows, dom, s in [(301, 3, 3000, 200, 0.8), (302, 4, 2000, 300, 1.0),
                                          (303, 5, 1500, 200, 0.5), (304, 2, 5000, 100, 1.3),
                                          (305, 6, 1200, 150, 0.7)]]


@pytest.mark.parametrize("q", _queries(), ids=lambda q: q.name)
def test_unit_weights_are_exact_counts(gctx, oracle_mod, q):
    o = oracle_mod.Oracle(q)
    Q, _ = o.join_size()
    _say("case unit", q.name, Q)
    assert Q < 2**53
    ones = [np.ones(q.n_rows(t)) for t in range(q.n_tables)]
    Wv, g = _run(gctx, q, ones, __import__("torch").float64)
    assert Wv == float(Q)
    for t in range(q.n_tables):
        assert np.array_equal(g[t], o.fanouts(t).astype(np.float64)), t


@pytest.mark.parametrize("q", _queries(), ids=lambda q: q.name)
def test_random_weights_f64(gctx, oracle_mod, q):
    import torch

    o = oracle_mod.Oracle(q)
    rng = np.random.default_rng(7)
    w = [rng.uniform(0.5, 2.0, q.n_rows(t)) for t in range(q.n_tables)]
    Wref, gref = o.weighted(w)
    _say("case f64", q.name, Wref)
    Wv, g = _run(gctx, q, w, torch.float64)
    assert abs(Wv - Wref) <= 1e-12 * abs(Wref)
    for t in range(q.n_tables):
        nz = gref[t] != 0
        assert np.all(g[t][~nz] == 0), t
        assert np.all(np.abs(g[t][nz] - gref[t][nz]) <= 1e-12 * np.abs(gref[t][nz])), t


def test_random_weights_f32(gctx, oracle_mod):
    import torch

    q = _queries()[1]
    o = oracle_mod.Oracle(q)
    rng = np.random.default_rng(8)
    w32 = [rng.uniform(0.5, 2.0, q.n_rows(t)).astype(np.float32) for t in range(q.n_tables)]
    # the oracle sees the float32 values exactly (upcast), the path accumulates in float64
    Wref, gref = o.weighted([x.astype(np.float64) for x in w32])
    Wv, g = _run(gctx, q, w32, torch.float32)
    assert abs(Wv - Wref) <= 1e-12 * abs(Wref)
    for t in range(q.n_tables):
        ref32 = gref[t].astype(np.float32).astype(np.float64)
        # one float32 rounding of a float64 result within 1e-12
        assert np.all(np.abs(g[t] - ref32) <= np.abs(ref32) * 2.0**-23), t


def test_autograd_function(gctx, oracle_mod):
    import torch

    from paper_2206_10435_amd import gj

    q = W.random_tree_query(306, 3, 300, 40, s=0.6, max_extra_cols=1, min_rows=100)
    o = oracle_mod.Oracle(q)
    tabs = gj.to_device_tables(q)
    f = gctx.build_factors(tabs, q.parent, q.sep_col, q.parent_col)
    rng = np.random.default_rng(9)
    wn = [rng.uniform(0.5, 2.0, q.n_rows(t)) for t in range(q.n_tables)]
    ws = [torch.from_numpy(x).to("cuda:0").requires_grad_(True) for x in wn]
    out = gj.WeightedJoinSize.apply(gctx, f, *ws)
    (3.0 * out).backward()
    Wref, gref = o.weighted(wn)
    assert abs(float(out) - Wref) <= 1e-12 * Wref
    for t in range(q.n_tables):
        got = ws[t].grad.cpu().numpy()
        assert np.allclose(got, 3.0 * gref[t], rtol=1e-12, atol=0), t


def test_cfg4_full_scale(gctx, oracle_mod):
    """4-table chain, 1e6 rows per table, Zipf(1.2) over 1e4: unit weights
    against int64 fan-outs (bit-exact), float64 weights against __float128
    gradients of every row and central finite differences on sampled rows."""
    import torch

    q, w64, w32 = W.cfg4()
    o = oracle_mod.Oracle(q)
    Q, ovf = o.join_size()
    _say("case cfg4", Q)
    assert not ovf and Q < 2**53
    ones = [np.ones(q.n_rows(t)) for t in range(4)]
    Wv, g = _run(gctx, q, ones, torch.float64)
    assert Wv == float(Q)
    for t in range(4):
        assert np.array_equal(g[t], o.fanouts(t).astype(np.float64)), t
    Wref, gref = o.weighted(w64)
    Wv, g = _run(gctx, q, w64, torch.float64)
    assert abs(Wv - Wref) <= 1e-12 * abs(Wref)
    for t in range(4):
        nz = gref[t] != 0
        rel = np.abs(g[t][nz] - gref[t][nz]) / np.abs(gref[t][nz])
        assert rel.max() <= 1e-12, (t, rel.max())
        assert np.all(g[t][~nz] == 0)
    # central finite differences (exact for a multilinear W), 8 rows per table
    rng = np.random.default_rng(11)
    for t in range(4):
        rows = rng.choice(q.n_rows(t), 8, replace=False)
        fd = o.weighted_fd(w64, t, rows, threads=16)
        ref = g[t][rows]
        nz = fd != 0
        assert np.all(np.abs(ref[nz] - fd[nz]) <= 1e-12 * np.abs(fd[nz])), t
        assert np.all(ref[~nz] == 0), t
    # float32 weights: float64 accumulation, gradients rounded once
    Wref32, gref32 = o.weighted([x.astype(np.float64) for x in w32])
    Wv, g = _run(gctx, q, w32, torch.float32)
    assert abs(Wv - Wref32) <= 1e-12 * abs(Wref32)
    for t in range(4):
        ref = gref32[t].astype(np.float32).astype(np.float64)
        assert np.all(np.abs(g[t] - ref) <= np.abs(ref) * 2.0**-23), t
