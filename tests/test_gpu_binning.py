"""Learned work binning: counts never depend on the binning; counters and features
agree with host models of the same quantities; the MLP trains reproducibly and its
device predictions agree with a numpy forward pass."""
import sys

import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ni():
    import paper_2606_29651_amd as m
    m.load_library()
    return m


GRAPHS = {
    "chung_lu": lambda: gg.chung_lu(20000, 2.2, 10.0, 2000.0, seed=2),
    "rmat12": lambda: gg.rmat(12, 16, seed=5),
    "planted": lambda: gg.relabel_random(gg.planted_cliques(800, 0.01, [20, 14, 9, 6], seed=6), seed=3),
    "K40": lambda: gg.complete(40),
    "ba": lambda: gg.barabasi_albert(3000, 6, seed=8),
}
_G = {}


def graph(name):
    if name not in _G:
        _G[name] = GRAPHS[name]()
    return _G[name]


_REF = {}


def ref(name):
    if name not in _REF:
        import oracle
        oracle.build(force=False)
        g = graph(name)
        _REF[name] = oracle.count(g.row_ptr, g.col)
    return _REF[name]


def _dev(g):
    import torch
    return torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col).cuda()


def rank_model(g):
    """Host model of the degree orientation (ranks, N+ sizes)."""
    n = g.n
    d = g.degrees().astype(np.int64)
    order = np.lexsort((np.arange(n), d))
    rank = np.empty(n, np.int64)
    rank[order] = np.arange(n)
    src = np.repeat(np.arange(n), d)
    dst = g.col.astype(np.int64)
    up = rank[dst] > rank[src]
    dplus = np.bincount(src[up], minlength=n)
    probes = np.bincount(src[up], weights=dplus[dst[up]], minlength=n).astype(np.int64)
    return d, dplus, rank, probes, src, dst, up


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_counters_and_features(ni, name):
    import torch
    g = graph(name)
    _say(f"[gpu] counters {name}")
    ctx = ni.Context(0)
    try:
        rp, cl = _dev(g)
        psi = ni.count(rp, cl, flags=ni.COUNTERS, ctx=ctx)
        c = ni.work_counters(g.n, ctx=ctx).cpu().numpy()
        f = ni.last_features(g.n, ctx=ctx).cpu().numpy()
        torch.cuda.synchronize()
    finally:
        ctx.close()
    assert np.array_equal(psi.cpu().numpy(), ref(name))
    d, dplus, rank, probes, src, dst, up = rank_model(g)
    assert np.array_equal(c[:, 0], probes)
    assert np.array_equal(c[:, 5], 2 * d)
    # each triangle is found once, at its lowest-ranked vertex
    assert c[:, 1].sum() * 3 == ref(name)[:, 3].sum()
    # every Stage I item ran (items with no probe at all close no triangle and are
    # left out)
    assert (c[:, 6] >= 0).all() and (c[:, 6][(dplus >= 2) & (probes > 0)] > 0).all()
    nds = np.bincount(src, weights=d[dst], minlength=g.n)
    mx = np.zeros(g.n)
    np.maximum.at(mx, src[up], dplus[dst[up]])
    expect = np.log2(1.0 + np.stack([d, dplus, d - dplus, nds, probes, mx], axis=1)).astype(np.float32)
    assert np.allclose(f, expect, rtol=1e-5, atol=1e-5)


def stage1_work(c):
    """Operation-count work of a Stage I/II item from its counters."""
    return c[:, 0] + 4 * c[:, 1] + c[:, 2]


def _trained_model(ni, ctx):
    import torch
    g = graph("chung_lu")
    rp, cl = _dev(g)
    ni.count(rp, cl, flags=ni.COUNTERS, ctx=ctx)
    c = ni.work_counters(g.n, ctx=ctx)
    X = ni.last_features(g.n, ctx=ctx)
    keep = c[:, 6] > 0
    y = torch.log2(1.0 + stage1_work(c[keep]).double()).float()
    return X[keep].contiguous(), y


def test_mlp_learns_a_synthetic_target(ni):
    import torch
    g = torch.Generator(device="cuda").manual_seed(5)
    X = torch.rand((20000, 6), device="cuda", generator=g) * 10
    y = (2 * X[:, 4] - X[:, 1] + 0.05 * X[:, 0] * X[:, 3]).contiguous()
    ctx = ni.Context(0)
    try:
        model, mse = ni.mlp_train(X, y, epochs=40, batch=1024, lr=3e-3, seed=2, ctx=ctx)
        var = float(torch.var(y.double()))
    finally:
        ctx.close()
    assert mse < 0.02 * var, (mse, var)


def test_mlp_training_is_reproducible_and_learns(ni):
    import torch
    ctx = ni.Context(0)
    try:
        X, y = _trained_model(ni, ctx)
        m1, mse1 = ni.mlp_train(X, y, epochs=30, batch=1024, lr=3e-3, seed=7, ctx=ctx)
        m2, mse2 = ni.mlp_train(X, y, epochs=30, batch=1024, lr=3e-3, seed=7, ctx=ctx)
        var = float(torch.var(y.double()))
    finally:
        ctx.close()
    assert np.array_equal(m1, m2) and mse1 == mse2
    assert mse1 < 0.2 * var, (mse1, var)


def numpy_forward(model, X):
    W1 = model[0:192].reshape(32, 6)
    b1 = model[192:224]
    W2 = model[224:1248].reshape(32, 32)
    b2 = model[1248:1280]
    W3 = model[1280:1312]
    b3 = model[1312]
    mean, istd = model[1313:1319], model[1319:1325]
    x = (X.astype(np.float64) - mean) * istd
    h1 = np.maximum(x @ W1.T.astype(np.float64) + b1, 0)
    h2 = np.maximum(h1 @ W2.T.astype(np.float64) + b2, 0)
    return h2 @ W3.astype(np.float64) + b3


def test_mlp_predict_matches_numpy(ni):
    import torch
    ctx = ni.Context(0)
    try:
        X, y = _trained_model(ni, ctx)
        model, _ = ni.mlp_train(X, y, epochs=1, batch=2048, lr=3e-3, seed=3, ctx=ctx)
        pred = ni.mlp_predict(model, X, ctx=ctx).cpu().numpy()
    finally:
        ctx.close()
    ref_pred = numpy_forward(model, X.cpu().numpy())
    assert np.allclose(pred, ref_pred, rtol=1e-4, atol=1e-4)


MODES = {
    "degree_default": ("deg", {}),
    "degree_all_thread": ("deg", {"bin_deg_thread": 1 << 30, "bin_deg_block": 1 << 30}),
    "degree_all_block": ("deg", {"bin_deg_thread": 0, "bin_deg_block": 1}),
    "mlp_mid": ("mlp", (8.0, 14.0)),
    "mlp_all_thread": ("mlp", (1e9, 2e9)),
    "mlp_all_block": ("mlp", (-1e9, -1e9)),
    "degree_all_group": ("deg", {"bin_deg_thread": 0, "bin_deg_group": 1 << 30, "bin_deg_block": 1 << 30}),
    "mlp_group": ("mlp", (8.0, 15.0, 12.0)),
    "mlp_all_group": ("mlp", (-1e9, 2e9, 1e9)),
}


@pytest.mark.parametrize("mode", sorted(MODES))
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_binning_never_changes_counts(ni, mode, name):
    import torch
    kind, arg = MODES[mode]
    g = graph(name)
    _say(f"[gpu] binning {mode} {name}")
    ctx = ni.Context(0)
    try:
        if kind == "deg":
            for k, v in arg.items():
                ctx.set_param(k, v)
            flags = ni.BIN_DEGREE
        else:
            X, y = _trained_model(ni, ctx)
            model, _ = ni.mlp_train(X, y, epochs=1, batch=4096, lr=3e-3, seed=1, ctx=ctx)
            ni.set_cost_model(model, *arg, ctx=ctx)
            flags = ni.BIN_MLP
        rp, cl = _dev(g)
        got = ni.count(rp, cl, flags=flags, ctx=ctx).cpu().numpy()
        torch.cuda.synchronize()
    finally:
        ctx.close()
    assert np.array_equal(got, ref(name))
