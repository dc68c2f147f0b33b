"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit-exact.

Every comparison is element by element on int64 (orbits, K4, f-variables) or
int32 (per-edge triangles).  Graphs span several work classes and ragged tails;
the class thresholds are also forced so that every kernel shape runs on small
graphs (a vertex's counts never depend on which shape handled it).
"""
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
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2606_29651_amd as m
    m.load_library()
    return m


class _CachedOracle:
    """The CPU oracle with results memoised per graph name (the graphs are seeded)."""

    def __init__(self):
        import oracle
        oracle.build(force=False)
        self.o = oracle
        self.memo = {}

    def count(self, name, g):
        key = ("count", name)
        if key not in self.memo:
            self.memo[key] = self.o.count(g.row_ptr, g.col)
        return self.memo[key]

    def intermediates(self, name, g):
        key = ("inter", name)
        if key not in self.memo:
            self.memo[key] = self.o.count_with_intermediates(g.row_ptr, g.col)
        return self.memo[key]


@pytest.fixture(scope="module")
def ora():
    return _CachedOracle()


_GCACHE = {}


def graph(name):
    if name not in _GCACHE:
        _GCACHE[name] = GRAPHS[name]()
    return _GCACHE[name]


def _dev(g):
    import torch
    return torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col).cuda()


def bipartite_matched(a):
    """K_{a,a} plus a perfect matching on the right side and one left-left edge:
    left vertex 0 then has a+1 > 480 neighbours that all rank above it (the
    global-scratch Stage I class), with triangles and a few 4-cliques."""
    left = np.repeat(np.arange(a), a)
    right = a + np.tile(np.arange(a), a)
    mu = a + np.arange(0, a - 1, 2)
    return gg.from_edges(2 * a, np.concatenate([left, mu, [0]]), np.concatenate([right, mu + 1, [1]]),
                         f"bip_matched({a})")


def hub_band(k, width, leaves):
    """Vertex 0 joined to v_1..v_k; v_i joined to v_{i+1..i+width} and to `leaves`
    leaves of its own.  Every v_i outranks vertex 0, so vertex 0's Stage I item has k
    segments of about `width` probes each (short segments: with width 1 a block of
    2048 probes covers more than 256 segments)."""
    v = 1 + np.arange(k)
    us, ws = [np.zeros(k, np.int64)], [v]
    for d in range(1, width + 1):
        us.append(v[:-d]); ws.append(v[d:])
    lv = 1 + k + np.arange(k * leaves)
    us.append(np.repeat(v, leaves)); ws.append(lv)
    return gg.from_edges(1 + k + k * leaves, np.concatenate(us), np.concatenate(ws), f"hub_band({k},{width})")


GRAPHS = {
    "K1": lambda: gg.complete(1),
    "K2": lambda: gg.complete(2),
    "K4": lambda: gg.complete(4),
    "K30": lambda: gg.complete(30),
    "K90": lambda: gg.complete(90),
    "bip_hub": lambda: bipartite_matched(520),
    "hub_band1": lambda: hub_band(300, 1, 301),
    "hub_band20": lambda: hub_band(300, 20, 301),
    "star300": lambda: gg.star(300),
    "path50": lambda: gg.path(50),
    "cycle4": lambda: gg.cycle(4),
    "cycle41": lambda: gg.cycle(41),
    "isolated": lambda: gg.empty(17),
    "er_tiny": lambda: gg.config_graph("er_tiny"),
    "er_dense": lambda: gg.er_gnp(200, 0.3, seed=4),
    "planted": lambda: gg.relabel_random(gg.planted_cliques(800, 0.01, [20, 14, 9, 6], seed=6), seed=3),
    "ba": lambda: gg.barabasi_albert(3000, 6, seed=8),
    "chung_lu_small": lambda: gg.chung_lu(20000, 2.2, 10.0, 2000.0, seed=2),
    "rmat12": lambda: gg.rmat(12, 16, seed=5),
    "union": lambda: gg.disjoint_union([gg.complete(7), gg.star(40), gg.empty(3), gg.cycle(4),
                                        gg.er_gnp(300, 0.05, seed=9)]),
}


@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_count_matches_oracle(ni, ora, name):
    g = graph(name)
    _say(f"[gpu] count {name} n={g.n} m={g.m}")
    rp, cl = _dev(g)
    got = ni.count(rp, cl, flags=ni.VALIDATE).cpu().numpy()
    ref = ora.count(name, g)
    assert got.shape == ref.shape
    if not np.array_equal(got, ref):
        bad = np.argwhere(got != ref)
        pytest.fail(f"{len(bad)} entries differ, first (vertex, orbit) {bad[:8].tolist()}")


@pytest.mark.parametrize("name", ["K30", "bip_hub", "planted", "ba", "chung_lu_small", "rmat12", "er_tiny"])
def test_stage_intermediates(ni, ora, name):
    g = graph(name)
    _say(f"[gpu] stages {name} n={g.n}")
    rp, cl = _dev(g)
    ref_psi, ref_tri, ref_k4, ref_fv = ora.intermediates(name, g)
    assert np.array_equal(ni.edge_triangles(rp, cl).cpu().numpy(), ref_tri)
    assert np.array_equal(ni.k4(rp, cl).cpu().numpy(), ref_k4)
    assert np.array_equal(ni.fvars(rp, cl).cpu().numpy(), ref_fv)


FORCED = {
    "all_block": dict(tri_wave=1),
    "all_large": dict(tri_wave=1, tri_block=1),
    "all_large_global": dict(tri_wave=1, tri_block=1, large_lds=0),
    "tri_cache_none": dict(tri_cache=0),
    "tri_cache_small": dict(tri_cache=2000, tri_wave=8),
    "tri_cache_partial": dict(tri_cache=300000, tri_wave=8, tri_block=32),
    "qh_wave_small": dict(qh_wave=64, heavy_k=32768),
    "qh_wave_max": dict(qh_wave=2048, heavy_k=32768),
    "q_global_light": dict(ql_wave=0, ql_block=0, heavy_k=0),
    "q_block_light": dict(ql_wave=0, heavy_k=0),
    "q_block_light_max": dict(ql_wave=0, ql_block=8192, heavy_k=0),
    "q_block_light_split": dict(ql_wave=0, ql_block=8192, ql_split=64, heavy_k=0),
    "q_wave_light_max": dict(ql_wave=2048, heavy_k=0),
    "q_dense_heavy": dict(qh_wave=0, qh_block=0, heavy_k=32768),
    "q_block_heavy": dict(qh_wave=0, heavy_k=32768),
    "heavy_half": dict(heavy_k=500),
}


@pytest.mark.parametrize("mode", sorted(FORCED))
@pytest.mark.parametrize("name", ["K90", "planted", "chung_lu_small", "rmat12"])
def test_forced_classes(ni, ora, mode, name):
    g = graph(name)
    _say(f"[gpu] forced {mode} {name}")
    ctx = ni.Context(0)
    try:
        for k, v in FORCED[mode].items():
            ctx.set_param(k, v)
        rp, cl = _dev(g)
        got = ni.count(rp, cl, ctx=ctx).cpu().numpy()
    finally:
        import torch
        torch.cuda.synchronize()
        ctx.close()
    assert np.array_equal(got, ora.count(name, g))


def test_repeat_calls_reuse_workspace(ni, ora):
    ctx = ni.Context(0)
    try:
        for name in ("chung_lu_small", "K30", "chung_lu_small"):
            g = graph(name)
            rp, cl = _dev(g)
            got = ni.count(rp, cl, ctx=ctx).cpu().numpy()
            assert np.array_equal(got, ora.count(name, g))
    finally:
        ctx.close()


def kn_row(n):
    from math import comb
    d = n - 1
    return [d, d * (d - 1), comb(d, 2), comb(d, 2), d * (d - 1) * (d - 2), d * (d - 1) * (d - 2),
            d * comb(d - 1, 2), comb(d, 3), 3 * comb(d, 3), d * comb(d - 1, 2),
            d * (d - 1) * (d - 2), comb(d, 2) * (d - 2), comb(d, 2) * (d - 2),
            d * comb(d - 1, 2), comb(d, 3)]


@pytest.mark.parametrize("n,large_lds", [(600, None), (1500, None), (600, 30000), (600, 0)])
def test_complete_graph_closed_form(ni, n, large_lds):
    """K_n: every vertex has the same 15 counts, derived by counting (no oracle).
    |N+| reaches n-1 > 480, so the top vertices use the large class; large_lds picks
    its layout (default: bitset copied to LDS for the 4-clique pass; 30000: hash in
    LDS, bitset in global memory; 0: all in global memory)."""
    g = gg.complete(n)
    _say(f"[gpu] K{n} closed form, large_lds={large_lds}")
    ctx = ni.Context(0)
    try:
        if large_lds is not None:
            ctx.set_param("large_lds", large_lds)
        rp, cl = _dev(g)
        got = ni.count(rp, cl, ctx=ctx).cpu().numpy()
    finally:
        import torch
        torch.cuda.synchronize()
        ctx.close()
    assert (got == np.array(kn_row(n), dtype=np.int64)).all()


def k2n_rows(N):
    """K_{2,N}: hubs a, b (not adjacent) joined to N leaves of degree 2."""
    from math import comb
    hub = [N, N, comb(N, 2), 0, N * (N - 1), N * (N - 1), 0, comb(N, 3), comb(N, 2)] + [0] * 6
    leaf = [2, 2 * (N - 1), 1, 0, 2 * (N - 1), 2 * (N - 1), 2 * comb(N - 1, 2), 0, N - 1] + [0] * 6
    return hub, leaf


@pytest.mark.parametrize("N", [3000, 70000])
def test_k2n_closed_form(ni, ora, N):
    """K_{2,N}: with N >= 2^16 a 4-cycle count per (hub, hub) pair exceeds 16 bits,
    which routes the hub through the int32 global-counter class."""
    u = np.concatenate([np.zeros(N, np.int64), np.ones(N, np.int64)])
    v = np.concatenate([2 + np.arange(N), 2 + np.arange(N)])
    g = gg.from_edges(N + 2, u, v, f"K2,{N}")
    _say(f"[gpu] K2,{N} closed form")
    rp, cl = _dev(g)
    got = ni.count(rp, cl).cpu().numpy()
    hub, leaf = k2n_rows(N)
    assert got[0].tolist() == hub and got[1].tolist() == hub
    assert (got[2:] == np.array(leaf, dtype=np.int64)).all()
    if N <= 3000:
        assert np.array_equal(got, ora.count(f"K2,{N}", g))
