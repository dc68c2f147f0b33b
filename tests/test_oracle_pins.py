"""Pins for the CPU oracle: brute force, closed forms, library routines and
orbit-sum invariants, all independent of the oracle's own arithmetic.

Every check here runs on the CPU.  The chain is:
  closed forms / networkx / matrix identities  -> pin oracle.brute (the definition)
  oracle.brute                                -> pins the C oracle (both formulations)
  C enumeration (definition) == C paper method -> on medium graphs
  orbit-sum invariants from independent global counts -> on every graph tried.
"""
from math import comb

import networkx as nx
import numpy as np
import pytest

import graphgen as gg
from oracle import brute


def _nx(g):
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    G.add_edges_from(map(tuple, g.edges().tolist()))
    return G


# --------------------------------------------------------------------------
# Closed forms for special graphs (derived from the definitions by counting).
# --------------------------------------------------------------------------

def kn_row(n):
    d = n - 1
    return [d, d * (d - 1), comb(d, 2), comb(d, 2), d * (d - 1) * (d - 2), d * (d - 1) * (d - 2),
            d * comb(d - 1, 2), comb(d, 3), 3 * comb(d, 3), d * comb(d - 1, 2),
            d * (d - 1) * (d - 2), comb(d, 2) * (d - 2), comb(d, 2) * (d - 2),
            d * comb(d - 1, 2), comb(d, 3)]


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_brute_complete_graph(n):
    psi = brute.orbit_counts_csr(*_csr(gg.complete(n)))
    for x in range(n):
        assert psi[x].tolist() == kn_row(n)


def test_k4_k5_rows_literal():
    assert kn_row(4) == [3, 6, 3, 3, 6, 6, 3, 1, 3, 3, 6, 3, 3, 3, 1]
    assert kn_row(5) == [4, 12, 6, 6, 24, 24, 12, 4, 12, 12, 24, 12, 12, 12, 4]


def _csr(g):
    return g.row_ptr, g.col


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_brute_star(k):
    psi = brute.orbit_counts_csr(*_csr(gg.star(k)))
    centre = [0] * 15
    centre[0], centre[2], centre[7] = k, comb(k, 2), comb(k, 3)
    leaf = [0] * 15
    leaf[0], leaf[1], leaf[6] = 1, k - 1, comb(k - 1, 2)
    assert psi[0].tolist() == centre
    for v in range(1, k + 1):
        assert psi[v].tolist() == leaf


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7, 8])
def test_brute_path(n):
    psi = brute.orbit_counts_csr(*_csr(gg.path(n)))
    for i in range(n):
        row = [0] * 15
        row[0] = (i > 0) + (i < n - 1)
        row[1] = (i - 2 >= 0) + (i + 2 < n)
        row[2] = 1 if 0 < i < n - 1 else 0
        row[4] = (i - 3 >= 0) + (i + 3 < n)
        # 4-vertex windows [s, s+3] with i at offset 1 or 2
        row[5] = sum(1 for s in range(0, n - 3) if i - s in (1, 2))
        assert psi[i].tolist() == row, (n, i)


@pytest.mark.parametrize("n", [3, 4, 5, 6, 7, 8])
def test_brute_cycle(n):
    psi = brute.orbit_counts_csr(*_csr(gg.cycle(n)))
    if n == 3:
        row = [2, 2, 1, 1] + [0] * 11
    elif n == 4:
        row = [2, 2, 1, 0, 2, 2, 0, 0, 1] + [0] * 6
    else:
        row = [2, 2, 1, 0, 2, 2] + [0] * 9
    for x in range(n):
        assert psi[x].tolist() == row


def test_brute_tailed_triangle_and_diamond_roles():
    # tailed triangle: hub 0, triangle 0-1-2, tail 3 on the hub
    paw = gg.from_edges(4, [0, 0, 1, 0], [1, 2, 2, 3])
    p = brute.orbit_counts_csr(*_csr(paw))
    assert p[3, 9] == 1 and p[1, 10] == 1 and p[2, 10] == 1 and p[0, 11] == 1
    assert p[:, 12:].sum() == 0 and p[:, 8].sum() == 0
    # diamond: 1-2 is the shared edge, 0 and 3 the degree-2 vertices
    dia = gg.from_edges(4, [0, 0, 1, 1, 2], [1, 2, 2, 3, 3])
    q = brute.orbit_counts_csr(*_csr(dia))
    assert q[0, 12] == 1 and q[3, 12] == 1 and q[1, 13] == 1 and q[2, 13] == 1
    assert q[:, 14].sum() == 0
    # the diamond contains one 4-cycle (through all four vertices)
    assert q[:, 8].tolist() == [1, 1, 1, 1]
    # and four tailed triangles (drop one of the four outer edges)
    assert q[:, 9].sum() == 4 and q[:, 11].sum() == 4 and q[:, 10].sum() == 8


def test_brute_automorphism_orbits_match_degree_classes():
    # classify() raises if an orbit of Aut(G') is not exactly a degree class
    for e in ([(0, 1), (1, 2), (2, 3)], [(0, 1), (0, 2), (0, 3)], [(0, 1), (1, 2), (2, 3), (3, 0)],
              [(0, 1), (0, 2), (1, 2), (0, 3)], [(0, 1), (0, 2), (1, 2), (1, 3), (2, 3)],
              [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]):
        brute.classify(range(4), e)


# --------------------------------------------------------------------------
# Library pins: networkx triangles, cliques, cycles.
# --------------------------------------------------------------------------

def _random_tiny(count, seed, nmax=10):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        n = int(rng.integers(1, nmax + 1))
        p = float(rng.choice([0.1, 0.2, 0.35, 0.5, 0.7, 0.85, 1.0]))
        yield gg.er_gnp(n, p, int(rng.integers(0, 2**31 - 1)))


def test_brute_vs_networkx():
    for g in _random_tiny(60, 7, 9):
        psi = brute.orbit_counts_csr(*_csr(g))
        G = _nx(g)
        tri = nx.triangles(G)
        k4 = np.zeros(g.n, np.int64)
        for c in nx.enumerate_all_cliques(G):
            if len(c) == 4:
                k4[c] += 1
            if len(c) > 4:
                break
        c4 = np.zeros(g.n, np.int64)
        for cyc in nx.simple_cycles(G, length_bound=4):
            if len(cyc) == 4:
                c4[cyc] += 1
        assert psi[:, 0].tolist() == [G.degree(v) for v in range(g.n)]
        assert psi[:, 3].tolist() == [tri[v] for v in range(g.n)]
        assert psi[:, 14].tolist() == k4.tolist()
        assert psi[:, 8].tolist() == c4.tolist()


# --------------------------------------------------------------------------
# The C oracle (both formulations) against the brute force.
# --------------------------------------------------------------------------

def test_c_oracle_vs_brute_random(oracle_lib):
    bad = 0
    checked = 0
    for g in _random_tiny(1000, 11, 10):
        b = brute.orbit_counts_csr(*_csr(g))
        c = oracle_lib.count(g.row_ptr, g.col)
        e = oracle_lib.enum_count(g.row_ptr, g.col)
        checked += 1
        if not (np.array_equal(b, c) and np.array_equal(b, e)):
            bad += 1
    assert checked == 1000 and bad == 0


def test_c_oracle_vs_brute_structured(oracle_lib):
    graphs = [gg.complete(7), gg.star(8), gg.path(9), gg.cycle(4), gg.cycle(9), gg.empty(5),
              gg.barabasi_albert(12, 3, seed=3),
              gg.disjoint_union([gg.complete(4), gg.cycle(5), gg.empty(2), gg.star(3)]),
              gg.relabel_random(gg.planted_cliques(12, 0.2, [5], seed=5), seed=9)]
    for g in graphs:
        b = brute.orbit_counts_csr(*_csr(g))
        assert np.array_equal(oracle_lib.count(g.row_ptr, g.col), b), g.name
        assert np.array_equal(oracle_lib.enum_count(g.row_ptr, g.col), b), g.name


def test_c_oracle_empty_graph(oracle_lib):
    g = gg.empty(0)
    assert oracle_lib.count(g.row_ptr, g.col).shape == (0, 15)
    g = gg.empty(3)
    assert not oracle_lib.count(g.row_ptr, g.col).any()


def test_c_oracle_closed_forms_larger(oracle_lib):
    for n in (10, 25):
        psi = oracle_lib.count(*_csr(gg.complete(n)))
        assert (psi == np.array(kn_row(n))).all()
    psi = oracle_lib.count(*_csr(gg.star(300)))
    assert psi[0, 7] == comb(300, 3) and psi[1, 6] == comb(299, 2)


# --------------------------------------------------------------------------
# Medium graphs: the definition (enumeration) against the paper method, Stage I/II
# intermediates against networkx, and the per-vertex entry against the full run.
# --------------------------------------------------------------------------

MEDIUM = [
    lambda: gg.config_graph("er_tiny"),
    lambda: gg.complete(30),
    lambda: gg.er_gnp(200, 0.3, seed=4),
    lambda: gg.planted_cliques(400, 0.02, [14, 10, 8, 6], seed=6),
    lambda: gg.barabasi_albert(600, 5, seed=8),
    lambda: gg.chung_lu(3000, 2.2, 8.0, 300.0, seed=2),
]


@pytest.mark.parametrize("make", MEDIUM)
def test_c_paper_method_vs_enumeration(oracle_lib, make):
    g = make()
    assert np.array_equal(oracle_lib.count(g.row_ptr, g.col), oracle_lib.enum_count(g.row_ptr, g.col))


@pytest.mark.parametrize("make", MEDIUM[:4])
def test_c_stage_intermediates_vs_networkx(oracle_lib, make):
    g = make()
    G = _nx(g)
    tri = oracle_lib.stage1(g.row_ptr, g.col)
    src = np.repeat(np.arange(g.n), g.degrees())
    for s in range(0, g.nnz, max(1, g.nnz // 2000)):
        u, v = int(src[s]), int(g.col[s])
        assert tri[s] == len(list(nx.common_neighbors(G, u, v)))
    k4 = oracle_lib.stage2(g.row_ptr, g.col)
    ref = np.zeros(g.n, np.int64)
    for c in nx.enumerate_all_cliques(G):
        if len(c) == 4:
            ref[c] += 1
        elif len(c) > 4:
            break
    assert np.array_equal(k4, ref)


@pytest.mark.parametrize("make", MEDIUM)
def test_c_orbits_at_matches_full(oracle_lib, make):
    g = make()
    full, tri, k4, fv = oracle_lib.count_with_intermediates(g.row_ptr, g.col)
    xs = np.unique(np.concatenate([np.arange(0, g.n, 7), np.argsort(-g.degrees())[:5]])).astype(np.int32)
    psi, fva = oracle_lib.orbits_at(g.row_ptr, g.col, xs, want_fvars=True)
    assert np.array_equal(psi, full[xs])
    assert np.array_equal(fva, fv[xs])


# --------------------------------------------------------------------------
# Orbit-sum invariants: column sums equal graphlet counts times the number of
# vertices of that graphlet in the orbit; the graphlet counts come from matrix
# identities and networkx, not from the oracle.
# --------------------------------------------------------------------------

def global_counts(g):
    A = np.zeros((g.n, g.n), dtype=np.int64)
    e = g.edges()
    A[e[:, 0], e[:, 1]] = 1
    A[e[:, 1], e[:, 0]] = 1
    d = A.sum(1)
    A2 = A @ A
    m = len(e)
    tri_v = np.diag(A2 @ A) // 2            # triangles at v
    T = int(tri_v.sum() // 3)
    t_e = A2[e[:, 0], e[:, 1]]             # common neighbours per edge
    closed4 = int(np.trace(A2 @ A2))
    c4 = (closed4 - 2 * int((d * d).sum()) + 2 * m) // 8
    G = _nx(g)
    k4 = sum(1 for c in nx.enumerate_all_cliques(G) if len(c) == 4)
    return dict(d=d, m=m, T=T, tri_v=tri_v, t_e=t_e, c4=c4, k4=k4, e=e)


def check_invariants(psi, gc):
    d, m, T = gc["d"], gc["m"], gc["T"]
    e, t_e, tri_v = gc["e"], gc["t_e"], gc["tri_v"]
    s = psi.sum(0)
    c2 = int(sum(comb(int(x), 2) for x in d))
    c3 = int(sum(comb(int(x), 3) for x in d))
    p4 = int(((d[e[:, 0]] - 1) * (d[e[:, 1]] - 1)).sum()) - 3 * T
    tt = int((tri_v * (d - 2)).sum())
    dia = int(sum(comb(int(t), 2) for t in t_e))
    assert s[0] == 2 * m
    assert s[1] == 2 * c2 and s[2] == c2
    assert s[3] == 3 * T
    assert s[4] == 2 * p4 and s[5] == 2 * p4
    assert s[6] == 3 * c3 and s[7] == c3
    assert s[8] == 4 * gc["c4"]
    assert s[9] == tt and s[11] == tt and s[10] == 2 * tt
    assert s[12] == 2 * dia and s[13] == 2 * dia
    assert s[14] == 4 * gc["k4"]


@pytest.mark.parametrize("make", [
    lambda: gg.er_gnp(300, 0.05, seed=1),
    lambda: gg.er_gnp(120, 0.4, seed=2),
    lambda: gg.planted_cliques(300, 0.03, [12, 8], seed=3),
    lambda: gg.barabasi_albert(400, 4, seed=4),
    lambda: gg.chung_lu(800, 2.2, 10.0, 200.0, seed=5),
])
def test_c_oracle_invariants(oracle_lib, make):
    g = make()
    check_invariants(oracle_lib.count(g.row_ptr, g.col), global_counts(g))


@pytest.mark.parametrize("make", MEDIUM)
def test_c_stage23_at_matches_full(oracle_lib, make):
    """Stages II and III on selected vertices from the whole graph's Stage I counts
    (the CPU baseline's timed sample) equal the full three-stage run."""
    g = make()
    full = oracle_lib.count(g.row_ptr, g.col)
    tri = oracle_lib.stage1(g.row_ptr, g.col)
    xs = np.unique(np.concatenate([np.arange(0, g.n, 5), np.argsort(-g.degrees())[:5]])).astype(np.int32)
    assert np.array_equal(oracle_lib.stage23_at(g.row_ptr, g.col, tri, xs), full[xs])
