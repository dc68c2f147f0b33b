"""Pins for the oracle's induced counts and its whole-graph counts (4-cycles,
4-cliques, 4-cliques through each edge), all on the CPU.

  * induced orbit counts (Section 3, Definition 2): Python brute force with the
    induced classification, closed forms, and the linear relation between
    non-induced and induced counts with its matrix derived here from the nine
    graphlets by brute force (the relation the section on ORCA and NI-ORCA uses,
    including its three printed induced equations);
  * #C4, #K4: adjacency-matrix identities, networkx cliques and cycles, closed
    forms, and the orbit sums of the definition-level enumeration;
  * 4-cliques per edge: networkx cliques, the closed form for K_n, and its sums;
  * planted mistakes in copies of the C source, each rejected by these pins.
"""
import ctypes
import itertools
import os
import subprocess
import tempfile
from math import comb

import networkx as nx
import numpy as np
import pytest

import graphgen as gg
from oracle import brute

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "niorca_ref.c")

from orbit_relations import GRAPHLETS, subgraph_matrix


def _random_tiny(count, seed, nmax=9):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        n = int(rng.integers(1, nmax + 1))
        p = float(rng.choice([0.15, 0.3, 0.5, 0.7, 0.9, 1.0]))
        yield gg.er_gnp(n, p, int(rng.integers(0, 2**31 - 1)))


# --------------------------------------------------------------------------
# Induced counts
# --------------------------------------------------------------------------

def test_subgraph_matrix_shape_and_printed_induced_equations():
    C = subgraph_matrix()
    # unit upper triangular in this numbering: more edges -> more subgraphs
    assert np.array_equal(np.diag(C), np.ones(15, np.int64))
    assert not np.tril(C, -1).any()
    # the three induced equations printed with ORCA's: with K4 = psi_14,
    #   psi'_13 = psi_13 - 3 psi_14, psi'_11 = psi_11 - 2 psi_13 + 3 psi_14,
    #   psi'_10 = psi_10 - 2 psi_12 - 2 psi_13 + 6 psi_14
    # (in f-variables: f13/2 - 3 K4, (f11 - f13)/2 + 3 K4, f10 - f13 + 6 K4)
    Ci = np.rint(np.linalg.inv(C.astype(float))).astype(np.int64)
    assert np.array_equal(Ci @ C, np.eye(15, dtype=np.int64))
    assert Ci[13].tolist() == [0] * 13 + [1, -3]
    assert Ci[11].tolist() == [0] * 11 + [1, 0, -2, 3]
    assert Ci[10].tolist() == [0] * 10 + [1, 0, -2, -2, 6]


def test_brute_induced_closed_forms():
    for n in (2, 3, 4, 5, 6):
        psi = brute.orbit_counts_csr(gg.complete(n).row_ptr, gg.complete(n).col, induced=True)
        row = [0] * 15
        row[0], row[3], row[14] = n - 1, comb(n - 1, 2), comb(n - 1, 3)
        assert (psi == np.array(row)).all()
    for k in (2, 3, 5):
        g = gg.star(k)
        psi = brute.orbit_counts_csr(g.row_ptr, g.col, induced=True)
        # a star is a tree: every connected vertex set induces its only spanning tree
        assert np.array_equal(psi, brute.orbit_counts_csr(g.row_ptr, g.col))
    g = gg.cycle(4)
    psi = brute.orbit_counts_csr(g.row_ptr, g.col, induced=True)
    assert (psi == np.array([2, 2, 1, 0, 0, 0, 0, 0, 1] + [0] * 6)).all()


def test_brute_induced_single_graphlet_roles():
    """A graphlet on its own: its vertex set is one induced occurrence of itself."""
    for name, (k, es) in GRAPHLETS.items():
        u, v = zip(*es)
        g = gg.from_edges(k, np.array(u), np.array(v), name)
        psi = brute.orbit_counts_csr(g.row_ptr, g.col, induced=True)
        top = brute.classify(list(range(k)), es)
        lo, hi = {2: (0, 1), 3: (1, 4), 4: (4, 15)}[k]
        for x in range(k):
            assert psi[x, lo:hi].sum() == 1 and psi[x, top[x]] == 1


def test_c_induced_vs_brute(oracle_lib):
    bad = 0
    for g in _random_tiny(400, 21):
        b = brute.orbit_counts_csr(g.row_ptr, g.col, induced=True)
        if not np.array_equal(oracle_lib.enum_induced(g.row_ptr, g.col), b):
            bad += 1
    assert bad == 0


@pytest.mark.parametrize("make", [
    lambda: gg.config_graph("er_tiny"),
    lambda: gg.planted_cliques(300, 0.03, [12, 8, 5], seed=3),
    lambda: gg.barabasi_albert(400, 4, seed=4),
    lambda: gg.er_gnp(80, 0.35, seed=5),
])
def test_noninduced_equals_subgraph_matrix_times_induced(oracle_lib, make):
    """psi = C psi', row by row, with both sides from the definition-level C oracle."""
    g = make()
    C = subgraph_matrix()
    ni = oracle_lib.enum_count(g.row_ptr, g.col)
    ind = oracle_lib.enum_induced(g.row_ptr, g.col)
    assert np.array_equal(ind @ C.T, ni)


# --------------------------------------------------------------------------
# Whole-graph 4-cycles and 4-cliques
# --------------------------------------------------------------------------

def _nx(g):
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    G.add_edges_from(map(tuple, g.edges().tolist()))
    return G


def _c4_trace(g):
    """#C4 from closed 4-walks: tr(A^4) = 8 C4 + 2 sum d^2 - 2m."""
    A = np.zeros((g.n, g.n), dtype=np.int64)
    e = g.edges()
    A[e[:, 0], e[:, 1]] = 1
    A[e[:, 1], e[:, 0]] = 1
    d = A.sum(1)
    A2 = A @ A
    return (int(np.trace(A2 @ A2)) - 2 * int((d * d).sum()) + 2 * len(e)) // 8


def _k4_nx(g):
    return sum(1 for c in nx.enumerate_all_cliques(_nx(g)) if len(c) == 4)


def test_totals_random_tiny(oracle_lib):
    for g in _random_tiny(300, 5, 11):
        assert oracle_lib.cycles4_total(g.row_ptr, g.col) == _c4_trace(g)
        assert oracle_lib.k4_total(g.row_ptr, g.col) == _k4_nx(g)


def test_totals_closed_forms(oracle_lib):
    for n in (1, 4, 5, 9, 40):
        g = gg.complete(n)
        assert oracle_lib.k4_total(g.row_ptr, g.col) == comb(n, 4)
        assert oracle_lib.cycles4_total(g.row_ptr, g.col) == 3 * comb(n, 4)
    for a, b in ((2, 7), (3, 5), (6, 6)):
        u = np.repeat(np.arange(a), b)
        v = a + np.tile(np.arange(b), a)
        g = gg.from_edges(a + b, u, v)
        assert oracle_lib.cycles4_total(g.row_ptr, g.col) == comb(a, 2) * comb(b, 2)
        assert oracle_lib.k4_total(g.row_ptr, g.col) == 0
    for n in (3, 4, 5, 12):
        g = gg.cycle(n)
        assert oracle_lib.cycles4_total(g.row_ptr, g.col) == (1 if n == 4 else 0)
    g = gg.empty(0)
    assert oracle_lib.cycles4_total(g.row_ptr, g.col) == 0 and oracle_lib.k4_total(g.row_ptr, g.col) == 0


@pytest.mark.parametrize("make", [
    lambda: gg.config_graph("er_tiny"),
    lambda: gg.planted_cliques(400, 0.02, [14, 10, 8, 6], seed=6),
    lambda: gg.barabasi_albert(600, 5, seed=8),
    lambda: gg.chung_lu(3000, 2.2, 8.0, 300.0, seed=2),
    lambda: gg.relabel_random(gg.planted_cliques(500, 0.04, [16, 9], seed=7), seed=1),
])
def test_totals_match_enumeration_orbit_sums(oracle_lib, make):
    """Orbit sums of the definition-level enumeration: sum psi_8 = 4 #C4 and
    sum psi_14 = 4 #K4."""
    g = make()
    s = oracle_lib.enum_count(g.row_ptr, g.col).sum(0)
    assert s[8] == 4 * oracle_lib.cycles4_total(g.row_ptr, g.col)
    assert s[14] == 4 * oracle_lib.k4_total(g.row_ptr, g.col)


# --------------------------------------------------------------------------
# 4-cliques through each edge
# --------------------------------------------------------------------------

def _edge_k4_nx(g):
    """Per CSR slot: +1 for every 4-clique containing both ends (networkx cliques)."""
    out = np.zeros(g.nnz, dtype=np.int64)
    slot = {}
    src = np.repeat(np.arange(g.n), g.degrees())
    for s in range(g.nnz):
        slot[(int(src[s]), int(g.col[s]))] = s
    for c in nx.enumerate_all_cliques(_nx(g)):
        if len(c) == 4:
            for a, b in itertools.permutations(c, 2):
                out[slot[(a, b)]] += 1
        elif len(c) > 4:
            break
    return out


def test_edge_k4_vs_networkx(oracle_lib):
    for g in list(_random_tiny(200, 9, 10)) + [gg.planted_cliques(120, 0.05, [9, 6], seed=2)]:
        assert np.array_equal(oracle_lib.edge_k4(g.row_ptr, g.col), _edge_k4_nx(g))


def test_edge_k4_closed_form_and_sums(oracle_lib):
    g = gg.complete(12)
    assert (oracle_lib.edge_k4(g.row_ptr, g.col) == comb(10, 2)).all()
    g = gg.planted_cliques(500, 0.03, [13, 9, 7], seed=4)
    ek = oracle_lib.edge_k4(g.row_ptr, g.col)
    k4v = oracle_lib.enum_count(g.row_ptr, g.col)[:, 14]
    # each 4-clique has 6 edges (12 slots); each clique through x has 3 edges at x
    assert ek.sum() == 12 * oracle_lib.k4_total(g.row_ptr, g.col)
    rows = np.add.reduceat(ek, g.row_ptr[:-1]) if g.nnz else ek
    rows[g.degrees() == 0] = 0
    assert np.array_equal(rows, 3 * k4v)
    # the listed-slot form agrees with the full form
    sl = np.arange(0, g.nnz, 7)
    assert np.array_equal(oracle_lib.edge_k4(g.row_ptr, g.col, sl), ek[sl])


# --------------------------------------------------------------------------
# Planted mistakes
# --------------------------------------------------------------------------

MUTANTS = {
    "induced_counts_all_subsets": ("oref_enum_induced", [("    if (induced) {\n", "    if (0) {\n")]),
    "c4_counts_k_not_pairs": ("oref_cycles4_total", [("total += kc * (kc - 1) / 2;", "total += kc;")]),
    "c4_middles_above_top": ("oref_cycles4_total",
                             [("for (i64 s = R.rp[v]; s < R.rp[v + 1] && R.col[s] < v; s++)",
                               "for (i64 s = R.rp[v]; s < R.rp[v + 1] && R.col[s] != v; s++)")]),
    "c4_far_end_may_be_top": ("oref_cycles4_total",
                              [("q < R.rp[b + 1] && R.col[q] < v; q++)", "q < R.rp[b + 1] && R.col[q] <= v; q++)")]),
    "k4_rows_hold_lower_neighbours": ("oref_k4_total",
                                      [("q >= R.rp[v] && R.col[q] > v; q--)", "q >= R.rp[v]; q--)")]),
    "k4_counts_edges_not_triangles": ("oref_k4_total",
                                      [("total += __builtin_popcountll(rows[i * words + x] & rows[p * words + x]);",
                                        "total += (x == 0);")]),
    "edge_k4_ends_not_halved": ("oref_edge_k4", [("ek4[q] = ends / 2;", "ek4[q] = ends;")]),
    "c4_at_counts_x_itself": ("oref_cycles4_at", [("                        if (z == x) continue;\n", "")]),
    "edge_k4_union_not_common": ("oref_edge_k4", [("else { w[nw++] = col[i]; i++; j++; }",
                                                   "else { w[nw++] = col[i]; i++; j++; }\n                }\n"
                                                   "                while (i < rp[a + 1]) { if (col[i] != b) "
                                                   "w[nw++] = col[i]; i++; }\n                {")]),
}


def _build(name, edits, td):
    src = open(SRC).read()
    for old, new in edits:
        assert src.count(old) == 1, (name, old)
        src = src.replace(old, new)
    cpath, so = os.path.join(td, name + ".c"), os.path.join(td, name + ".so")
    open(cpath, "w").write(src)
    subprocess.run(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-w", "-o", so, cpath], check=True)
    return ctypes.CDLL(so)


def _call(lib, fn, g):
    P = ctypes.c_void_p
    rp, cl = g.row_ptr.ctypes.data_as(P), g.col.ctypes.data_as(P)
    f = getattr(lib, fn)
    if fn == "oref_cycles4_at":
        out = np.zeros(g.n, np.int64)
        f.argtypes = [ctypes.c_int32, P, P, ctypes.c_int32, P, P]
        xs = np.arange(g.n, dtype=np.int32)
        rc = f(g.n, rp, cl, g.n, xs.ctypes.data_as(P), out.ctypes.data_as(P))
    elif fn == "oref_enum_induced":
        out = np.zeros((g.n, 15), np.int64)
        f.argtypes = [ctypes.c_int32, P, P, P]
        rc = f(g.n, rp, cl, out.ctypes.data_as(P))
    elif fn == "oref_edge_k4":
        out = np.zeros(g.nnz, np.int64)
        f.argtypes = [ctypes.c_int32, P, P, ctypes.c_int64, P, P]
        rc = f(g.n, rp, cl, 0, None, out.ctypes.data_as(P))
    else:
        out = np.zeros(1, np.int64)
        f.argtypes = [ctypes.c_int32, P, P, P]
        rc = f(g.n, rp, cl, out.ctypes.data_as(P))
    return rc, out


def _expected(fn, g):
    if fn == "oref_cycles4_at":
        return brute.orbit_counts_csr(g.row_ptr, g.col)[:, 8]
    if fn == "oref_enum_induced":
        return brute.orbit_counts_csr(g.row_ptr, g.col, induced=True)
    if fn == "oref_edge_k4":
        return _edge_k4_nx(g)
    if fn == "oref_cycles4_total":
        return np.array([_c4_trace(g)])
    return np.array([_k4_nx(g)])


@pytest.fixture(scope="module")
def mutant_graphs():
    rng = np.random.default_rng(77)
    out = [gg.complete(6), gg.cycle(4), gg.from_edges(4, [0, 0, 1, 1, 2], [1, 2, 2, 3, 3])]
    for _ in range(60):
        n = int(rng.integers(4, 10))
        out.append(gg.er_gnp(n, float(rng.choice([0.4, 0.6, 0.8])), int(rng.integers(0, 2**31 - 1))))
    return out


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_global_mutant(name, mutant_graphs):
    fn, edits = MUTANTS[name]
    with tempfile.TemporaryDirectory() as td:
        lib = _build(name, edits, td)
        caught = any(rc != 0 or not np.array_equal(out, _expected(fn, g))
                     for g in mutant_graphs for rc, out in [_call(lib, fn, g)])
    assert caught, f"mutant {name} survived the pins"


def test_unmutated_global_functions_pass(mutant_graphs):
    with tempfile.TemporaryDirectory() as td:
        lib = _build("clean", [], td)
        for fn in ("oref_enum_induced", "oref_cycles4_total", "oref_k4_total", "oref_edge_k4", "oref_cycles4_at"):
            for g in mutant_graphs:
                rc, out = _call(lib, fn, g)
                assert rc == 0 and np.array_equal(out, _expected(fn, g)), (fn, g.name)


def test_cycles4_at_vs_enumeration(oracle_lib):
    """psi_8 of selected vertices from common-neighbour pairs equals the definition-
    level enumeration's column 8."""
    for g in [gg.config_graph("er_tiny"), gg.chung_lu(3000, 2.2, 8.0, 300.0, seed=2),
              gg.planted_cliques(400, 0.02, [14, 10, 8, 6], seed=6), gg.complete(12)]:
        xs = np.unique(np.concatenate([np.arange(0, g.n, 3), np.argsort(-g.degrees())[:4]])).astype(np.int32)
        ref = oracle_lib.enum_count(g.row_ptr, g.col)[xs, 8]
        assert np.array_equal(oracle_lib.cycles4_at(g.row_ptr, g.col, xs), ref)


@pytest.mark.parametrize("make", [
    lambda: gg.config_graph("er_tiny"),
    lambda: gg.chung_lu(3000, 2.2, 8.0, 300.0, seed=2),
    lambda: gg.planted_cliques(400, 0.02, [14, 10, 8, 6], seed=6),
    lambda: gg.barabasi_albert(600, 5, seed=8),
    lambda: gg.complete(11),
])
def test_direct_forms_vs_enumeration(oracle_lib, make):
    """The per-column direct forms the full-size GPU test applies to the highest-degree
    vertices, against the definition-level enumeration."""
    from test_gpu_fullsize import direct_forms
    g = make()
    ref = oracle_lib.enum_count(g.row_ptr, g.col)
    tri = oracle_lib.stage1(g.row_ptr, g.col)
    xs = np.unique(np.concatenate([np.arange(0, g.n, 4), np.argsort(-g.degrees())[:5]])).astype(np.int32)
    for k, got in direct_forms(g, tri, xs, oracle_lib).items():
        assert np.array_equal(got, ref[xs, k]), k
