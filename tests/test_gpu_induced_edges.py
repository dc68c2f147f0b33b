"""GPU parity of the induced orbit counts (NIORCA_INDUCED) and of the 4-cliques
through each edge (niorca_edge_k4), through the C ABI, bit-exact.

Induced counts: against the oracle's definition-level enumeration (Section 3,
Definition 2) where it finishes in seconds, and on larger graphs against the
oracle's non-induced counts mapped through the inverse of the subgraph relation
(derived by brute force on the nine graphlets, not taken from the kernel).

4-cliques per edge: against the oracle's per-edge count, in every Stage I/II work
class (forced by the class knobs and by binning), with and without the kept
triangle records, and the closed form C(n-2, 2) on complete graphs large enough
for the global-scratch class.
"""
import sys
from math import comb

import numpy as np
import pytest

import graphgen as gg
from orbit_relations import subgraph_matrix

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ni():
    import paper_2606_29651_amd as m
    m.load_library()
    return m


@pytest.fixture(scope="module")
def ora():
    import oracle
    oracle.build(force=False)
    return oracle


def _dev(g):
    import torch
    return torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col).cuda()


SMALL = {
    "K1": lambda: gg.complete(1),
    "K5": lambda: gg.complete(5),
    "K30": lambda: gg.complete(30),
    "star40": lambda: gg.star(40),
    "cycle4": lambda: gg.cycle(4),
    "path9": lambda: gg.path(9),
    "isolated": lambda: gg.empty(5),
    "er_tiny": lambda: gg.config_graph("er_tiny"),
    "er_dense": lambda: gg.er_gnp(120, 0.3, seed=4),
    "planted": lambda: gg.relabel_random(gg.planted_cliques(800, 0.01, [20, 14, 9, 6], seed=6), seed=3),
    "union": lambda: gg.disjoint_union([gg.complete(7), gg.star(40), gg.empty(3), gg.cycle(4),
                                        gg.er_gnp(300, 0.05, seed=9)]),
}
LARGER = {
    "ba": lambda: gg.barabasi_albert(3000, 6, seed=8),
    "chung_lu_small": lambda: gg.chung_lu(20000, 2.2, 10.0, 2000.0, seed=2),
    "rmat12": lambda: gg.rmat(12, 16, seed=5),
    "K600": lambda: gg.complete(600),
}


@pytest.mark.parametrize("name", sorted(SMALL))
def test_induced_matches_definition(ni, ora, name):
    g = SMALL[name]()
    _say(f"[gpu] induced {name} n={g.n}")
    rp, cl = _dev(g)
    got = ni.count(rp, cl, flags=ni.INDUCED | ni.VALIDATE).cpu().numpy()
    ref = ora.enum_induced(g.row_ptr, g.col)
    if not np.array_equal(got, ref):
        bad = np.argwhere(got != ref)
        pytest.fail(f"{len(bad)} entries differ, first (vertex, orbit) {bad[:8].tolist()}")


@pytest.mark.parametrize("name", sorted(LARGER))
def test_induced_matches_inverse_relation(ni, ora, name):
    g = LARGER[name]()
    _say(f"[gpu] induced {name} n={g.n}")
    rp, cl = _dev(g)
    got = ni.count(rp, cl, flags=ni.INDUCED).cpu().numpy()
    C = subgraph_matrix()
    Ci = np.rint(np.linalg.inv(C.astype(float))).astype(np.int64)
    assert np.array_equal(Ci @ C, np.eye(15, dtype=np.int64))
    ref = ora.count(g.row_ptr, g.col) @ Ci.T
    assert np.array_equal(got, ref)


def test_induced_batched_and_captured(ni, ora):
    import torch
    graphs = gg.batch_mix(60, 5, 300, seed=3) + [gg.complete(12), gg.cycle(4), gg.empty(2)]
    vtx_off, rp, col = gg.pack_batch(graphs)
    ref = np.concatenate([ora.enum_induced(g.row_ptr, g.col) for g in graphs])
    drp, dcol = torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()
    got = ni.count_batched(vtx_off, drp, dcol, flags=ni.INDUCED).cpu().numpy()
    assert np.array_equal(got, ref)
    ctx = ni.Context(0)
    stream = torch.cuda.Stream()
    try:
        out = torch.empty((int(vtx_off[-1]), 15), dtype=torch.int64, device="cuda")
        for _ in range(2):
            out.fill_(-1)
            torch.cuda.synchronize()
            ni.count_batched(vtx_off, drp, dcol, flags=ni.INDUCED | ni.GRAPH_CAPTURE, out=out, ctx=ctx,
                             stream=stream)
            stream.synchronize()
            assert np.array_equal(out.cpu().numpy(), ref)
            ctx.device_status(stream)
    finally:
        torch.cuda.synchronize()
        ctx.close()


EDGE_GRAPHS = {
    "K4": lambda: gg.complete(4),
    "K30": lambda: gg.complete(30),
    "K90": lambda: gg.complete(90),
    "planted": lambda: gg.relabel_random(gg.planted_cliques(800, 0.01, [20, 14, 9, 6], seed=6), seed=3),
    "er_dense": lambda: gg.er_gnp(200, 0.3, seed=4),
    "ba": lambda: gg.barabasi_albert(3000, 6, seed=8),
    "chung_lu_small": lambda: gg.chung_lu(20000, 2.2, 10.0, 2000.0, seed=2),
    "rmat12": lambda: gg.rmat(12, 16, seed=5),
    "union": lambda: gg.disjoint_union([gg.complete(7), gg.star(40), gg.empty(3), gg.cycle(4),
                                        gg.er_gnp(300, 0.05, seed=9)]),
}
EDGE_MODES = {
    "default": {},
    "all_block": dict(tri_wave=1),
    "all_large": dict(tri_wave=1, tri_block=1),
    "all_large_global": dict(tri_wave=1, tri_block=1, large_lds=0),
    "no_records": dict(tri_cache=0),
    "few_records": dict(tri_cache=2000, tri_wave=8),
    # one-lane and sixteen-lane classes, reached through degree binning
    "lanes": dict(bin_mode=1, bin_deg_thread=1 << 20, bin_deg_group=1 << 20),
    "groups": dict(bin_mode=1, bin_deg_thread=0, bin_deg_group=1 << 20),
}


@pytest.mark.parametrize("mode", sorted(EDGE_MODES))
@pytest.mark.parametrize("name", sorted(EDGE_GRAPHS))
def test_edge_k4_matches_oracle(ni, ora, name, mode):
    import torch
    g = EDGE_GRAPHS[name]()
    _say(f"[gpu] edge_k4 {name} {mode}")
    ctx = ni.Context(0)
    try:
        for k, v in EDGE_MODES[mode].items():
            ctx.set_param(k, v)
        rp, cl = _dev(g)
        got = ni.edge_k4(rp, cl, ctx=ctx).cpu().numpy()
        ctx.device_status()
        # the per-vertex counts of the same context agree with the per-edge ones
        k4v = ni.k4(rp, cl, ctx=ctx).cpu().numpy()
    finally:
        torch.cuda.synchronize()
        ctx.close()
    ref = ora.edge_k4(g.row_ptr, g.col)
    if not np.array_equal(got, ref):
        bad = np.flatnonzero(got != ref)
        pytest.fail(f"{len(bad)} slots differ, first {bad[:8].tolist()}: got {got[bad[:8]].tolist()} "
                    f"want {ref[bad[:8]].tolist()}")
    if g.nnz:
        cs = np.concatenate([[0], np.cumsum(got)])
        assert np.array_equal(cs[g.row_ptr[1:]] - cs[g.row_ptr[:-1]], 3 * k4v)


@pytest.mark.parametrize("n,large_lds", [(600, None), (600, 0), (1100, None)])
def test_edge_k4_complete_closed_form(ni, n, large_lds):
    """K_n: every edge lies in C(n-2, 2) 4-cliques; |N+| reaches n-1 > 480, the
    global-scratch Stage I class (large_lds = 0: everything in global memory)."""
    import torch
    g = gg.complete(n)
    ctx = ni.Context(0)
    try:
        if large_lds is not None:
            ctx.set_param("large_lds", large_lds)
        rp, cl = _dev(g)
        got = ni.edge_k4(rp, cl, ctx=ctx).cpu().numpy()
    finally:
        torch.cuda.synchronize()
        ctx.close()
    assert (got == comb(n - 2, 2)).all()


def test_device_status_after_each_entry_point(ni):
    import torch
    g = gg.planted_cliques(500, 0.03, [10, 7], seed=2)
    rp, cl = _dev(g)
    ctx = ni.Context(0)
    try:
        ctx.device_status()  # nothing counted yet
        for f in (lambda: ni.count(rp, cl, ctx=ctx), lambda: ni.edge_triangles(rp, cl, ctx=ctx),
                  lambda: ni.k4(rp, cl, ctx=ctx), lambda: ni.fvars(rp, cl, ctx=ctx),
                  lambda: ni.edge_k4(rp, cl, ctx=ctx), lambda: ni.count(rp, cl, ctx=ctx, flags=ni.INDUCED)):
            f()
            ctx.device_status()
    finally:
        torch.cuda.synchronize()
        ctx.close()
