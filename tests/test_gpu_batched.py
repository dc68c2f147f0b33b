"""Batched counting: many packed graphs in one call, and the hipGraph-captured
form replayed several times with other eager work on the same context and
stream synchronisations in between; every result is checked against the CPU
oracle graph by graph.  The measured batch itself (50,000 ER/BA graphs of 20 to
2000 vertices, seed 42) is checked whole, at the library's default knobs and at
the tuned knobs the bench times (paper_2606_29651_amd/tuning.txt), captured."""
import os
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


@pytest.fixture(scope="module")
def batch():
    import oracle
    oracle.build(force=False)
    graphs = gg.batch_mix(160, 5, 400, seed=11)
    graphs += [gg.complete(20), gg.star(60), gg.empty(3), gg.cycle(4), gg.path(7), gg.complete(1),
               gg.planted_cliques(300, 0.03, [12, 7], seed=2), gg.barabasi_albert(900, 8, seed=4)]
    vtx_off, rp, col = gg.pack_batch(graphs)
    ref = np.concatenate([oracle.count(g.row_ptr, g.col) for g in graphs])
    return graphs, vtx_off, rp, col, ref


def _check(got, ref, vtx_off):
    if not np.array_equal(got, ref):
        bad = np.argwhere(got != ref)
        g = np.searchsorted(vtx_off, bad[0][0], side="right") - 1
        pytest.fail(f"{len(bad)} entries differ; first at packed row {bad[0][0]} (graph {g}), orbit {bad[0][1]}")


def test_batched_matches_oracle(ni, batch):
    import torch
    graphs, vtx_off, rp, col, ref = batch
    _say(f"[gpu] batched {len(graphs)} graphs, {vtx_off[-1]} vertices")
    got = ni.count_batched(vtx_off, torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda(),
                           flags=ni.VALIDATE).cpu().numpy()
    _check(got, ref, vtx_off)


def test_batched_graph_capture_replays(ni, batch):
    import torch
    graphs, vtx_off, rp, col, ref = batch
    _say("[gpu] batched capture")
    ctx = ni.Context(0)
    stream = torch.cuda.Stream()
    drp, dcol = torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()
    out = torch.empty((int(vtx_off[-1]), 15), dtype=torch.int64, device="cuda")
    other = gg.chung_lu(5000, 2.2, 8.0, 500.0, seed=3)
    orp, ocol = torch.from_numpy(other.row_ptr).cuda(), torch.from_numpy(other.col).cuda()
    import oracle
    oref = oracle.count(other.row_ptr, other.col)
    try:
        for rep in range(3):
            out.fill_(-1)
            torch.cuda.synchronize()
            ni.count_batched(vtx_off, drp, dcol, flags=ni.GRAPH_CAPTURE, out=out, ctx=ctx, stream=stream)
            stream.synchronize()
            _check(out.cpu().numpy(), ref, vtx_off)
            # eager work on the same context between replays (it reuses the workspace)
            got = ni.count(orp, ocol, ctx=ctx).cpu().numpy()
            torch.cuda.synchronize()
            assert np.array_equal(got, oref)
    finally:
        torch.cuda.synchronize()
        ctx.close()


def test_batched_rejects_bad_offsets(ni):
    import torch
    g = gg.complete(4)
    vtx_off, rp, col = gg.pack_batch([g, g])
    bad = vtx_off.copy()
    bad[1] = 5  # decreasing afterwards? 0,5,8: graph 1 would have 3 vertices -> ids out of range locally
    with pytest.raises(ValueError):
        ni.count_batched(np.array([0, 3]), torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda())
    with pytest.raises(ni.NiorcaError):
        ni.count_batched(np.array([0, 9, 8]), torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda())


TUNING = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2606_29651_amd",
                      "tuning.txt")


@pytest.fixture(scope="module")
def big_batch():
    """The bench's batch and the oracle's counts of it (unions of 5000 graphs at a
    time, so the oracle's per-thread scratch stays small)."""
    import time
    import oracle
    oracle.build(force=False)
    t0 = time.time()
    graphs = gg.batch_mix(50000, 20, 2000, seed=42)
    vtx_off, rp, col = gg.pack_batch(graphs)
    _say(f"[gpu] batch_mix generated: {len(graphs)} graphs, n={vtx_off[-1]} in {time.time() - t0:.0f}s")
    t0 = time.time()
    parts = []
    for i in range(0, len(graphs), 5000):
        u = gg.disjoint_union(graphs[i:i + 5000])
        parts.append(oracle.count(u.row_ptr, u.col))
    ref = np.concatenate(parts)
    _say(f"[gpu] oracle on the whole batch in {time.time() - t0:.0f}s")
    return vtx_off, rp, col, ref


@pytest.mark.parametrize("knobs", ["default", "tuned"])
def test_measured_batch_matches_oracle(ni, big_batch, knobs):
    import torch
    from paper_2606_29651_amd import autotune
    vtx_off, rp, col, ref = big_batch
    ctx = ni.Context(0)
    stream = torch.cuda.Stream()
    try:
        if knobs == "tuned":
            assert autotune.load(TUNING, "batch_mix"), "no tuned knobs for batch_mix"
            ctx.load_tuning(TUNING, "batch_mix")
        drp, dcol = torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()
        out = torch.empty((int(vtx_off[-1]), 15), dtype=torch.int64, device="cuda")
        for rep in range(2):  # capture, then a replay
            out.fill_(-1)
            torch.cuda.synchronize()
            ni.count_batched(vtx_off, drp, dcol, flags=ni.GRAPH_CAPTURE, out=out, ctx=ctx, stream=stream)
            stream.synchronize()
            ctx.device_status(stream)
            _check(out.cpu().numpy(), ref, vtx_off)
            _say(f"[gpu] batch_mix {knobs} pass {rep} equal to the oracle")
    finally:
        torch.cuda.synchronize()
        ctx.close()


def test_batched_row_longer_than_bound_is_refused(ni):
    """A row with more entries than its graph has other vertices (here duplicates)
    would overrun buffers sized from that bound: the degree pass refuses it and
    niorca_device_status reports it; the other graphs are still counted."""
    import oracle
    import torch
    good = gg.complete(6)
    bad_g = gg.complete(5)
    vtx_off, rp, col = gg.pack_batch([good, bad_g])
    # graph 1, vertex 0: its row [1, 2, 3, 4] becomes [1, 1, 2, 2, 3, 3, 4, 4] (8 > 5 - 1)
    r0, r1 = int(rp[6]), int(rp[7])
    row = np.repeat(col[r0:r1], 2)
    col2 = np.concatenate([col[:r0], row, col[r1:]]).astype(np.int32)
    rp2 = rp.copy()
    rp2[7:] += len(row) - (r1 - r0)
    ctx = ni.Context(0)
    try:
        out = ni.count_batched(vtx_off, torch.from_numpy(rp2).cuda(), torch.from_numpy(col2).cuda(), ctx=ctx)
        with pytest.raises(ni.NiorcaError) as e:
            ctx.device_status()
        assert e.value.status == ni.EINVAL
        got = out.cpu().numpy()
        assert np.array_equal(got[:6], oracle.count(good.row_ptr, good.col))
    finally:
        torch.cuda.synchronize()
        ctx.close()
