"""niorca_count_noalloc (the fixed-scratch form of niorca_count for callers that
cannot allocate) through the raw C ABI: equal to niorca_count, bit for bit, on two
calls in a row, the second on a smaller graph (the shared scratch keeps the first
call's contents), in every work class the default knobs reach; and graphs too large
for the scratch are refused with ENOMEM, which names the size needed."""
import ctypes
import sys

import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _raw_noalloc(ni, ctx, g, out, flags=0):
    import torch
    rp, cl = torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col).cuda()
    P = ctypes.c_void_p
    rc = ni.load_library().niorca_count_noalloc(ctx.h, g.n, g.nnz, P(rp.data_ptr()), P(cl.data_ptr() if g.nnz else 0),
                                                P(out.data_ptr()), None, flags)
    torch.cuda.synchronize()
    return rc


def _ref(ni, ctx, g, flags=0):
    import torch
    out = ni.count(torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col).cuda(), ctx=ctx, flags=flags)
    torch.cuda.synchronize()
    return out.cpu().numpy()


PAIRS = {
    # first graph, then a smaller one that reuses the same scratch
    "chung_lu_then_planted": (lambda: gg.chung_lu(60000, 2.2, 10.0, 3000.0, seed=2),
                              lambda: gg.relabel_random(gg.planted_cliques(800, 0.01, [20, 14, 9, 6], seed=6), seed=3)),
    "rmat_then_er": (lambda: gg.rmat(14, 16, seed=5), lambda: gg.config_graph("er_tiny")),
    "k700_then_k30": (lambda: gg.complete(700), lambda: gg.complete(30)),
}


@pytest.mark.parametrize("flags_name", ["plain", "induced"])
@pytest.mark.parametrize("pair", sorted(PAIRS))
def test_noalloc_equals_count_twice(pair, flags_name):
    import torch
    import paper_2606_29651_amd as ni
    flags = ni.INDUCED if flags_name == "induced" else 0
    ctx = ni.Context(0)
    try:
        for step, make in enumerate(PAIRS[pair]):
            g = make()
            _say(f"[gpu] noalloc {pair} call {step}: n={g.n} m={g.m} flags={flags_name}")
            want = _ref(ni, ctx, g, flags)
            out = torch.full((g.n, 15), -1, dtype=torch.int64, device="cuda")
            rc = _raw_noalloc(ni, ctx, g, out, flags)
            assert rc == ni.OK, ni.load_library().niorca_last_error(ctx.h)
            ctx.device_status()
            assert np.array_equal(out.cpu().numpy(), want)
    finally:
        torch.cuda.synchronize()
        ctx.close()


def test_noalloc_refuses_graph_beyond_scratch():
    import torch
    import paper_2606_29651_amd as ni
    g = gg.config_graph("er_1m_8")  # 1M vertices, 8M slots: about 0.4 GB of workspace
    ctx = ni.Context(0)
    try:
        out = torch.empty((g.n, 15), dtype=torch.int64, device="cuda")
        rc = _raw_noalloc(ni, ctx, g, out)
        assert rc == ni.ENOMEM
        assert b"bytes of workspace" in ni.load_library().niorca_last_error(ctx.h)
        # the context still counts a graph that fits
        small = gg.config_graph("er_tiny")
        out2 = torch.empty((small.n, 15), dtype=torch.int64, device="cuda")
        assert _raw_noalloc(ni, ctx, small, out2) == ni.OK
        assert np.array_equal(out2.cpu().numpy(), _ref(ni, ctx, small))
    finally:
        torch.cuda.synchronize()
        ctx.close()
