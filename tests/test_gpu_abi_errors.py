"""Error behaviour of the C ABI on the GPU: every documented status is reached
from the host, without any kernel faulting."""
import ctypes

import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ni():
    import paper_2606_29651_amd as m
    m.load_library()
    return m


def _raw(ni, ctx, n, nnz, rp, cl, out, flags=0):
    return ni.load_library().niorca_count(ctx.h, n, nnz, rp, cl, out, None, flags)


def test_argument_errors(ni):
    import torch
    ctx = ni.Context(0)
    lib = ni.load_library()
    g = gg.complete(5)
    rp = torch.from_numpy(g.row_ptr).cuda()
    cl = torch.from_numpy(g.col).cuda()
    out = torch.empty((5, 15), dtype=torch.int64, device="cuda")
    P = ctypes.c_void_p
    ok = lambda t: P(t.data_ptr())
    assert _raw(ni, ctx, -1, 0, None, None, None) == ni.EINVAL
    assert _raw(ni, ctx, 5, 19, ok(rp), ok(cl), ok(out)) == ni.EINVAL          # odd nnz
    assert _raw(ni, ctx, 5, 20, None, ok(cl), ok(out)) == ni.EINVAL            # NULL row_ptr
    assert _raw(ni, ctx, 5, 20, ok(rp), None, ok(out)) == ni.EINVAL            # NULL col
    assert _raw(ni, ctx, 5, 20, ok(rp), ok(cl), None) == ni.EINVAL             # NULL out
    assert _raw(ni, ctx, 5, 20, ok(rp), ok(cl), ok(out), 0x80) == ni.EINVAL    # unknown flag
    assert _raw(ni, ctx, 5, 22, ok(rp), ok(cl), ok(out)) == ni.EINVAL          # nnz > n(n-1)
    # slot ids are int32: 2^31 slots are refused on the host, before any buffer is read
    assert _raw(ni, ctx, 100000, 1 << 31, ok(rp), ok(cl), ok(out)) == ni.ENOTIMPL
    assert _raw(ni, ctx, 0, 0, None, None, None) == ni.OK                      # empty graph
    assert lib.niorca_set_param(ctx.h, b"no_such_knob", 1) == ni.EINVAL
    assert lib.niorca_set_param(ctx.h, b"tri_wave", 65) == ni.EINVAL
    assert lib.niorca_count_batched(ctx.h, 0, None, 0, None, None, None, None, 0) == ni.OK
    assert lib.niorca_count_batched(ctx.h, 1, None, 0, None, None, None, None, 0) == ni.EINVAL
    assert _raw(ni, ctx, 5, 20, ok(rp), ok(cl), ok(out)) == ni.OK
    torch.cuda.synchronize()
    ctx.close()


def _bad_graphs():
    g = gg.complete(6)
    rp, cl = g.row_ptr.copy(), g.col.copy()
    unsorted = cl.copy()
    unsorted[[0, 1]] = unsorted[[1, 0]]
    loop = cl.copy()
    loop[0] = 0
    dup = cl.copy()
    dup[1] = dup[0]
    asym = gg.from_edges(6, [0, 1, 2], [1, 2, 3])
    acol = asym.col.copy()
    acol[0] = 4  # row 0 now says 0~4, row 4 does not list 0
    oob = cl.copy()
    oob[3] = 99
    return {"unsorted": (rp, unsorted), "self_loop": (rp, loop), "duplicate": (rp, dup),
            "asymmetric": (asym.row_ptr, acol), "out_of_range": (rp, oob)}


@pytest.mark.parametrize("case", sorted(_bad_graphs()))
def test_validate_rejects(ni, case):
    import torch
    rp, cl = _bad_graphs()[case]
    ctx = ni.Context(0)
    out = torch.empty((len(rp) - 1, 15), dtype=torch.int64, device="cuda")
    rc = _raw(ni, ctx, len(rp) - 1, len(cl), ctypes.c_void_p(torch.from_numpy(rp).cuda().data_ptr()),
              ctypes.c_void_p(torch.from_numpy(cl).cuda().data_ptr()), ctypes.c_void_p(out.data_ptr()),
              ni.VALIDATE)
    torch.cuda.synchronize()
    ctx.close()
    assert rc == ni.ENOTSIMPLE


def test_out_of_range_without_validate_is_einval(ni):
    import torch
    rp, cl = _bad_graphs()["out_of_range"]
    with pytest.raises(ni.NiorcaError) as e:
        ni.count(torch.from_numpy(rp).cuda(), torch.from_numpy(cl).cuda())
    assert e.value.status == ni.EINVAL
    torch.cuda.synchronize()


def test_workspace_limit_enomem(ni):
    import torch
    g = gg.config_graph("er_tiny")
    ctx = ni.Context(0)
    ctx.set_workspace_limit(4096)
    with pytest.raises(ni.NiorcaError) as e:
        ni.count(torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col).cuda(), ctx=ctx)
    assert e.value.status == ni.ENOMEM
    ctx.set_workspace_limit(0)
    got = ni.count(torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col).cuda(), ctx=ctx)
    torch.cuda.synchronize()
    assert got.shape == (g.n, 15)
    ctx.close()


def test_degree_overflow_guard(ni):
    """A degree above 1.2 million could overflow the int64 counts (psi_7 = C(d, 3) and
    the f-variable products): the call stops after the degree statistics with
    EOVERFLOW instead of returning wrapped counts."""
    import torch
    g = gg.star(1_200_001)
    ctx = ni.Context(0)
    with pytest.raises(ni.NiorcaError) as e:
        ni.count(torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col).cuda(), ctx=ctx)
    assert e.value.status == ni.EOVERFLOW
    torch.cuda.synchronize()
    ctx.close()


def test_oriented_degree_limit_enotimpl(ni):
    """|N+(v)| above 16384 (the largest row the orientation pass sorts in LDS) is
    refused with ENOTIMPL after the degree statistics, before any counting kernel:
    K_16386 is the smallest simple graph that reaches it (its lowest-ranked vertex
    has 16385 neighbours above it)."""
    import torch
    n = 16386
    # K_n in CSR directly: row x lists every other vertex, ascending
    col = np.broadcast_to(np.arange(n, dtype=np.int32), (n, n))[~np.eye(n, dtype=bool)]
    row_ptr = np.arange(n + 1, dtype=np.int64) * (n - 1)
    ctx = ni.Context(0)
    try:
        with pytest.raises(ni.NiorcaError) as e:
            ni.count(torch.from_numpy(row_ptr).cuda(), torch.from_numpy(np.ascontiguousarray(col)).cuda(), ctx=ctx)
        assert e.value.status == ni.ENOTIMPL
    finally:
        torch.cuda.synchronize()
        ctx.close()


def test_tuning_file_and_bin_mode_errors(ni, tmp_path):
    import torch
    ctx = ni.Context(0)
    try:
        path = tmp_path / "t.txt"
        path.write_text("# comment\nmine tri_wave 32\nmine heavy_k 0  # trailing\nother tri_wave 99\n")
        ctx.load_tuning(str(path), "mine")
        with pytest.raises(ni.NiorcaError) as e:
            ctx.load_tuning(str(path), "absent")
        assert e.value.status == ni.EINVAL
        with pytest.raises(ni.NiorcaError) as e:
            ctx.load_tuning(str(path), "other")  # 99 is out of range for tri_wave
        assert e.value.status == ni.EINVAL
        with pytest.raises(ni.NiorcaError):
            ctx.load_tuning(str(tmp_path / "missing.txt"), "mine")
        with pytest.raises(ni.NiorcaError):
            ctx.set_param("bin_mode", 2)  # no cost model loaded
        with pytest.raises(ni.NiorcaError):
            ctx.set_param("bin_mode", 3)
        g = gg.config_graph("er_tiny")
        got = ni.count(torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col).cuda(), ctx=ctx)
        import oracle
        assert np.array_equal(got.cpu().numpy(), oracle.count(g.row_ptr, g.col))
    finally:
        torch.cuda.synchronize()
        ctx.close()
