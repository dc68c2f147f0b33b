"""Input generators: the inputs are simple symmetric sorted CSR graphs of the stated
shapes, and seeded generation is reproducible (also across thread counts)."""
import os
import subprocess
import sys

import numpy as np

import graphgen as gg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def assert_simple_csr(g):
    rp, col = g.row_ptr, g.col
    assert rp[0] == 0 and rp[-1] == len(col) and (np.diff(rp) >= 0).all()
    src = np.repeat(np.arange(g.n), np.diff(rp))
    assert (src != col).all()                       # no self-loops
    key = src * g.n + col
    assert (np.diff(key) > 0).all()                 # rows sorted, no duplicates
    rkey = col.astype(np.int64) * g.n + src
    assert np.array_equal(np.sort(rkey), key)       # symmetric


def test_er_fast_is_simple_and_sized():
    g = gg.er_gnm_fast(50000, 12, seed=5)
    assert_simple_csr(g)
    m = 50000 * 12 // 2
    assert m * 0.99 < g.m <= m                       # a few pairs merge or are loops


def test_er_fast_same_for_any_thread_count():
    code = ("import sys; sys.path.insert(0, %r); import graphgen as gg, hashlib; "
            "g = gg.er_gnm_fast(30000, 10, seed=9); "
            "print(hashlib.sha256(g.row_ptr.tobytes() + g.col.tobytes()).hexdigest())") % ROOT
    outs = set()
    for threads in ("1", "4"):
        env = dict(os.environ, OMP_NUM_THREADS=threads)
        outs.add(subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                                check=True).stdout.strip())
    assert len(outs) == 1


def test_chung_lu_and_rmat_small_are_simple():
    assert_simple_csr(gg.chung_lu(20000, 2.2, 10.0, 2000.0, seed=2))
    assert_simple_csr(gg.rmat(12, 16, seed=5))


def test_batch_mix_and_packing():
    graphs = gg.batch_mix(40, 20, 200, seed=3)
    assert len(graphs) == 40
    for g in graphs:
        assert 20 <= g.n <= 200
        assert_simple_csr(g)
    vtx_off, rp, col = gg.pack_batch(graphs)
    assert vtx_off[0] == 0 and vtx_off[-1] == sum(g.n for g in graphs)
    for i, g in enumerate(graphs):
        a, b = vtx_off[i], vtx_off[i + 1]
        assert np.array_equal(rp[a:b + 1] - rp[a], g.row_ptr)
        assert np.array_equal(col[rp[a]:rp[b]], g.col)   # graph-local ids
