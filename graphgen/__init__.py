"""Seeded synthetic graph generators shared by the tests, the bench and the oracle.

This module holds no part of the orbit-counting arithmetic: it only draws random
graphs and packs them as simple, undirected, symmetric CSR adjacency with every
row sorted ascending by vertex id (the precondition of the problem statement,
Section 3, Definitions 1-3: a simple graph G = (V, E)).

Layout of every CSR returned here:
    row_ptr : numpy int64[n + 1], row_ptr[0] = 0, row_ptr[n] = 2m
    col     : numpy int32[2m], col[row_ptr[v]:row_ptr[v+1]] = N(v) sorted ascending
Self-loops are dropped and multi-edges are merged before packing.

Recipes (all take a numpy PCG64 seed):
  * er_gnp(n, p)          exact G(n, p): one independent coin per vertex pair,
                          drawn by geometric skipping over the pair index space.
  * er_gnm(n, avg_deg)    n*avg_deg/2 uniform vertex pairs, self-loops dropped,
                          duplicates merged (G(n, m)-like; the paper's ER series
                          in Section 7 is drawn with an ER generator).
  * chung_lu(n, ...)      expected-degree power law, w_i = min(cap, c (i+1)^(-1/(gamma-1)))
                          with c chosen so that mean(w) equals the target, then
                          n*mean/2 endpoint pairs drawn proportionally to w.
  * rmat(scale, ef, ...)  recursive-matrix generator, 2^scale vertices,
                          ef * 2^scale edge samples.
  * barabasi_albert(n, k) preferential attachment, k edges per new vertex.
  * complete, star, path, cycle and a few hand graphs for the closed-form pins.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass

import numpy as np

__all__ = [
    "CSR", "from_edges", "er_gnp", "er_gnm", "chung_lu", "rmat", "barabasi_albert",
    "complete", "star", "path", "cycle", "empty", "planted_cliques", "relabel_random",
    "disjoint_union", "batch_mix", "pack_batch", "config_graph",
]


@dataclass
class CSR:
    """Symmetric sorted CSR of a simple undirected graph."""

    row_ptr: np.ndarray  # int64[n+1]
    col: np.ndarray      # int32[2m]
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def edges(self) -> np.ndarray:
        """Undirected edges (u < v) as an int64[m, 2] array, sorted by (u, v)."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))
        dst = self.col.astype(np.int64)
        keep = src < dst
        return np.stack([src[keep], dst[keep]], axis=1)

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(self.row_ptr).tobytes())
        h.update(np.ascontiguousarray(self.col).tobytes())
        return h.hexdigest()


def from_edges(n: int, u: np.ndarray, v: np.ndarray, name: str = "") -> CSR:
    """Pack an arbitrary edge list into simple symmetric sorted CSR.

    Self-loops are dropped, both directions are added and duplicates merged.
    """
    u = np.asarray(u, dtype=np.int64).ravel()
    v = np.asarray(v, dtype=np.int64).ravel()
    if u.shape != v.shape:
        raise ValueError("edge endpoint arrays differ in length")
    if n < 0:
        raise ValueError("n must be non-negative")
    if u.size and (u.min() < 0 or v.min() < 0 or u.max() >= n or v.max() >= n):
        raise ValueError("edge endpoint out of range")
    if n >= 2**31:
        raise ValueError("vertex ids must fit int32")
    keep = u != v
    u, v = u[keep], v[keep]
    # One key per directed slot; unique() sorts by (row, col) and merges duplicates.
    keys = np.concatenate([u * n + v, v * n + u])
    keys = np.unique(keys)
    rows = keys // n if n else keys
    cols = keys - rows * n if n else keys
    counts = np.bincount(rows, minlength=n).astype(np.int64) if n else np.zeros(0, np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return CSR(row_ptr, cols.astype(np.int32), name)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _pair_from_index(k: np.ndarray, n: int):
    """Map a linear index over the strict upper triangle (row-major) to (i, j), i < j."""
    # Row i starts at S(i) = i*n - i*(i+1)/2; invert with the quadratic formula and fix
    # the floating point guess by one step either way.
    k = k.astype(np.int64)
    nf = float(n)
    i = np.floor(((2 * nf - 1) - np.sqrt((2 * nf - 1) ** 2 - 8.0 * k)) / 2).astype(np.int64)
    i = np.clip(i, 0, max(n - 2, 0))
    start = i * n - i * (i + 1) // 2
    over = start > k
    i[over] -= 1
    start = i * n - i * (i + 1) // 2
    nxt = (i + 1) * n - (i + 1) * (i + 2) // 2
    under = nxt <= k
    i[under] += 1
    start = i * n - i * (i + 1) // 2
    j = k - start + i + 1
    return i, j


def er_gnp(n: int, p: float, seed: int = 42) -> CSR:
    """Exact G(n, p): every unordered pair is an edge with probability p independently."""
    rng = _rng(seed)
    total = n * (n - 1) // 2
    if total == 0 or p <= 0.0:
        return from_edges(n, np.zeros(0), np.zeros(0), f"er_gnp({n},{p})")
    if p >= 1.0:
        idx = np.arange(total, dtype=np.int64)
    else:
        # Geometric gaps between successive chosen pair indices.
        chunks = []
        pos = -1
        expect = int(total * p * 1.1) + 64
        while True:
            gaps = rng.geometric(p, size=expect).astype(np.int64)
            cand = pos + np.cumsum(gaps)
            chunks.append(cand[cand < total])
            if cand[-1] >= total:
                break
            pos = int(cand[-1])
        idx = np.concatenate(chunks)
    i, j = _pair_from_index(idx, n)
    return from_edges(n, i, j, f"er_gnp({n},{p})")


def er_gnm(n: int, avg_deg: float, seed: int = 42) -> CSR:
    """n*avg_deg/2 uniformly drawn vertex pairs; self-loops dropped, duplicates merged."""
    rng = _rng(seed)
    m = int(round(n * avg_deg / 2))
    u = rng.integers(0, n, size=m, dtype=np.int64)
    v = rng.integers(0, n, size=m, dtype=np.int64)
    return from_edges(n, u, v, f"er_gnm({n},{avg_deg})")


def chung_lu(n: int, gamma: float = 2.2, mean_deg: float = 20.0, cap: float = 50000.0,
             seed: int = 42, permute: bool = False) -> CSR:
    """Chung-Lu expected-degree graph with a capped power-law weight sequence.

    w_i = min(cap, c (i+1)^(-1/(gamma-1))); c is found by bisection so that the mean
    weight equals mean_deg.  n*mean_deg/2 pairs are drawn with both endpoints chosen
    proportionally to w (inverse-CDF sampling); self-loops and duplicates are removed.
    With permute=True a seeded random relabelling spreads the hubs over the id range.
    """
    rng = _rng(seed)
    expo = -1.0 / (gamma - 1.0)
    base = np.power(np.arange(1, n + 1, dtype=np.float64), expo)

    def mean_w(c):
        return np.minimum(cap, c * base).mean()

    lo, hi = 0.0, 1.0
    while mean_w(hi) < mean_deg:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mean_w(mid) < mean_deg:
            lo = mid
        else:
            hi = mid
    w = np.minimum(cap, hi * base)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    pairs = int(round(n * mean_deg / 2))
    u = np.searchsorted(cdf, rng.random(pairs), side="right")
    v = np.searchsorted(cdf, rng.random(pairs), side="right")
    u = np.minimum(u, n - 1)
    v = np.minimum(v, n - 1)
    if permute:
        perm = rng.permutation(n)
        u, v = perm[u], perm[v]
    return from_edges(n, u, v, f"chung_lu({n},{gamma},{mean_deg},{cap})")


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, seed: int = 42, permute: bool = False) -> CSR:
    """R-MAT graph: edge_factor * 2^scale samples, symmetrised and deduplicated."""
    rng = _rng(seed)
    n = 1 << scale
    m = edge_factor * n
    u = np.zeros(m, dtype=np.int64)
    v = np.zeros(m, dtype=np.int64)
    ab, abc = a + b, a + b + c
    chunk = 1 << 23
    for s in range(0, m, chunk):
        e = min(m, s + chunk)
        uu = np.zeros(e - s, dtype=np.int64)
        vv = np.zeros(e - s, dtype=np.int64)
        for level in range(scale):
            r = rng.random(e - s)
            bit = np.int64(1) << np.int64(scale - 1 - level)
            right = ((r >= a) & (r < ab)) | (r >= abc)
            down = r >= ab
            vv += np.where(right, bit, 0)
            uu += np.where(down, bit, 0)
        u[s:e], v[s:e] = uu, vv
    if permute:
        perm = rng.permutation(n)
        u, v = perm[u], perm[v]
    return from_edges(n, u, v, f"rmat({scale},{edge_factor})")


def barabasi_albert(n: int, k: int, seed: int = 42) -> CSR:
    """Preferential attachment: each new vertex joins k distinct earlier vertices."""
    rng = _rng(seed)
    if n <= k:
        return complete(n)
    src, dst = [], []
    # Seed with a star on k+1 vertices so every early vertex has positive degree.
    targets_pool = []
    for t in range(1, k + 1):
        src.append(0)
        dst.append(t)
        targets_pool += [0, t]
    pool = np.empty(2 * k * n + 8, dtype=np.int64)
    pool[: len(targets_pool)] = targets_pool
    plen = len(targets_pool)
    for new in range(k + 1, n):
        chosen = set()
        while len(chosen) < k:
            chosen.add(int(pool[rng.integers(0, plen)]))
        for t in chosen:
            src.append(new)
            dst.append(t)
            pool[plen] = new
            pool[plen + 1] = t
            plen += 2
    return from_edges(n, np.array(src), np.array(dst), f"ba({n},{k})")


def complete(n: int) -> CSR:
    i, j = np.triu_indices(n, 1)
    return from_edges(n, i, j, f"K{n}")


def star(k: int) -> CSR:
    """Star S_k: centre 0 joined to leaves 1..k."""
    return from_edges(k + 1, np.zeros(k, np.int64), np.arange(1, k + 1), f"S{k}")


def path(n: int) -> CSR:
    return from_edges(n, np.arange(n - 1), np.arange(1, n), f"P{n}")


def cycle(n: int) -> CSR:
    return from_edges(n, np.arange(n), (np.arange(n) + 1) % n, f"C{n}")


def empty(n: int) -> CSR:
    return from_edges(n, np.zeros(0), np.zeros(0), f"empty({n})")


def planted_cliques(n: int, p: float, clique_sizes, seed: int = 42) -> CSR:
    """G(n, p) background plus cliques planted on random disjoint vertex sets."""
    rng = _rng(seed + 1)
    g = er_gnp(n, p, seed)
    e = g.edges()
    us, vs = [e[:, 0]], [e[:, 1]]
    order = rng.permutation(n)
    at = 0
    for s in clique_sizes:
        if at + s > n:
            break
        mem = order[at: at + s]
        at += s
        i, j = np.triu_indices(s, 1)
        us.append(mem[i])
        vs.append(mem[j])
    return from_edges(n, np.concatenate(us), np.concatenate(vs),
                      f"planted({n},{p},{list(clique_sizes)})")


def relabel_random(g: CSR, seed: int = 42) -> CSR:
    rng = _rng(seed)
    perm = rng.permutation(g.n)
    e = g.edges()
    return from_edges(g.n, perm[e[:, 0]], perm[e[:, 1]], g.name + "~perm")


def disjoint_union(graphs) -> CSR:
    us, vs, off = [], [], 0
    for g in graphs:
        e = g.edges()
        us.append(e[:, 0] + off)
        vs.append(e[:, 1] + off)
        off += g.n
    if not us:
        return empty(0)
    return from_edges(off, np.concatenate(us), np.concatenate(vs), "union")


def batch_mix(num_graphs: int, n_lo: int = 20, n_hi: int = 2000, seed: int = 42):
    """Many small graphs of uneven size: even positions Erdos-Renyi (average degree
    uniform in [2, 12]), odd positions Barabasi-Albert (k uniform in 2..8); n uniform
    in [n_lo, n_hi]."""
    rng = _rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, size=num_graphs)
    degs = rng.uniform(2.0, 12.0, size=num_graphs)
    ks = rng.integers(2, 9, size=num_graphs)
    subs = rng.integers(0, 2**31 - 1, size=num_graphs)
    out = [None] * num_graphs
    ba_idx = []
    for gi in range(num_graphs):
        n = int(ns[gi])
        if gi % 2 == 0:
            out[gi] = er_gnp(n, min(1.0, float(degs[gi]) / max(n - 1, 1)), int(subs[gi]))
        else:
            ba_idx.append(gi)
    if ba_idx:
        for gi, g in zip(ba_idx, ba_many(ns[ba_idx], ks[ba_idx], seed + 7)):
            out[gi] = g
    return out


_BA_LIB = None


def _ba_lib():
    """Compile and load graphgen/ba.c (gcc), once."""
    global _BA_LIB
    if _BA_LIB is None:
        import ctypes
        import os
        import subprocess
        here = os.path.dirname(os.path.abspath(__file__))
        so = os.path.join(here, "libba.so")
        src = os.path.join(here, "ba.c")
        if not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
            tmp = so + f".tmp{os.getpid()}"
            subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, src], check=True)
            os.replace(tmp, so)
        lib = ctypes.CDLL(so)
        P = ctypes.c_void_p
        lib.ba_edges.argtypes = [ctypes.c_int64, P, P, ctypes.c_uint64, P, P, P]
        lib.ba_edges.restype = ctypes.c_int
        _BA_LIB = lib
    return _BA_LIB


_ER_LIB = None


def _er_lib():
    """Compile and load graphgen/er.c (gcc, OpenMP), once."""
    global _ER_LIB
    if _ER_LIB is None:
        import ctypes
        import os
        import subprocess
        here = os.path.dirname(os.path.abspath(__file__))
        so = os.path.join(here, "liber.so")
        src = os.path.join(here, "er.c")
        if not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
            tmp = so + f".tmp{os.getpid()}"
            subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src], check=True)
            os.replace(tmp, so)
        lib = ctypes.CDLL(so)
        P = ctypes.c_void_p
        lib.er_gnm_csr.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, P, P]
        lib.er_gnm_csr.restype = ctypes.c_int64
        _ER_LIB = lib
    return _ER_LIB


def er_gnm_fast(n: int, avg_deg: float, seed: int = 42) -> CSR:
    """G(n, m = n*avg_deg/2) built directly as CSR by graphgen/er.c (multithreaded):
    uniform pairs from a counter-based stream, self-loops dropped, duplicates merged.
    Same distribution as er_gnm, a different sample for the same seed."""
    import ctypes
    m = int(round(n * avg_deg / 2))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    col = np.empty(max(2 * m, 1), dtype=np.int32)
    nnz = _er_lib().er_gnm_csr(n, m, ctypes.c_uint64((seed * 0x9E3779B97F4A7C15 + 1) & (2**64 - 1)),
                               row_ptr.ctypes.data_as(ctypes.c_void_p), col.ctypes.data_as(ctypes.c_void_p))
    if nnz < 0:
        raise MemoryError("er_gnm_csr failed")
    return CSR(row_ptr, col[:nnz].copy(), f"er_gnm({n},{avg_deg})")


def ba_many(ns, ks, seed: int):
    """Preferential-attachment graphs (see ba.c), one per (n, k) pair, k <= 16."""
    import ctypes
    ns = np.ascontiguousarray(ns, dtype=np.int64)
    ks = np.ascontiguousarray(np.clip(ks, 1, 16), dtype=np.int64)
    small = ns <= ks
    cap = int((ns * ks)[~small].sum() + (ns * ns)[small].sum() + 1)
    src = np.empty(cap, np.int64)
    dst = np.empty(cap, np.int64)
    eoff = np.zeros(len(ns) + 1, np.int64)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    _ba_lib().ba_edges(len(ns), ptr(ns), ptr(ks), ctypes.c_uint64(seed & (2**64 - 1)), ptr(src), ptr(dst),
                       ptr(eoff))
    out = []
    for j in range(len(ns)):
        a, b = eoff[j], eoff[j + 1]
        out.append(from_edges(int(ns[j]), src[a:b], dst[a:b], f"ba({int(ns[j])},{int(ks[j])})"))
    return out


def _ba_fast(n: int, k: int, seed: int) -> CSR:
    """Vectorised-enough preferential attachment for batch generation.

    Each new vertex picks k targets from the endpoint pool (duplicates collapse, so
    a vertex may get fewer than k edges, which keeps the generator O(n k))."""
    rng = _rng(seed)
    if n <= k + 1:
        return complete(n)
    pool = np.empty(2 * k * n + 2 * k, dtype=np.int64)
    pool[0:2 * k:2] = 0
    pool[1:2 * k:2] = np.arange(1, k + 1)
    plen = 2 * k
    src = [np.zeros(k, np.int64)]
    dst = [np.arange(1, k + 1, dtype=np.int64)]
    r = rng.random((n, k))
    for new in range(k + 1, n):
        t = pool[(r[new] * plen).astype(np.int64)]
        t = np.unique(t)
        src.append(np.full(t.shape[0], new, np.int64))
        dst.append(t)
        cnt = t.shape[0]
        pool[plen: plen + 2 * cnt: 2] = new
        pool[plen + 1: plen + 2 * cnt: 2] = t
        plen += 2 * cnt
    return from_edges(n, np.concatenate(src), np.concatenate(dst), f"ba({n},{k})")


def pack_batch(graphs):
    """Pack graphs into one CSR with per-graph vertex offsets.

    Returns (vtx_off int64[G+1], row_ptr int64[sum n + 1], col int32[...]) where
    column ids are LOCAL to their graph (0..n_g-1) and row_ptr is global.
    """
    G = len(graphs)
    vtx_off = np.zeros(G + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        vtx_off[i + 1] = vtx_off[i] + g.n
    total_n = int(vtx_off[-1])
    row_ptr = np.zeros(total_n + 1, dtype=np.int64)
    cols = []
    base = 0
    for i, g in enumerate(graphs):
        row_ptr[vtx_off[i] + 1: vtx_off[i + 1] + 1] = g.row_ptr[1:] + base
        base += g.nnz
        cols.append(g.col)
    col = np.concatenate(cols) if cols else np.zeros(0, np.int32)
    return vtx_off, row_ptr, col.astype(np.int32)


def config_graph(name: str, seed: int = 42) -> CSR:
    """Named workloads, sized as the paper-shaped synthetic configurations."""
    if name == "er_tiny":
        return er_gnp(2000, 0.005, seed)
    if name == "chung_lu_4m":
        return chung_lu(4_000_000, 2.2, 20.0, 50_000.0, seed)
    if name == "rmat22":
        return rmat(22, 16, 0.57, 0.19, 0.19, seed)
    if name.startswith("batch_"):
        # batch_<count>: packed mix of small ER and BA graphs (use pack_batch)
        raise KeyError("batched workloads are lists of graphs: use batch_mix")
    if name.startswith("er_"):
        # er_<n>_<deg>, e.g. er_1m_8
        _, ns, ds = name.split("_")
        mult = {"k": 1_000, "m": 1_000_000}[ns[-1]]
        return er_gnm_fast(int(ns[:-1]) * mult, float(ds), seed)
    raise KeyError(name)
