"""Test infrastructure: brute-force orbit counts straight from the definitions.

Only tests, the smoke check and the bench's CPU-baseline leg may import this module.
It is not part of the product path and shares no code with the HIP library.

What is computed (Section 3, Definitions 3-5, and the orbit counts psi_k(x) of
Section 5): for every vertex subset S with 2 <= |S| <= 4 and every edge subset
E' of the edges of G inside S such that (S, E') is connected, the pair (S, E') is
one non-induced occurrence of a connected graphlet.  The automorphism group of
(S, E') is found by trying every permutation of S; each orbit of that group is a
set of vertices with one role, and every vertex of S gets +1 on its orbit number.

Orbit numbering.  The paper's orbit figure is missing from the text; the numbering
used (and the only one under which the paper's equations hold, which the tests
check) is the standard one for 2-4 vertex graphlets, with the graphlets in the
order edge, 3-path, triangle, 4-path, 3-star, 4-cycle, tailed triangle, diamond,
4-clique and, inside a graphlet, orbits in order of increasing vertex degree in
that graphlet.  The text fixes part of it: orbit 0 is the edge end (psi_0 is the
degree), 1 and 2 the end and middle of a 3-path, 3 the triangle, 7 the centre of
a 3-star, 14 the 4-clique, 9-11 the tailed triangle and 12-13 the diamond.

Pure Python: use it only on graphs with at most ~14 vertices.
"""
from __future__ import annotations

import itertools

import numpy as np

# (number of vertices, number of edges, sorted degree sequence) -> first orbit id.
# Orbits of one graphlet are numbered upward from this base in order of increasing
# degree inside the graphlet.
GRAPHLET_BASE = {
    (2, 1, (1, 1)): 0,              # edge
    (3, 2, (1, 1, 2)): 1,           # 3-path: ends 1, middle 2
    (3, 3, (2, 2, 2)): 3,           # triangle
    (4, 3, (1, 1, 2, 2)): 4,        # 4-path: ends 4, inner 5
    (4, 3, (1, 1, 1, 3)): 6,        # 3-star: leaves 6, centre 7
    (4, 4, (2, 2, 2, 2)): 8,        # 4-cycle
    (4, 4, (1, 2, 2, 3)): 9,        # tailed triangle: tail 9, triangle 10, hub 11
    (4, 5, (2, 2, 3, 3)): 12,       # diamond: 12 (degree 2), 13 (degree 3)
    (4, 6, (3, 3, 3, 3)): 14,       # 4-clique
}

NUM_ORBITS = 15


def _connected(vertices, edges) -> bool:
    vs = list(vertices)
    adj = {v: set() for v in vs}
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    seen = {vs[0]}
    stack = [vs[0]]
    while stack:
        a = stack.pop()
        for b in adj[a]:
            if b not in seen:
                seen.add(b)
                stack.append(b)
    return len(seen) == len(vs)


def automorphism_orbits(vertices, edges):
    """Orbits of Aut(G') for G' = (vertices, edges), by trying every bijection
    (Definitions 4 and 5).  Returns a dict vertex -> frozenset(orbit)."""
    vs = list(vertices)
    es = {frozenset(e) for e in edges}
    orbit = {v: {v} for v in vs}
    for img in itertools.permutations(vs):
        f = dict(zip(vs, img))
        if all(frozenset((f[a], f[b])) in es for a, b in (tuple(e) for e in es)):
            for v in vs:
                orbit[v].add(f[v])
    return {v: frozenset(o) for v, o in orbit.items()}


def classify(vertices, edges):
    """Orbit id of every vertex of a connected graphlet occurrence (S, E')."""
    vs = list(vertices)
    deg = {v: 0 for v in vs}
    for a, b in edges:
        deg[a] += 1
        deg[b] += 1
    key = (len(vs), len(edges), tuple(sorted(deg.values())))
    base = GRAPHLET_BASE[key]
    orbs = automorphism_orbits(vs, edges)
    # The orbits of these nine graphlets are separated by in-graphlet degree: check it
    # from the automorphism group rather than assume it.
    levels = sorted({deg[v] for v in vs})
    for v in vs:
        for w in orbs[v]:
            if deg[w] != deg[v]:
                raise AssertionError("orbit mixes degrees")
    for v in vs:
        same = [w for w in vs if deg[w] == deg[v]]
        if set(same) != set(orbs[v]):
            raise AssertionError("degree class is not one orbit")
    return {v: base + levels.index(deg[v]) for v in vs}


def orbit_counts(n: int, edge_list, induced: bool = False) -> np.ndarray:
    """psi[x, k] for a simple undirected graph given as n and a list of (u, v).
    With induced=True, psi'[x, k]: only the full edge set of G inside S counts
    (Definition 2), so each connected vertex set S is one occurrence."""
    E = set()
    for a, b in edge_list:
        a, b = int(a), int(b)
        if a == b:
            raise ValueError("self-loop")
        E.add((min(a, b), max(a, b)))
    psi = np.zeros((n, NUM_ORBITS), dtype=np.int64)
    for k in (2, 3, 4):
        for S in itertools.combinations(range(n), k):
            inside = [e for e in itertools.combinations(S, 2) if e in E]
            if len(inside) < k - 1:
                continue
            for r in ([len(inside)] if induced else range(k - 1, len(inside) + 1)):
                for sub in itertools.combinations(inside, r):
                    touched = {v for e in sub for v in e}
                    if len(touched) != k or not _connected(S, sub):
                        continue
                    for v, o in classify(S, sub).items():
                        psi[v, o] += 1
    return psi


def orbit_counts_csr(row_ptr, col, induced: bool = False) -> np.ndarray:
    row_ptr = np.asarray(row_ptr)
    col = np.asarray(col)
    n = row_ptr.shape[0] - 1
    edges = []
    for x in range(n):
        for s in range(row_ptr[x], row_ptr[x + 1]):
            y = int(col[s])
            if x < y:
                edges.append((x, y))
    return orbit_counts(n, edges, induced)
