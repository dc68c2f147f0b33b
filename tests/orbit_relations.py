"""The linear relation between non-induced and induced orbit counts, derived by
brute force from the nine connected graphlets on 2-4 vertices (test helper)."""
import itertools

import numpy as np

from oracle import brute

# Graphlets of 2-4 vertices with the orbit of each vertex (brute.classify decides).
GRAPHLETS = {
    "edge": (2, [(0, 1)]),
    "path3": (3, [(0, 1), (1, 2)]),
    "triangle": (3, [(0, 1), (1, 2), (0, 2)]),
    "path4": (4, [(0, 1), (1, 2), (2, 3)]),
    "star3": (4, [(0, 1), (0, 2), (0, 3)]),
    "cycle4": (4, [(0, 1), (1, 2), (2, 3), (3, 0)]),
    "paw": (4, [(0, 1), (0, 2), (1, 2), (0, 3)]),
    "diamond": (4, [(0, 1), (0, 2), (1, 2), (1, 3), (2, 3)]),
    "k4": (4, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]),
}


def subgraph_matrix():
    """C[k, j]: for a vertex x in orbit j of graphlet G_j, the number of connected
    spanning edge subsets of G_j in which x is in orbit k.  An induced occurrence of
    G_j on a vertex set S holds exactly these non-induced occurrences on S, so
    psi = C psi' for every vertex of every graph."""
    C = np.zeros((15, 15), dtype=np.int64)
    for k, es in GRAPHLETS.values():
        vs = list(range(k))
        top = brute.classify(vs, es)
        for x in vs:
            j = top[x]
            col = np.zeros(15, dtype=np.int64)
            for r in range(k - 1, len(es) + 1):
                for sub in itertools.combinations(es, r):
                    if {v for e in sub for v in e} != set(vs) or not brute._connected(vs, sub):
                        continue
                    col[brute.classify(vs, sub)[x]] += 1
            if C[:, j].any():
                assert np.array_equal(C[:, j], col)  # every vertex of orbit j agrees
            C[:, j] = col
    return C
