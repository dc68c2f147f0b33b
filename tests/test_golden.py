"""Golden fixtures (tests/golden/): orbit counts fixed by the definitions of
Section 3, checked against the brute-force definition, both formulations of the C
oracle (connected-set enumeration and the paper's three stages), and the
Section 5 / Appendix equations evaluated on Table 1's f-variables."""
import os

import numpy as np
import pytest

import graphgen as gg
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "graphlets_self.txt")


def load_golden(path=GOLDEN):
    graphs, cur = {}, None
    with open(path) as fh:
        for line in fh:
            p = line.split()
            if not p or p[0].startswith("#"):
                continue
            if p[0] == "graph":
                cur = {"n": int(p[2]), "edges": [], "rows": {}}
                graphs[p[1]] = cur
            elif p[0] == "edge":
                cur["edges"].append((int(p[1]), int(p[2])))
            elif p[0] == "row":
                vals = [int(x) for x in p[2:]]
                assert len(vals) == 15, line
                cur["rows"][int(p[1])] = vals
    out = {}
    for name, d in graphs.items():
        e = np.array(d["edges"], dtype=np.int64)
        g = gg.from_edges(d["n"], e[:, 0], e[:, 1], name)
        want = np.array([d["rows"][v] for v in range(d["n"])], dtype=np.int64)
        out[name] = (g, want)
    return out


CASES = load_golden()


def test_golden_file_is_complete():
    # the nine connected graphlets on 2..4 vertices, every vertex listed
    assert sorted(CASES) == sorted(["edge", "path3", "triangle", "path4", "star3", "cycle4", "paw", "diamond",
                                    "clique4"])
    for name, (g, want) in CASES.items():
        assert want.shape == (g.n, 15)
        assert (want[:, 0] == g.degrees()).all(), name


@pytest.mark.parametrize("name", sorted(CASES))
def test_brute_matches_golden(name):
    g, want = CASES[name]
    assert np.array_equal(brute.orbit_counts_csr(g.row_ptr, g.col), want)


@pytest.mark.parametrize("name", sorted(CASES))
def test_c_oracle_matches_golden(oracle_lib, name):
    g, want = CASES[name]
    assert np.array_equal(oracle_lib.count(g.row_ptr, g.col), want)
    assert np.array_equal(oracle_lib.enum_count(g.row_ptr, g.col), want)


@pytest.mark.gpu
@pytest.mark.parametrize("name", sorted(CASES))
def test_gpu_matches_golden(name):
    import torch
    import paper_2606_29651_amd as ni
    g, want = CASES[name]
    got = ni.count(torch.from_numpy(g.row_ptr).cuda(), torch.from_numpy(g.col).cuda(), flags=ni.VALIDATE)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), want)
