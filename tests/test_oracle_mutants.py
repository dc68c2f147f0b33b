"""Planted mistakes: each mutant is a copy of the oracle's C source with one
plausible slip (a dropped term, a wrong sign, a transposed operand, a misread
passage), built on the CPU into a temporary library.  The pins must reject every
mutant, which shows they can see such slips in the real oracle."""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

import graphgen as gg
from oracle import brute

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "niorca_ref.c")

MUTANTS = {
    # f6_9 with the triangles on e_yz excluded instead of those on e_xy
    "f6_on_e_yz": [("fv[F6_9] += dy - 2 - txy;", "fv[F6_9] += dy - 2 - tyz;")],
    "f12_dropped_minus_one": [("fv[F12_14] += tyz - 1;", "fv[F12_14] += tyz;")],
    "f10_sign": [("(dz - 1 - tyz);\n", "(dz - 1 + tyz);\n")],
    "f13_transposed": [("(txy - 1) + (txz - 1)", "(txy - 1) + (txy - 1)")],
    "f5_transposed": [("(dz - 1 - txz);", "(dz - 1 - txy);")],
    "f9_wrong_edge": [("fv[F9_12] += tyz;", "fv[F9_12] += txy;")],
    "f4_wrong_vertex": [("fv[F4_8] += dz - 1 - tyz;", "fv[F4_8] += dy - 1 - tyz;")],
    "f8_common_not_minus_one": [("fv[F8_12] += sc->common[z] - 1;", "fv[F8_12] += sc->common[z];")],
    "psi4_single_f12": [("psi[4] = 2 * fv[F12_14]", "psi[4] = fv[F12_14]")],
    "psi9_no_half": [("psi[9] = fv[F12_14] + h9 / 2;", "psi[9] = fv[F12_14] + h9;")],
    "psi6_plus_f13": [("i64 h8 = fv[F13_14] + fv[F8_12], h6 = fv[F6_9] - fv[F13_14];",
                       "i64 h8 = fv[F13_14] + fv[F8_12], h6 = fv[F6_9] + fv[F13_14];")],
    "stage1_merge_skips": [("else { c++; i++; j++; }", "else { c++; i += 2; j++; }")],
    # Stage II: triangles inside N(x) found from both orders of their last two
    # vertices, or without checking that the third vertex closes the triangle
    "k4_third_vertex_unordered": [("if (c > b && inx[c] && ina[c]) cliques++;",
                                   "if (c != a && inx[c] && ina[c]) cliques++;")],
    "k4_third_vertex_not_adjacent": [("if (c > b && inx[c] && ina[c]) cliques++;",
                                      "if (c > b && inx[c]) cliques++;")],
    # paths x - y - z that run back to x
    "paths_return_to_x": [("if (z == x || sc->tx[z] >= 0) continue;", "if (sc->tx[z] >= 0) continue;", -1)],
    # paths whose far end is a neighbour of x (the second, summing pass only)
    "paths_keep_neighbours": [("if (z == x || sc->tx[z] >= 0) continue;\n            i64 dz",
                               "if (z == x) continue;\n            i64 dz")],
    "enum_misses_exclusive_rule": [("if (adjacent_to_set(rp, col, S, k, u)) continue;", "")],
}


def _build_mutant(name, edits, tmpdir):
    src = open(SRC).read()
    for edit in edits:
        old, new = edit[0], edit[1]
        times = edit[2] if len(edit) > 2 else 1
        assert src.count(old) >= 1, (name, old)
        src = src.replace(old, new, times)
    cpath = os.path.join(tmpdir, f"{name}.c")
    so = os.path.join(tmpdir, f"{name}.so")
    with open(cpath, "w") as f:
        f.write(src)
    subprocess.run(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-w", "-o", so, cpath],
                   check=True)
    lib = ctypes.CDLL(so)
    P = ctypes.c_void_p
    lib.oref_count.argtypes = [ctypes.c_int32, P, P, P]
    lib.oref_enum_count.argtypes = [ctypes.c_int32, P, P, P]
    return lib


def _run(fn, g):
    psi = np.zeros((g.n, 15), np.int64)
    rc = fn(g.n, g.row_ptr.ctypes.data_as(ctypes.c_void_p), g.col.ctypes.data_as(ctypes.c_void_p),
            psi.ctypes.data_as(ctypes.c_void_p))
    return rc, psi


def _pin_graphs():
    rng = np.random.default_rng(123)
    out = [gg.complete(5), gg.cycle(4), gg.path(5), gg.star(4),
           gg.from_edges(4, [0, 0, 1, 0], [1, 2, 2, 3]),
           gg.from_edges(4, [0, 0, 1, 1, 2], [1, 2, 2, 3, 3])]
    for _ in range(150):
        n = int(rng.integers(4, 10))
        out.append(gg.er_gnp(n, float(rng.choice([0.3, 0.5, 0.7, 0.9])), int(rng.integers(0, 2**31 - 1))))
    return out


@pytest.fixture(scope="module")
def pin_cases():
    return [(g, brute.orbit_counts_csr(g.row_ptr, g.col)) for g in _pin_graphs()]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name, pin_cases):
    with tempfile.TemporaryDirectory() as td:
        lib = _build_mutant(name, MUTANTS[name], td)
        fn = lib.oref_enum_count if name.startswith("enum_") else lib.oref_count
        caught = False
        for g, ref in pin_cases:
            rc, psi = _run(fn, g)
            if rc != 0 or not np.array_equal(psi, ref):
                caught = True
                break
        assert caught, f"mutant {name} survived the pins"


def test_unmutated_source_passes_same_pins(pin_cases):
    with tempfile.TemporaryDirectory() as td:
        lib = _build_mutant("clean", [], td)
        for g, ref in pin_cases:
            for fn in (lib.oref_count, lib.oref_enum_count):
                rc, psi = _run(fn, g)
                assert rc == 0 and np.array_equal(psi, ref)
