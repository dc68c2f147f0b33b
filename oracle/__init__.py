"""Test infrastructure: the CPU oracle for the 15 non-induced orbit counts.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library
(``paper_2606_29651_amd``) and never imports it.

Contents
  * ``brute``          -- definition-level brute force in pure Python (tiny graphs).
  * ``niorca_ref.c``   -- plain C: the definition by connected-set enumeration
                          (``enum_count``; ``enum_induced`` for the induced
                          counts), the paper's three-stage method
                          (``stage1``/``stage2``/``stage3``/``count``),
                          ``orbits_at`` for selected vertices of large graphs, and
                          whole-graph counts for exact checks at any size
                          (``cycles4_total``, ``k4_total``, ``edge_k4``).
  * ``build()``        -- compiles ``niorca_ref.c`` with gcc into
                          ``oracle/libniorca_ref.so``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "niorca_ref.c")
_LIB = os.path.join(_HERE, "libniorca_ref.so")
_lib = None

F_NAMES = ["f12_14", "f10_13", "f13_14", "f11_13", "f5_8", "f6_9", "f9_12", "f4_8", "f8_12"]


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc -O2 -fopenmp) and return the library path (also
    when the library is older than its source)."""
    global _lib
    if force or not os.path.exists(_LIB) or os.path.getmtime(_SRC) > os.path.getmtime(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
               "-Wno-unused-function", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
        _lib = None
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        lib.oref_enum_count.argtypes = [i32, P, P, P]
        lib.oref_enum_induced.argtypes = [i32, P, P, P]
        lib.oref_cycles4_total.argtypes = [i32, P, P, P]
        lib.oref_k4_total.argtypes = [i32, P, P, P]
        lib.oref_edge_k4.argtypes = [i32, P, P, i64, P, P]
        lib.oref_stage23_at.argtypes = [i32, P, P, P, i32, P, P]
        lib.oref_cycles4_at.argtypes = [i32, P, P, i32, P, P]
        lib.oref_stage1.argtypes = [i32, P, P, P]
        lib.oref_stage2.argtypes = [i32, P, P, P]
        lib.oref_stage3.argtypes = [i32, P, P, P, P, P, P]
        lib.oref_count.argtypes = [i32, P, P, P]
        lib.oref_orbits_at.argtypes = [i32, P, P, i32, P, P, P, P]
        lib.oref_set_threads.argtypes = [ctypes.c_int]
        lib.oref_num_threads.restype = ctypes.c_int
        for name in ("oref_enum_count", "oref_stage1", "oref_stage2", "oref_stage3",
                     "oref_count", "oref_orbits_at", "oref_enum_induced", "oref_cycles4_total",
                     "oref_k4_total", "oref_edge_k4", "oref_stage23_at", "oref_cycles4_at"):
            getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr(row_ptr, col):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    n = rp.shape[0] - 1
    if n < 0 or rp[-1] != cl.shape[0]:
        raise ValueError("malformed CSR")
    return n, rp, cl


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def set_threads(t: int) -> None:
    _load().oref_set_threads(int(t))


def num_threads() -> int:
    return int(_load().oref_num_threads())


def enum_count(row_ptr, col) -> np.ndarray:
    """psi int64[n, 15] by enumerating every connected vertex set (the definition)."""
    n, rp, cl = _csr(row_ptr, col)
    psi = np.zeros((max(n, 0), 15), dtype=np.int64)
    _check(_load().oref_enum_count(n, _ptr(rp), _ptr(cl), _ptr(psi)), "enum_count")
    return psi


def enum_induced(row_ptr, col) -> np.ndarray:
    """Induced orbit counts psi' int64[n, 15] (each connected vertex set S counted
    once, as the graphlet G[S]: Section 3, Definition 2)."""
    n, rp, cl = _csr(row_ptr, col)
    psi = np.zeros((max(n, 0), 15), dtype=np.int64)
    _check(_load().oref_enum_induced(n, _ptr(rp), _ptr(cl), _ptr(psi)), "enum_induced")
    return psi


def cycles4_total(row_ptr, col) -> int:
    """Number of 4-cycles of the graph (each once)."""
    n, rp, cl = _csr(row_ptr, col)
    out = np.zeros(1, dtype=np.int64)
    _check(_load().oref_cycles4_total(n, _ptr(rp), _ptr(cl), _ptr(out)), "cycles4_total")
    return int(out[0])


def k4_total(row_ptr, col) -> int:
    """Number of 4-cliques of the graph (each once)."""
    n, rp, cl = _csr(row_ptr, col)
    out = np.zeros(1, dtype=np.int64)
    _check(_load().oref_k4_total(n, _ptr(rp), _ptr(cl), _ptr(out)), "k4_total")
    return int(out[0])


def edge_k4(row_ptr, col, slots=None) -> np.ndarray:
    """4-cliques through the edge of each CSR slot: int64[nnz], or int64[len(slots)]
    for the listed slots."""
    n, rp, cl = _csr(row_ptr, col)
    if slots is None:
        out = np.zeros(cl.shape[0], dtype=np.int64)
        _check(_load().oref_edge_k4(n, _ptr(rp), _ptr(cl), 0, None, _ptr(out)), "edge_k4")
        return out
    sl = np.ascontiguousarray(slots, dtype=np.int64)
    out = np.zeros(sl.shape[0], dtype=np.int64)
    _check(_load().oref_edge_k4(n, _ptr(rp), _ptr(cl), sl.shape[0], _ptr(sl), _ptr(out)), "edge_k4")
    return out


def stage1(row_ptr, col) -> np.ndarray:
    """Per-CSR-slot triangle counts t(e), int32[2m] (Algorithm 1)."""
    n, rp, cl = _csr(row_ptr, col)
    tri = np.zeros(cl.shape[0], dtype=np.int32)
    _check(_load().oref_stage1(n, _ptr(rp), _ptr(cl), _ptr(tri)), "stage1")
    return tri


def stage2(row_ptr, col) -> np.ndarray:
    """Per-vertex 4-clique counts, int64[n] (Algorithm 2)."""
    n, rp, cl = _csr(row_ptr, col)
    k4 = np.zeros(n, dtype=np.int64)
    _check(_load().oref_stage2(n, _ptr(rp), _ptr(cl), _ptr(k4)), "stage2")
    return k4


def stage3(row_ptr, col, tri, k4, want_fvars: bool = False):
    """psi int64[n, 15] (and f-variables int64[n, 9]) from Stage I/II results."""
    n, rp, cl = _csr(row_ptr, col)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    k4 = np.ascontiguousarray(k4, dtype=np.int64)
    psi = np.zeros((n, 15), dtype=np.int64)
    fv = np.zeros((n, 9), dtype=np.int64) if want_fvars else None
    _check(_load().oref_stage3(n, _ptr(rp), _ptr(cl), _ptr(tri), _ptr(k4), _ptr(psi),
                               _ptr(fv) if fv is not None else None), "stage3")
    return (psi, fv) if want_fvars else psi


def count(row_ptr, col) -> np.ndarray:
    """psi int64[n, 15] by the paper's three stages."""
    n, rp, cl = _csr(row_ptr, col)
    psi = np.zeros((n, 15), dtype=np.int64)
    _check(_load().oref_count(n, _ptr(rp), _ptr(cl), _ptr(psi)), "count")
    return psi


def count_with_intermediates(row_ptr, col):
    """(psi, tri, k4, fvars) of the paper's three stages."""
    tri = stage1(row_ptr, col)
    k4 = stage2(row_ptr, col)
    psi, fv = stage3(row_ptr, col, tri, k4, want_fvars=True)
    return psi, tri, k4, fv


def cycles4_at(row_ptr, col, xs) -> np.ndarray:
    """psi_8 (4-cycles through x) of selected vertices, int64[len(xs)], from the
    definition: pairs of common neighbours with every vertex opposite x."""
    n, rp, cl = _csr(row_ptr, col)
    xs = np.ascontiguousarray(xs, dtype=np.int32)
    out = np.zeros(xs.shape[0], dtype=np.int64)
    _check(_load().oref_cycles4_at(n, _ptr(rp), _ptr(cl), xs.shape[0], _ptr(xs), _ptr(out)), "cycles4_at")
    return out


def stage23_at(row_ptr, col, tri, xs) -> np.ndarray:
    """psi int64[len(xs), 15] of selected vertices from the whole graph's Stage I
    counts tri (stage1): Stage II and Stage III for those vertices only."""
    n, rp, cl = _csr(row_ptr, col)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    xs = np.ascontiguousarray(xs, dtype=np.int32)
    psi = np.zeros((xs.shape[0], 15), dtype=np.int64)
    _check(_load().oref_stage23_at(n, _ptr(rp), _ptr(cl), _ptr(tri), xs.shape[0], _ptr(xs), _ptr(psi)),
           "stage23_at")
    return psi


def orbits_at(row_ptr, col, xs, want_fvars: bool = False):
    """psi int64[len(xs), 15] for selected vertices of a (possibly large) graph."""
    n, rp, cl = _csr(row_ptr, col)
    xs = np.ascontiguousarray(xs, dtype=np.int32)
    psi = np.zeros((xs.shape[0], 15), dtype=np.int64)
    fv = np.zeros((xs.shape[0], 9), dtype=np.int64) if want_fvars else None
    scratch = np.zeros(max(cl.shape[0], 1), dtype=np.int32)
    _check(_load().oref_orbits_at(n, _ptr(rp), _ptr(cl), xs.shape[0], _ptr(xs), _ptr(psi),
                                  _ptr(fv) if fv is not None else None, _ptr(scratch)),
           "orbits_at")
    return (psi, fv) if want_fvars else psi
