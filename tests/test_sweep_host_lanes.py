"""The 4-cycle sweep kernels of the library, run on host threads (one per lane,
`tests/host_lanes/`) under AddressSanitizer and compared vertex by vertex with a
direct count over the same per-slot wedge runs.

Lanes run in no fixed order between their rendezvous (shuffles, ballots, wave and
workgroup barriers), so a lane that reads LDS another lane rewrites without a
barrier in between, or any access outside an LDS or graph array, fails here on
the CPU: on the GPU such a race shows only as a rare wrong count or fault.  The
kernels' code is taken from the library's source as is; only `__shared__` arrays
become per-workgroup host buffers.  Parity with the oracle is the GPU tests' job.
"""
import os
import re
import shutil
import subprocess
import sys

import numpy as np
import pytest

import graphgen as gg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_29651_amd", "csrc")
HERE = os.path.join(ROOT, "tests", "host_lanes")


def _block(lines, start, end):
    i = next(k for k, l in enumerate(lines) if re.search(start, l))
    j = next(k for k in range(i + 1, len(lines)) if re.search(end, lines[k]))
    return lines[i:j]


def _function(text, signature):
    """The definition containing signature, with its template line if it has one."""
    i = text.index(signature)
    i = text.rfind("\n", 0, i) + 1
    j = text.index("\n}\n", i) + 3
    prev = text.rfind("\n", 0, i - 1) + 1
    if text[prev:i].startswith("template"):
        i = prev
    return text[i:j]


def kernel_source():
    """The library's 4-cycle code with its item and segment helpers, ready for the host build."""
    count = open(os.path.join(CSRC, "count.hip")).read().split("\n")
    common = open(os.path.join(CSRC, "common.hpp")).read()
    out = [_function(common, "void atomic_add_i64(i64 *p, i64 v)"),
           _function(common, "u32 hslot(u32 key, u32 mask)"),
           _function(common, "void wave_run_add(T *dst, int si, int val)")]
    out += _block(count, r"^// An item is worked on by NT threads", r"^// Classification into work lists")
    out += _block(count, r"^// Largest i in \[0, len\) with off\[i\] <= e, for the QK elements", r"^// Probe pass modes")
    defines = [l for l in count if re.match(r"#define QS ", l)]
    out += defines
    out += _block(count, r"^enum \{ Q_LIGHT", r"^// Light largest vertices whose wedges overflow")
    text = "\n".join(out)
    text = re.sub(r"// Wave-wide inclusive maximum.*?\n}\n", "", text, flags=re.S)  # DPP form: the host has its own
    text = text.replace('__builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");', "")
    text = text.replace("__builtin_amdgcn_wave_barrier();", "emu_wsync();")
    text = text.replace("extern __shared__ __align__(16) char s_dyn[];", "char *s_dyn = emu_blk->dyn;")
    text = re.sub(r"__shared__ (\w+) (\w+)\[(.+?)\];",
                  lambda m: f"{m.group(1)} *{m.group(2)} = emu_shared<{m.group(1)}>(__LINE__, {m.group(3)});", text)
    assert "__shared__" not in text and "update_dpp" not in text
    return text + "\n"


@pytest.fixture(scope="module")
def sweep_host(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no g++")
    d = tmp_path_factory.mktemp("host_lanes")
    inc = d / "kernels.inc"
    inc.write_text(kernel_source())
    exe = d / "sweep_host"
    cmd = [cxx, "-std=c++20", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer", "-pthread",
           f"-I{HERE}", f'-DEMU_INC="{inc}"', os.path.join(HERE, "sweep_host.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "barrier" in r.stderr and "No such file" in r.stderr:
        pytest.skip("no C++20 <barrier>")
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


CASES = {
    # light wave and workgroup items, heavy wave and workgroup items
    "planted_heavy300": (lambda: gg.relabel_random(gg.planted_cliques(1500, 0.02, [40, 30, 20], seed=6), seed=3), 300),
    # light wave items, heavy wave, workgroup and dense items (single- and multi-step)
    "rmat10_heavy300": (lambda: gg.rmat(10, 24, seed=5), 300),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_sweep_on_host_lanes(sweep_host, tmp_path, name):
    make, heavy_k = CASES[name]
    g = make()
    path = tmp_path / "g.bin"
    with open(path, "wb") as f:
        np.array([g.n], np.int32).tofile(f)
        np.array([g.nnz], np.int64).tofile(f)
        g.row_ptr.astype(np.int64).tofile(f)
        g.col.astype(np.int32).tofile(f)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([str(sweep_host), str(path), str(heavy_k)], capture_output=True, text=True, timeout=600, env=env)
    sys.stdout.write(r.stdout)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-3000:])
    assert "ok: 0 vertices differ" in r.stdout
