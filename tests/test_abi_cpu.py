"""CPU checks of the C ABI library: it loads, and it exports every function that
include/niorca.h declares (no compute call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "niorca.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(niorca_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_2606_29651_amd as ni
    if not os.path.exists(ni.LIB_PATH):
        from paper_2606_29651_amd import build
        build.build()
    return ctypes.CDLL(ni.LIB_PATH)


def test_header_declares_expected_set():
    import paper_2606_29651_amd as ni
    assert declared_functions() == sorted(ni.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_binding_refuses_host_tensors():
    import torch
    import paper_2606_29651_amd as ni
    with pytest.raises((ValueError, TypeError)):
        ni.count(torch.zeros(3, dtype=torch.int64), torch.zeros(0, dtype=torch.int32))


def test_tuning_file_roundtrip(tmp_path):
    """The autotuner's file is the text the library reads (key name value lines)."""
    from paper_2606_29651_amd import autotune
    p = str(tmp_path / "t.txt")
    autotune.save(p, "a", {"tri_wave": 32, "heavy_k": 0}, note="first")
    autotune.save(p, "b", {"qh_wave": 256})
    autotune.save(p, "a", {"tri_wave": 64})
    assert autotune.load(p, "a") == {"tri_wave": 64}
    assert autotune.load(p, "b") == {"qh_wave": 256}
    assert autotune.load(p, "c") is None
    lines = [ln.split("#")[0].split() for ln in open(p) if ln.split("#")[0].strip()]
    assert all(len(x) == 3 and x[2].lstrip("-").isdigit() for x in lines)


def test_committed_tuning_file_parses():
    from paper_2606_29651_amd import autotune
    path = os.path.join(ROOT, "paper_2606_29651_amd", "tuning.txt")
    got = autotune.load(path, "batch_mix")
    assert got and set(got) <= set(autotune.DEFAULTS)


def test_documented_class_bounds_match_the_kernels():
    """The header's ranges for the Stage I class knobs and the autotuner's defaults
    are the class capacities the kernels are compiled for."""
    caps = dict(re.findall(r"#define (TRI_WAVE_CAP|TRI_BLOCK_CAP) (\d+)",
                           open(os.path.join(ROOT, "paper_2606_29651_amd", "csrc", "kernels.hpp")).read()))
    doc = dict(re.findall(r'"(tri_wave|tri_block)"\s+1\.\.(\d+)', open(HEADER).read()))
    assert doc == {"tri_wave": caps["TRI_WAVE_CAP"], "tri_block": caps["TRI_BLOCK_CAP"]}
    from paper_2606_29651_amd.autotune import DEFAULTS
    assert DEFAULTS["tri_wave"] == int(caps["TRI_WAVE_CAP"])
    assert DEFAULTS["tri_block"] == int(caps["TRI_BLOCK_CAP"])
