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
