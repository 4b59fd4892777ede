"""The C-ABI library loads and exports every entry point its header declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "clipalign.h")
LIB = os.path.join(ROOT, "paper_2512_13133_amd", "libclipalign.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:ca_status|const char\*)\s+(ca_\w+)\s*\(", text, re.M)))


def test_header_declares_the_calls():
    names = declared()
    for must in ("ca_create", "ca_clips_create", "ca_align_pairs", "ca_prune", "ca_cluster"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libclipalign.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    import paper_2512_13133_amd as ca
    assert sorted(ca.SYMBOLS) == declared()


def test_create_without_gpu_fails_cleanly():
    """With no visible device ca_create returns an error code, not a crash."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    import paper_2512_13133_amd as ca
    lib = ca.load()
    h = ctypes.c_void_p()
    st = lib.ca_create(ctypes.byref(ca._Config(0, 0, 0)), ctypes.byref(h))
    assert st == ca.CA_EDEVICE
    assert b"device" in lib.ca_last_error(None)
