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


def test_read_probe_rejects_bad_arguments_before_any_device_call():
    """The read-bandwidth probe validates its arguments on the host: a null
    buffer, a size that is zero or not a multiple of 16, a misaligned buffer or
    no repetitions return CA_EINVAL without touching the device."""
    import paper_2512_13133_amd as ca
    lib = ca.load()
    ms = ctypes.c_double(-1.0)
    aligned = 1 << 20  # never dereferenced: every call below fails validation first
    cases = [(None, 1024, 1), (aligned, 0, 1), (aligned, 1000, 1), (aligned + 8, 1024, 1), (aligned, 1024, 0)]
    for buf, size, reps in cases:
        st = lib.ca_probe_read_bandwidth(None, buf, size, reps, ctypes.byref(ms))
        assert st == ca.CA_EINVAL, (buf, size, reps)
    assert ms.value == -1.0
    assert lib.ca_probe_read_bandwidth(None, aligned, 1024, 1, None) == ca.CA_EINVAL
