"""The C-ABI library loads and exports every function the header declares;
host-only calls behave.  No device work (runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rift_ile.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rift_ile_\w+)\s*\(", txt)))


def test_header_declares_the_entry_points():
    names = declared()
    for n in ("rift_ile_create", "rift_ile_lnL", "rift_ile_marginalize", "rift_ile_backward",
              "rift_ile_sample", "rift_ile_reduce", "rift_ile_adapt", "rift_ile_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2210_07912_amd import ile
    if not os.path.exists(ile.LIB_PATH):
        from paper_2210_07912_amd import build
        build.build()
    L = ctypes.CDLL(ile.LIB_PATH)
    for n in declared():
        assert hasattr(L, n), n
    assert set(declared()) == set(ile.FUNCTIONS)


def test_host_only_calls():
    from paper_2210_07912_amd import ile
    L = ile.lib()
    assert L.rift_ile_abi_version() == 1
    assert L.rift_ile_status_string(0) == b"ok"
    assert L.rift_ile_status_string(-4).startswith(b"pad")
    # create rejects bad descriptors on the host, before touching a device
    h = ctypes.c_void_p()
    assert L.rift_ile_create(ctypes.byref(h), None, None) == -1
    assert b"no points" in L.rift_ile_last_error(None)


def test_binding_refuses_without_device():
    import torch
    from paper_2210_07912_amd import ile
    if torch.cuda.is_available():
        pytest.skip("device present")
    with pytest.raises(RuntimeError):
        ile.RiftILE([{}])
