"""The C-ABI library loads and exports every symbol include/rbicgstab.h declares (no GPU work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rbicgstab.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_boundary():
    names = _declared()
    for fn in ("rbicgstab_setup", "rbicgstab_solve", "recycle_update", "rbicgstab_workspace_bytes",
               "rbicgstab_destroy", "rbicgstab_last_error"):
        assert fn in names


def test_library_exports_every_declared_symbol():
    from paper_1406_2831_amd import rbicgstab as rb
    if not os.path.exists(rb.LIB_PATH):
        pytest.skip("librbicgstab.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(rb.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(rb.EXPORTS) == set(_declared())


def test_workspace_query_is_host_only():
    from paper_1406_2831_amd import rbicgstab as rb
    if not os.path.exists(rb.LIB_PATH):
        pytest.skip("librbicgstab.so not built")
    n, k, s = 262144, 20, 256
    b = rb.rbicgstab_workspace_bytes(n, 7, k, s)
    # at least the recycle blocks, the Lanczos store and two sliced matrices
    assert b > 10 * n * k * 8 + 3 * n * (k + s) * 8 + 2 * n * 7 * 12
    assert rb.rbicgstab_workspace_bytes(0, 7, k, s) == 0
    assert rb.rbicgstab_workspace_bytes(n, 7, 65, s) == 0       # k_max above 64
    assert rb.rbicgstab_workspace_bytes(n, 7, k, 513) == 0      # s_max above 512
