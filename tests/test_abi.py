"""C-ABI surface checks that need no GPU: the library loads and exports every symbol the
header declares; argument errors that the host rejects before touching a device."""
import ctypes
import os
import re

import paper_1608_05138_amd as glt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "glt.h")) as f:
        src = f.read()
    # function declarations: "<type> glt_name(" at the start of a line
    return sorted(set(re.findall(r"^[a-z_]+[a-z_0-9 ]*\*?\s*\b(glt_[a-z_0-9]+)\(", src, re.M)))


def test_header_declares_expected_entry_points():
    assert _declared() == sorted(glt.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = glt.load_library()
    for name in _declared():
        assert hasattr(lib, name), name
        assert ctypes.cast(getattr(lib, name), ctypes.c_void_p).value


def test_version_string():
    assert glt.version().startswith("glt ")


def test_python_slots_match_header():
    with open(os.path.join(ROOT, "include", "glt.h")) as f:
        src = f.read()
    for s, gid in enumerate(glt.EDGE_SLOTS):
        assert re.search(rf"\b{s}\s+H{gid}\b", src), (s, gid)
