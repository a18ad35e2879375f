"""The C-ABI library loads and exports every function include/im.h declares (CPU only)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "im.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(im_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = _declared()
    for must in ("im_select", "im_initial_gains", "im_snapshot_masks", "im_transpose",
                 "im_workspace_create", "im_workspace_destroy", "im_stats_get", "im_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1212_4779_amd import _native
    lib = ctypes.CDLL(_native.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_native.EXPORTS) <= set(_declared())


def test_struct_layout_matches_header():
    from paper_1212_4779_amd import _native
    assert ctypes.sizeof(_native.ImGraph) == 40
    assert ctypes.sizeof(_native.ImStats) == 64 * 8
    assert ctypes.sizeof(_native.ImInstance) == 56
