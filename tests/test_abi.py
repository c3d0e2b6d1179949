"""The C ABI library loads and exports every entry point include/dsi.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dsi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dsi_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_1701_03891_amd import _lib
    L = _lib.lib()
    names = _declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(_lib.EXPORTS) == names
    assert _lib.dsi_version().startswith("dsi")


def test_error_codes_without_device():
    """Argument checks that run before any device call."""
    from paper_1701_03891_amd import _lib
    L = _lib.lib()
    assert L.dsi_create(None, 0) == _lib.DSI_E_NULL
    assert L.dsi_measure(None, None, None, None, 1, 1, 1, None) == _lib.DSI_E_NULL
    assert L.dsi_recover(None, None, None, None, 1, None) == _lib.DSI_E_NULL
    assert "NULL" in _lib.dsi_last_error()
    z = ctypes.c_size_t()
    assert L.dsi_workspace_size(None, 1, 0, ctypes.byref(z)) == _lib.DSI_E_NULL


def test_oracle_and_library_share_no_code():
    """The oracle's C source and the GPU sources include nothing of each other."""
    csrc = os.path.join(ROOT, "paper_1701_03891_amd", "csrc")
    for f in os.listdir(csrc):
        text = open(os.path.join(csrc, f)).read()
        assert "orc.h" not in text and "oracle" not in text.lower(), f
    orc = open(os.path.join(ROOT, "oracle", "orc.c")).read()
    assert "dsi.h" not in orc and "csrc" not in orc
    for f in ("__init__.py", "_lib.py"):
        text = open(os.path.join(ROOT, "paper_1701_03891_amd", f)).read()
        assert "import oracle" not in text and "from oracle" not in text
