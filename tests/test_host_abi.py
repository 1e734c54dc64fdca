"""CPU-side checks of the C-ABI library: it loads, exports every entry point the
public header declares, and the binding's declarations match the header."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "srmd.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(srmd_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1506_05094_amd import srmd
    if not os.path.exists(srmd.library_path()):
        from paper_1506_05094_amd import build
        build.build()
    return srmd.load()


def test_header_declares_entry_points():
    names = _declared()
    assert "srmd_create" in names and "srmd_step" in names and "srmd_compute_forces" in names
    assert len(names) >= 15


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_1506_05094_amd import srmd
    assert sorted(srmd.EXPORTED) == _declared()
    for name in srmd.EXPORTED:
        assert callable(getattr(srmd, name))


def test_thermo_struct_layout():
    from paper_1506_05094_amd import srmd
    assert ctypes.sizeof(srmd.srmd_thermo) == 9 * 8 + 2 * 8 + 2 * 4
    assert ctypes.sizeof(srmd.srmd_stats) == 3 * 8 + 10 * 4


def test_null_arguments_rejected_without_gpu(lib):
    from paper_1506_05094_amd import srmd
    # argument validation happens before any device call
    h = ctypes.c_void_p()
    st = lib.srmd_create(ctypes.byref(h), 1, 1, None, None, None, None, None, 0, None)
    assert st == srmd.SRMD_EINVAL
    assert b"particles" in lib.srmd_last_error(None)
    assert lib.srmd_set_skin(None, 0.3) == srmd.SRMD_EINVAL
    assert lib.srmd_step(None, 10, 0, None, 0) == srmd.SRMD_EINVAL
    assert lib.srmd_set_persistent(None, -1) == srmd.SRMD_EINVAL
    assert lib.srmd_destroy(None) == srmd.SRMD_OK


def test_package_import_does_not_need_gpu():
    import paper_1506_05094_amd
    assert hasattr(paper_1506_05094_amd, "System")
