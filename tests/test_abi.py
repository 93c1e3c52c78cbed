"""The C-ABI library loads without a GPU and exports every function include/lat.h declares;
the Python binding covers exactly those entry points."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "lat.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lat_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_2603_10741_amd import binding
    lib = ctypes.CDLL(binding.LIB_PATH)
    names = _declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_2603_10741_amd import binding
    assert sorted(binding.exported_symbols()) == _declared()


def test_status_strings():
    from paper_2603_10741_amd import binding
    L = binding._lib()
    for code in range(8):
        assert L.lat_status_string(code)
