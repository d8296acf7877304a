"""The C-ABI library loads and exports every symbol include/sfm_gm.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "sfm_gm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|const char\s*\*)\s+(sfm_\w+)\s*\(", src,
                                 flags=re.M)))


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ("sfm_create", "sfm_register_images", "sfm_guided_match", "sfm_guided_match_plain",
              "sfm_bruteforce_match", "sfm_strerror", "sfm_server_start", "sfm_server_submit",
              "sfm_server_poll", "sfm_server_stop", "sfm_server_now_ns"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1512_06235_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("library not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(pkg.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(pkg.exported_symbols()) == set(declared_functions())


def test_strerror_without_gpu():
    import paper_1512_06235_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("library not built")
    assert pkg.sfm_strerror(pkg.SFM_EINVAL) == "invalid argument"
    assert pkg.sfm_strerror(12345) == "unknown status"


def test_no_oracle_in_product_path():
    """The product package never imports or loads the oracle."""
    pkg_dir = os.path.join(ROOT, "paper_1512_06235_amd")
    for dirpath, _, files in os.walk(pkg_dir):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower(), f
