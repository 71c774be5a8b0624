"""The C-ABI library loads on the host and exports every symbol the header declares.

No compute call is made (no GPU here); only argument checks that fail before
any device work.
"""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fsmlmc.h")
LIB = os.path.join(ROOT, "paper_2212_04430_amd", "libfsmlmc.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fs_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2212_04430_amd.build import build
        build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    fns = declared_functions()
    for f in ["fs_create", "fs_destroy", "fs_upload_gauge", "fs_apply_dirac", "fs_z4_noise", "fs_displace",
              "fs_bilinear", "fs_solve_shifted", "fs_estimate", "fs_batch_create", "fs_batch_estimate",
              "fs_batch_destroy", "fs_autotune", "fs_time_dslash", "fs_last_error"]:
        assert f in fns


def test_library_exports_every_declared_symbol(lib):
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_2212_04430_amd import _lib as L
    assert set(L.EXPORTED) == set(declared_functions())
    for f in declared_functions():
        assert callable(getattr(L, f))


def test_struct_layouts_match_header():
    """Every struct the binding passes has the size the library was compiled with."""
    import ctypes as C
    from paper_2212_04430_amd import _lib as L
    sizes = L.fs_struct_sizes()
    assert len(sizes) == len(L.STRUCTS)
    for st, n in zip(L.STRUCTS, sizes):
        assert C.sizeof(st) == n, (st.__name__, C.sizeof(st), n)


def test_argument_errors_before_device_work():
    from paper_2212_04430_amd import _lib as L
    with pytest.raises(L.FsError) as e:
        L.fs_create((1, 4, 4, 4))
    assert e.value.code == L.FS_E_ARG
    assert "extent" in L.fs_last_error()
    assert L.fs_version().startswith("fsmlmc")
    # a null context is rejected by every entry point
    rc = L._lib.fs_upload_gauge(None, None, 0)
    assert rc == L.FS_E_ARG
    assert L._lib.fs_set_tuning(None, 1, 4, 256, 2, 0) == L.FS_E_ARG
    assert L._lib.fs_gauge_info(None, None, None) == L.FS_E_ARG


def test_plain_library_has_no_oracle_dependency():
    """The product path never imports the oracle or falls back to the CPU."""
    pkg = os.path.join(ROOT, "paper_2212_04430_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in src.replace("oracle is", ""), f
