"""Host-only checks of the C ABI (no GPU needed): the built library loads,
exports every entry point include/stag.h declares, the binding declares the
same set, and argument validation that precedes any device call works."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stag.h")
LIB = os.path.join(ROOT, "paper_1010_5433_amd", "libstag.so")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(stag_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libstag.so not built (run __graft_entry__.build())")
    from paper_1010_5433_amd._abi import load_library
    return load_library(LIB)


def test_header_declares_the_boundary():
    names = header_functions()
    for required in ("stag_dslash_eo", "stag_normal_op", "stag_multishift_cg"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    raw = ctypes.CDLL(LIB)
    for name in header_functions():
        assert hasattr(raw, name), name


def test_binding_covers_header():
    from paper_1010_5433_amd._abi import SIGNATURES
    assert sorted(SIGNATURES) == header_functions()


def test_stats_struct_matches_header(lib):
    from paper_1010_5433_amd._abi import CgStats, MAX_SHIFTS
    # 4 ints + 1 int array + 3 double arrays + 1 int array + 1 double, naturally aligned
    expect = 4 * 4 + 4 * MAX_SHIFTS + 8 * 3 * MAX_SHIFTS + 4 * MAX_SHIFTS + 8
    assert ctypes.sizeof(CgStats) == expect
    assert "#define STAG_MAX_SHIFTS 64" in open(HEADER).read()


def test_validation_before_device_use(lib):
    h = ctypes.c_void_p()
    for dims in [(3, 4, 4, 4), (4, 4, 4, 0), (4, 4, 5, 4), (1, 2, 2, 2)]:
        rc = lib.stag_lattice_create((ctypes.c_int * 4)(*dims), 1, ctypes.byref(h))
        assert rc == -1, dims
        assert b"even" in lib.stag_last_error()
    assert lib.stag_lattice_create(None, 1, ctypes.byref(h)) == -1
    assert lib.stag_lattice_destroy(None) == 0
    assert lib.stag_half_volume(None) == 0
    assert lib.stag_dslash_eo(None, 0, None, None, 0, None) == -1
    assert lib.stag_multishift_cg(None, 0.1, None, 1, None, None, 1e-10, 10, 0, None, None) == -1
    assert lib.stag_net_create(None) == -1
    assert lib.stag_net_destroy(None) == 0
    assert lib.stag_net_set_params(None, None) == -1
    assert lib.stag_net_get_params(None, None) == -1
    assert lib.stag_net_apply(None, None, None, None, 0, None) == -1
    assert lib.stag_net_grad(None, None, None, None, None, 0, None) == -1
    assert lib.stag_net_train_step(None, None, None, None, 1, 1e-3, 0, None, None) == -1
    assert lib.stag_fcg_solve(None, 0.1, 0.0, None, None, None, 0, 1e-10, 10, None, None) == -1
    assert lib.stag_rational_apply(None, 0.1, 0.0, None, None, 1, None, None, 1e-10, 10, None, None, None) == -1
    assert lib.stag_fermion_force(None, 1, None, None, None, None) == -1
    for rc in (0, 1, 2, -1, -2, -3):
        assert lib.stag_status_string(rc)


def test_no_oracle_in_product_path():
    """The library package never imports, loads or links the oracle."""
    pkg = os.path.join(ROOT, "paper_1010_5433_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liborc" not in text, f
    import subprocess
    out = subprocess.run(["ldd", LIB], capture_output=True, text=True).stdout
    assert "liborc" not in out
