"""AddressSanitizer and UndefinedBehaviorSanitizer runs on the CPU:

  * the oracle (plain C) built with gcc -fsanitize=address,undefined and
    driven through its Python binding on small lattices (operator, tables,
    multi-shift solve, true residual, fermion force, network);
  * the host code of the HIP library (argument validation, Zolotarev and
    Remez coefficients, status strings) built with the sanitizers on the
    host side only, driven through the C ABI in a process without a GPU.

Each run happens in a child process that preloads the sanitizer runtime; a
report of either sanitizer fails the test.  (The library's device code and
the host code that needs a device -- work-arena carving, launches -- are not
covered: GPU sanitizers are not available on this hardware.)
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _run_child(script, lib, preload, tmp_path):
    path = tmp_path / "child.py"
    path.write_text(script)
    env = dict(os.environ, LD_PRELOAD=preload, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, str(path), lib], env=env, capture_output=True, text=True, timeout=600)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report[-4000:]
    for marker in ("AddressSanitizer", "runtime error", "UndefinedBehaviorSanitizer"):
        assert marker not in report, report[-4000:]
    assert "child ok" in r.stdout


ORACLE_CHILD = r'''
import sys
import numpy as np
import oracle
import stag_synth as syn
o = oracle.load(sys.argv[1])
for dims in [(4, 2, 6, 4), (2, 2, 2, 2)]:
    U = syn.smooth_links(dims, 0.5, 3)
    b = syn.gaussian_source(dims, 4)
    o.dslash_eo(dims, U, 0, b)
    o.dslash_eo(dims, U, 1, b)
    o.normal_op(dims, U, 0.1, 0.2, b)
    o.tables(dims)
    o.tables(dims, antiperiodic_t=False)
    x, rc, info = o.multishift_cg(dims, U, 0.1, [0.0, 0.3, 1.0], b, tol=1e-10)
    assert rc == 0
    assert o.true_residual(dims, U, 0.1, 0.3, b, x[1]) <= 1e-10
    y, rc, _ = o.cg(dims, U, 0.1, 0.3, b, tol=1e-10)
    assert rc == 0
    o.fermion_force(dims, U, [0.5, 1.0, 2.0], x)
    theta = np.random.default_rng(5).standard_normal(o.L.orc_net_nparam())
    o.net_forward(dims, U, theta, b)
    o.net_backward(dims, U, theta, b, b)
print("child ok")
'''


def test_oracle_under_asan_and_ubsan(tmp_path):
    gcc = "gcc"
    libasan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(libasan):
        pytest.skip("gcc has no AddressSanitizer runtime")
    lib = str(tmp_path / "liborc_san.so")
    srcs = [os.path.join(ROOT, "oracle", f) for f in ("orc.c", "orc_net.c")]
    subprocess.run([gcc, "-std=c11", "-O1", "-g", "-fopenmp", "-fPIC", "-shared", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-o", lib] + srcs + ["-lm"],
                   check=True)
    _run_child(ORACLE_CHILD, lib, libasan, tmp_path)


LIBRARY_CHILD = r'''
import ctypes
import sys
from paper_1010_5433_amd._abi import load_library
L = load_library(sys.argv[1])
d = ctypes.c_double
for power in (1, -1):
    for n in (1, 4, 16, 24, 64):
        a0, err = d(), d()
        al, sh = (d * 64)(), (d * 64)()
        assert L.stag_zolotarev(power, 1e-4, 16.0001, n, ctypes.byref(a0), al, sh, ctypes.byref(err)) == 0
for p in (0.25, -0.25, -0.5, 0.5, 0.75):
    for n in (4, 12, 20):
        a0, err = d(), d()
        al, sh = (d * 64)(), (d * 64)()
        rc = L.stag_rational_power(p, 1e-4, 16.0001, n, ctypes.byref(a0), al, sh, ctypes.byref(err))
        assert rc in (0, -1), (p, n, rc)
h = ctypes.c_void_p()
for dims in [(3, 4, 4, 4), (4, 4, 4, 0), (1, 2, 2, 2), (4, 4, 5, 4)]:
    assert L.stag_lattice_create((ctypes.c_int * 4)(*dims), 1, ctypes.byref(h)) == -1
assert L.stag_lattice_create(None, 1, ctypes.byref(h)) == -1
assert L.stag_zolotarev(2, 1e-4, 1.0, 4, None, None, None, None) == -1
assert L.stag_zolotarev(1, 1.0, 0.5, 4, None, None, None, None) == -1
assert L.stag_zolotarev(1, 1e-4, 1.0, 65, None, None, None, None) == -1
assert L.stag_rational_power(0.25, 1e-4, 1.0, 0, None, None, None, None) == -1
null = ctypes.c_void_p()
assert L.stag_dslash_eo(null, 0, null, null, 0, null) == -1
assert L.stag_normal_op(null, 0.1, 0.0, null, null, 0, null) == -1
assert L.stag_normal_op_noalloc(null, 0.1, 0.0, null, null, 0, null) == -1
assert L.stag_multishift_cg(null, 0.1, None, 1, null, None, 1e-10, 10, 0, None, null) == -1
assert L.stag_gauge_action(null, 5.0, None, null) == -1
assert L.stag_md_integrate(null, None, null, 0, None, None, null) == -1
assert L.stag_rhmc_trajectory(null, None, null, 0, None, -1.0, None, null) == -1
for s in (0, 1, 2, -1, -2, -3, 7, -100):
    assert L.stag_status_string(s)
assert L.stag_last_error()
print("child ok")
'''


def test_library_host_code_under_asan_and_ubsan(tmp_path):
    sys.path.insert(0, os.path.join(ROOT, "paper_1010_5433_amd"))
    import build as B
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt or not os.path.exists(B.HIPCC):
        pytest.skip("no hipcc AddressSanitizer runtime")
    import concurrent.futures as cf
    srcs = sorted(glob.glob(os.path.join(B.CSRC, "*.hip")))

    def comp(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        r = subprocess.run([B.HIPCC, "-c", src, "-o", obj] + B.CFLAGS + HOST_SAN, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with cf.ThreadPoolExecutor(min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(comp, srcs))
    lib = str(tmp_path / "libstag_san.so")
    subprocess.run([B.HIPCC, "-shared", "-fPIC", f"--offload-arch={B.ARCH}", "-o", lib] + objs + HOST_SAN + B.LDFLAGS,
                   check=True, capture_output=True)
    _run_child(LIBRARY_CHILD, lib, rt[-1], tmp_path)
