"""The C-ABI library loads and exports every function include/mr1l.h declares (no GPU
calls), and the Python binding binds each of them."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mr1l.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(mr1l_[a-z0-9_]+)\s*\(", src)
    return sorted(set(n for n in names if not n.endswith("_fn")))


@pytest.fixture(scope="module")
def libpath():
    import paper_2006_13053_amd as m
    if not os.path.exists(m.LIB_PATH):
        from paper_2006_13053_amd import build
        build.build(verbose=False)
    return m.LIB_PATH


def test_header_declares_the_boundary():
    names = declared()
    for must in ("mr1l_sample", "mr1l_fft", "mr1l_hash_count", "mr1l_extract", "mr1l_adjoint",
                 "mr1l_dimincr", "mr1l_plan_create", "mr1l_plan_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol(libpath):
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (mr1l_[a-z0-9_]+)\b", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


def test_binding_binds_every_declared_symbol(libpath):
    import paper_2006_13053_amd as m
    L = m.lib()
    for n in declared():
        assert n in m.SIGNATURES, n
        assert getattr(L, n) is not None
    assert L.mr1l_version() >= 10000


def test_host_validation_errors_without_gpu(libpath):
    """Argument checks that fail before touching a device."""
    import ctypes as C

    import numpy as np

    import paper_2006_13053_amd as m
    L = m.lib()
    h = C.c_void_p()
    M = np.array([15], np.int64)        # not prime
    z = np.array([1, 2], np.int64)
    rc = L.mr1l_plan_create(C.byref(h), 2, 1, 1, M.ctypes.data_as(C.c_void_p), z.ctypes.data_as(C.c_void_p), 2, None)
    assert rc == -2 and b"not prime" in L.mr1l_last_error()
    M = np.array([17], np.int64)
    z = np.array([1, 17], np.int64)     # z outside [0, M)
    rc = L.mr1l_plan_create(C.byref(h), 2, 1, 1, M.ctypes.data_as(C.c_void_p), z.ctypes.data_as(C.c_void_p), 2, None)
    assert rc == -1
    rc = L.mr1l_plan_create(C.byref(h), 0, 1, 1, M.ctypes.data_as(C.c_void_p), z.ctypes.data_as(C.c_void_p), 2, None)
    assert rc == -1
    rc = L.mr1l_plan_create(C.byref(h), 2, 1, 33, M.ctypes.data_as(C.c_void_p), z.ctypes.data_as(C.c_void_p), 2, None)
    assert rc == -1
    assert L.mr1l_num_lattices(13000, 10.33, 0.9) == 7
    assert L.mr1l_num_lattices(4225, 10.33, 0.9) == 5
    assert L.mr1l_num_lattices(0, 10.33, 0.9) == -1


def test_eq42_library_matches_oracle_count():
    import numpy as np

    import oracle
    import paper_2006_13053_amd as m
    rng = np.random.default_rng(0)
    for _ in range(2000):
        nJ = int(rng.integers(1, 10**8))
        delta = float(rng.uniform(0.01, 0.99))
        assert m.mr1l_num_lattices(nJ, 10.33, delta) == oracle.num_lattices_eq42(nJ, 10.33, delta)
