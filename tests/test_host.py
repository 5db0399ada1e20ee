"""Host-side checks of the C-ABI library (no GPU needed)."""
import ctypes
import re
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "ascc.h"
LIB = ROOT / "paper_2501_10515_amd" / "libascc.so"


def declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ascc_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    assert LIB.exists(), "build first: python -m paper_2501_10515_amd.build"
    lib = ctypes.CDLL(str(LIB))
    names = declared_functions()
    assert "ascc_residual" in names and "ascc_build_ints" in names and "ascc_solve" in names
    assert "ascc_update" in names
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_the_abi():
    import paper_2501_10515_amd as P

    for name in declared_functions():
        if name in ("ascc_ints_free", "ascc_diis_free", "ascc_ints_shape"):
            continue  # owned by the Ints / Diis wrappers
        if name.startswith("ascc_server_"):
            method = {"create": "__init__", "free": "close", "submit_state": "submit"}.get(
                name[len("ascc_server_"):], name[len("ascc_server_"):])
            assert hasattr(P.Server, method), name
            continue
        assert hasattr(P, name), name


def test_argument_errors_are_reported_not_thrown():
    import paper_2501_10515_amd as P

    with pytest.raises(P.AsccError) as e:
        P.ascc_workspace_bytes(0, 5, 5)
    assert e.value.code == P.ASCC_E_SHAPE
    with pytest.raises(P.AsccError) as e:
        P.ascc_workspace_bytes(2, 5, 5, diis_size=0)
    assert e.value.code == P.ASCC_E_ARG
    lib = P.load_library()
    h = ctypes.c_void_p()
    rc = lib.ascc_build_ints(None, None, 1, 2, 3, 4, 0, 0, None, ctypes.byref(h))
    assert rc == P.ASCC_E_ARG and "device pointers" in P.ascc_last_error()
    assert lib.ascc_residual(None, None, None, None, None, None, None) == P.ASCC_E_ARG
    # the 1-CSF entries reject a hole that is not occupied or a particle that is not virtual
    for hole, particle in [(-1, 3), (2, 3), (0, 1), (0, 5)]:  # no = 2, nv = 3
        h = ctypes.c_void_p(1)
        rc = lib.ascc_build_ints_hbar(None, None, 1, 2, 3, 4, 0, 0, hole, particle, 1, None, ctypes.byref(h))
        assert rc == P.ASCC_E_ARG and "orbital index" in P.ascc_last_error() and not h.value
    rc = lib.ascc_build_ints_hbar(None, None, 1, 2, 3, 4, 0, 0, 1, 2, 1, None, ctypes.byref(h))
    assert rc == P.ASCC_E_ARG and "device pointers" in P.ascc_last_error()
    rc = lib.ascc_build_ints_hbar(None, None, 1, 2, 3, 4, 0, 0, 1, 2, 0, None, ctypes.byref(h))
    assert rc == P.ASCC_E_ARG and "s_sign" in P.ascc_last_error()
    opts = P._lib.Opts(1e-8, 0, 0, 10, 8, 1, 0.0, 0.0, 0)
    res = P._lib.TwoAnsatzResult()
    two = (ctypes.c_void_p * 2)(1, 1)
    rc = lib.ascc_two_ansatz(None, None, 1, 2, 3, 4, 0, 0, 1, 2, 1.0, ctypes.byref(opts), two, two, ctypes.byref(res),
                             None)
    assert rc == P.ASCC_E_ARG and "alpha" in P.ascc_last_error()
    assert lib.ascc_initial_guess(None, None, 2, 3, 0, 2, 1.0, -0.5, None) == P.ASCC_E_ARG


def test_workspace_bytes_scale_with_the_shape():
    import paper_2501_10515_amd as P

    a, d = P.ascc_workspace_bytes(20, 180, 600)
    v = 180
    assert a > 8 * v ** 4  # the full (ac|bd) matrix is part of the integral set
    assert d >= 2 * 8 * 8 * (20 * v + 400 * v * v)


@pytest.mark.parametrize("shapes", [["1,1,1,1", "2,3,8,1", "3,5,12,0", "5,20,60,1", "7,45,37,0"],
                                    ["1,1,1,1,1", "2,3,8,1,1", "3,5,12,0,1", "5,20,60,1,1", "7,45,37,0,1"],
                                    ["20,180,600,1", "40,360,1200,1,1", "30,270,900,0,1", "20,180,600,1,1"],
                                    ["2,3,8,1,0,1", "5,20,60,1,1,2", "7,45,37,0,0,2", "20,180,600,1,1,2",
                                     "40,360,1200,1,1,1"]])
def test_every_launch_stays_in_bounds_dry_run(shapes):
    """The full build / residual / update / solve launch sequence, bounds-checked without a GPU."""
    r = subprocess.run([sys.executable, str(ROOT / "tests" / "dry_run_driver.py"), *shapes], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.count("OK ") == len(shapes)
