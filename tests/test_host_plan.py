"""Host logic of the planner, on the CPU: the destination tile tables of the
reorders (gathers) of every operation list ((0h,0p), (0h,1p), (0h,2p)) stay
inside the destination, cover no element twice and cover every element except
those an accumulating gather leaves unchanged (all maps zero), for systems
with empty irreps, ragged blocks and active spaces; and the same holds for
the affine tiles, whose every affine term reproduces the term's index map
(offset, row and column stride, sign) element by element.  The planner source is compiled with g++
(it uses no HIP)."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import fsgen

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2004_03682_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("host") / "libplancheck.so")
    subprocess.run([gxx, "-O1", "-std=c++17", "-shared", "-fPIC", "-I" + CSRC, "-o", out,
                    os.path.join(HERE, "host", "plan_tiles_check.cpp"), os.path.join(CSRC, "plan_ccsd.cpp")],
                   check=True)
    lib = ctypes.CDLL(out)
    lib.plan_tiles_check.restype = ctypes.c_int
    return lib


SYSTEMS = [("o8v24", None, 0), ("z4", (6, 14, 4, 0.1, 21), 5), ("z6", (5, 12, 6, 0.1, 4), 4),
           ("ragged-z5", (9, 37, 5, 0.05, 17), 6), ("z4-v40", (8, 40, 4, 0.05, 9), 6), ("o20v120z8", None, 0)]


@pytest.mark.parametrize("spec", SYSTEMS, ids=[s[0] for s in SYSTEMS])
def test_gather_tiles_partition_every_destination(checker, spec):
    name, p, nact = spec
    s = fsgen.workload_system(name) if p is None else fsgen.make_system(*p, nact=nact)
    irr = np.ascontiguousarray(s.irrep, dtype=np.int32)
    eps = np.ascontiguousarray(s.eps, dtype=np.float64)
    act = np.ascontiguousarray(s.active if s.active is not None else [], dtype=np.int32)
    nops = ctypes.c_int()
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    bad = checker.plan_tiles_check(s.nocc, s.nvirt, s.nirrep, ptr(irr), ptr(eps), len(act), ptr(act),
                                   ctypes.byref(nops))
    assert nops.value > 0
    assert bad == 0
