"""Host-side checks (CPU only): the tiler's index structures and the resident
LDS placement under AddressSanitizer / UBSan, and that the C-ABI library loads and exports every
symbol the header declares and rejects bad inputs before touching a GPU."""
from __future__ import annotations

import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BIN = os.path.join(ROOT, "tests", "_tiling_check")


@pytest.fixture(scope="module")
def checker():
    src = [os.path.join(ROOT, "tests", "tiling_check.cpp"),
           os.path.join(ROOT, "paper_1909_03355_amd", "csrc", "fed_tiling.cpp"),
           os.path.join(ROOT, "paper_1909_03355_amd", "csrc", "fed_lds_order.cpp")]
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all"] + src + ["-o", BIN]
    subprocess.run(cmd, check=True)
    yield BIN
    os.remove(BIN)


@pytest.mark.parametrize("args", [
    ("hex", 5, 6, 7, 1000), ("hex", 5, 6, 7, 37), ("hex", 9, 9, 9, 64), ("hex", 1, 1, 1, 1),
    ("tet", 4, 5, 3, 50), ("tet", 6, 6, 6, 400), ("tet", 2, 2, 2, 3),
    ("hex", 4, 3, 5, 30, 5), ("tet", 3, 3, 3, 40, 4),
    ("hex", 6, 7, 5, 40, 1, 2), ("hex", 9, 9, 9, 200, 1, 3), ("tet", 5, 4, 6, 60, 1, 2),
    ("hex", 4, 3, 5, 30, 3, 2), ("tet", 4, 4, 4, 100, 2, 3), ("hex", 3, 3, 3, 500, 1, 4),
])
def test_tiling_invariants(checker, args):
    r = subprocess.run([checker] + [str(a) for a in args], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert r.stdout.startswith("OK")


def test_header_symbols_exported():
    from paper_1909_03355_amd import _lib as L
    lib = L.lib()
    hdr = open(os.path.join(ROOT, "include", "fedfem.h")).read()
    declared = set(re.findall(r"\b(fed_[a-z_]+)\s*\(", hdr))
    assert declared == set(L.SIGNATURES), declared ^ set(L.SIGNATURES)
    for name in declared:
        assert hasattr(lib, name), name


def _expect(prob, code, **kw):
    from paper_1909_03355_amd import FedError, Simulation
    with pytest.raises(FedError) as ei:
        Simulation(prob, **kw)
    assert ei.value.code == code, str(ei.value)


def test_validation_rejects_bad_inputs():
    """All of these fail in host validation, before any HIP call."""
    from paper_1909_03355_amd import _lib as L
    from workloads import mesh as M, problems as P
    p = P.cube_plain(3, 10)
    c = p["conn"].copy()
    c[2, 5] = -1
    _expect(dict(p, conn=c), L.FED_E_ARG)
    _expect(dict(p, T_lo=10.0, T_hi=10.0), L.FED_E_ARG)
    _expect(dict(p, dt=-1.0), L.FED_E_ARG)
    mats = [dict(p["materials"][0], rho=0.0)]
    _expect(dict(p, materials=mats), L.FED_E_ARG)
    mats = [dict(p["materials"][0], c0=-5.0)]
    _expect(dict(p, materials=mats), L.FED_E_ARG)
    _expect(dict(p, elem_kscale=np.full(27, -1.0)), L.FED_E_ARG)
    _expect(dict(p, dir_nodes=np.array([10 ** 6], np.int32), dir_T=np.array([1.0])), L.FED_E_ARG)
    faces, _ = M.box_side_faces(M.box_hex(3, 3, 3))
    q = P.set_faces(dict(p), faces, h=-1.0)
    _expect(q, L.FED_E_ARG)
    q = P.set_faces(dict(p), faces, eps=np.linspace(0.1, 0.5, faces.shape[0]),
                    Ta=np.linspace(0, 10, faces.shape[0]))
    _expect(q, L.FED_E_ARG)          # radiating faces with different Ta at a node
    two = P.batched_hex(2, 2, 3, 5)
    inst = two["node_instance"].copy()
    inst[two["conn"][3, 0]] = 1 - inst[two["conn"][3, 0]]
    _expect(dict(two, node_instance=inst), L.FED_E_ARG)   # element spans instances
    _expect(p, L.FED_E_ARG, block_threads=100)
    # multiplier tables: T must increase, a k table needs s0 = 1, s1 = 0, a c
    # table c1 = 0
    tab = (np.array([0.0, 50.0, 40.0]), np.array([1.0, 2.0, 3.0]))
    _expect(dict(p, k_table=tab), L.FED_E_ARG)
    ok_tab = (np.array([0.0, 50.0]), np.array([1.0, 2.0]))
    mats = [dict(p["materials"][0], s1=0.01)]
    _expect(dict(p, materials=mats, k_table=ok_tab), L.FED_E_ARG)
    mats = [dict(p["materials"][0], c1=0.5)]
    _expect(dict(p, materials=mats, c_table=ok_tab), L.FED_E_ARG)
    _expect(dict(p, c_table=(ok_tab[0], np.array([1.0, -1.0]))), L.FED_E_ARG)
    # the uniform-gradient hexahedron takes no temporal blocking
    _expect(dict(p, hex_gradient="mean"), L.FED_E_ARG, fuse_steps=2)
    # health-check and allocator options
    _expect(p, L.FED_E_ARG, check_margin=-1.0)
    _expect(p, L.FED_E_ARG, energy_tol=-1.0)
    _expect(p, L.FED_E_ARG, check_every=-2)
    _expect(dict(p, hourglass=0.5), L.FED_E_ARG)                      # needs the mean gradient
    _expect(dict(p, hex_gradient="mean", hourglass=-1.0), L.FED_E_ARG)
