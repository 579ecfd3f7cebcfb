"""The C-ABI from plain C: tests/c_abi/solve_demo (gcc, C11, no Python) solves
a 48-tet P2 FP64 problem through the host-pointer and the device-pointer
calls, requires both to agree bit for bit, and writes mesh, inputs and the
filtered fields, which must match the FP64 oracle's CMCG solution.
tests/c_abi/solve_demo2d does the same for the 2-D transverse-magnetic PEC
cavity with j = 1 (Section 6) on a 3 x 3 Cartesian mesh, P2."""
import math
import os
import subprocess

import numpy as np
import pytest

from oracle import cmcg as ocmcg
from oracle import dg, dg2d
from paper_2106_02858_amd import inputs
from tests._pairs import rel_norm_c

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(__file__), "c_abi", "solve_demo")
EXE2D = os.path.join(os.path.dirname(__file__), "c_abi", "solve_demo2d")


def test_c_program_solves_like_the_oracle(tmp_path):
    if not os.path.exists(EXE):
        pytest.fail("tests/c_abi/solve_demo is missing: build the library first")
    out = tmp_path / "demo.bin"
    r = subprocess.run([EXE, str(out)], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr
    raw = out.read_bytes()
    nv, K, Np = np.frombuffer(raw[:24], dtype=np.int64)
    off = 24
    xyz = np.frombuffer(raw, np.float64, 3 * nv, off).reshape(nv, 3); off += 24 * nv
    tet = np.frombuffer(raw, np.int64, 4 * K, off).reshape(K, 4); off += 32 * K
    eps = np.frombuffer(raw, np.float64, K, off); off += 8 * K
    j = np.frombuffer(raw, np.float64, K * Np * 3, off).reshape(K, Np, 3); off += 24 * K * Np
    f = np.frombuffer(raw, np.float64, 4 * K * Np * 3, off).reshape(4, K, Np, 3)
    e = f[0] + 1j * f[1]
    h = f[2] + 1j * f[3]
    got = np.concatenate([np.transpose(e, (0, 2, 1)), np.transpose(h, (0, 2, 1))], axis=1)
    tags = np.full((K, 4), 2, dtype=np.int8)
    op = dg.make_problem(xyz, tet, tags, 2, eps, np.ones(K), omega=2 * np.pi, j=j)
    ref = ocmcg.solve(op, tol=1e-10, max_iter=500)
    err = rel_norm_c(op, got, ref.F)
    print(f"C program vs oracle: rel err {err:.2e}")
    assert err < 1e-8


def test_c_program_solves_the_2d_cavity_like_the_oracle(tmp_path):
    if not os.path.exists(EXE2D):
        pytest.fail("tests/c_abi/solve_demo2d is missing: build the library first")
    out = tmp_path / "demo2d.bin"
    r = subprocess.run([EXE2D, str(out)], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stderr
    raw = out.read_bytes()
    nv, K, Np = np.frombuffer(raw[:24], dtype=np.int64)
    off = 24
    xy = np.frombuffer(raw, np.float64, 2 * nv, off).reshape(nv, 2); off += 16 * nv
    tri = np.frombuffer(raw, np.int64, 3 * K, off).reshape(K, 3); off += 24 * K
    tags = np.frombuffer(raw, np.int8, 3 * K, off).reshape(K, 3); off += 3 * K
    eps = np.frombuffer(raw, np.float64, K, off); off += 8 * K
    f = np.frombuffer(raw, np.float64, 6 * K * Np, off)
    e = f[:K * Np] + 1j * f[K * Np:2 * K * Np]
    h = f[2 * K * Np:4 * K * Np] + 1j * f[4 * K * Np:]
    # the C program's mesh is the Cartesian recipe of the 2-D workloads
    cxy, ctri, ctags = inputs.cartesian_triangles(3, 3, side_tags=(inputs.TAG_PEC,) * 4)
    assert np.array_equal(xy, cxy) and np.array_equal(tri, ctri) and np.array_equal(tags, ctags)
    got = np.concatenate([e.reshape(K, 1, Np), np.transpose(h.reshape(K, Np, 2), (0, 2, 1))], axis=1)
    op = dg2d.make_problem(xy, tri, tags, 2, eps, np.ones(K), omega=2 * math.pi, j=np.ones((K, Np)))
    ref = ocmcg.solve(op, tol=1e-10, max_iter=500)
    d = got - ref.F
    err = math.sqrt(sum(abs(dg2d.inner(op, x, x)) for x in (d.real, d.imag))
                    / sum(abs(dg2d.inner(op, x, x)) for x in (ref.F.real, ref.F.imag)))
    print(f"2-D C program vs oracle: rel err {err:.2e}")
    assert err < 1e-8
