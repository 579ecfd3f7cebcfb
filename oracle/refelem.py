"""Reference P_q tetrahedron for the nodal DG space (Section 5.2, DG
discretisation; the paper's 2-D triangles lifted to 3-D tetrahedra).

Everything here is computed in exact rational arithmetic (``fractions``):

* nodes: equispaced lattice xi = (i, j, k)/q, ordered k slowest, then j,
  then i fastest (the library's documented node order);
* basis for P_q: homogeneous barycentric monomials lambda^a, |a| = q;
* integrals: the Dirichlet moment formula on a simplex of measure |S| in
  dimension d,  int_S lambda^a = |S| d! a! / (|a| + d)!;
* nodal mass, differentiation and lift matrices for a unit-volume element
  with unit-area faces (the affine scalings are applied in the operator).

Local face f is opposite local vertex f; barycentric lambda_0 = 1 - xi1 -
xi2 - xi3, lambda_k = xi_k.
"""
from __future__ import annotations

import itertools
from fractions import Fraction
from functools import lru_cache
from math import factorial

import numpy as np


def np_count(q: int) -> int:
    return (q + 1) * (q + 2) * (q + 3) // 6


def nfp_count(q: int) -> int:
    return (q + 1) * (q + 2) // 2


def lattice(q: int):
    """Integer node labels (i, j, k), k slowest, i fastest."""
    out = []
    for k in range(q + 1):
        for j in range(q + 1 - k):
            for i in range(q + 1 - j - k):
                out.append((i, j, k))
    return out


def bary_of_label(q: int, lab):
    i, j, k = lab
    return (q - i - j - k, i, j, k)


def nodes(q: int) -> np.ndarray:
    """Reference node coordinates xi [Np, 3] (float64)."""
    return np.array(lattice(q), dtype=np.float64) / q


def face_nodes(q: int):
    """For each local face f, the element-node indices with lambda_f = 0, in
    element node order."""
    labs = lattice(q)
    out = []
    for f in range(4):
        out.append([n for n, lab in enumerate(labs) if bary_of_label(q, lab)[f] == 0])
    return out


def _multi_indices(q: int, nvar: int):
    return [a for a in itertools.product(range(q + 1), repeat=nvar) if sum(a) == q]


def _dirichlet(a, dim: int) -> Fraction:
    """int over a unit-measure simplex of prod lambda_i^{a_i} (Dirichlet)."""
    num = factorial(dim)
    for ai in a:
        num *= factorial(ai)
    return Fraction(num, factorial(sum(a) + dim))


def _frac_inv(A):
    """Exact inverse of a square Fraction matrix by Gauss-Jordan."""
    n = len(A)
    M = [list(row) + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(A)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        piv = M[c][c]
        M[c] = [x / piv for x in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [row[n:] for row in M]


def _matmul(A, B):
    return [[sum(A[i][k] * B[k][j] for k in range(len(B))) for j in range(len(B[0]))]
            for i in range(len(A))]


def _transpose(A):
    return [list(r) for r in zip(*A)]


@lru_cache(maxsize=None)
def exact_matrices(q: int):
    """Exact (Fraction) reference matrices for degree q.

    Returns a dict with
      V    [Np][Np]  V[n][a] = lambda^a(node n)
      C    [Np][Np]  nodal basis phi_n = sum_a C[a][n] lambda^a  (C = V^-1)
      M    [Np][Np]  int_T phi_i phi_j, unit-volume element
      D    3 x [Np][Np]  D_k[i][j] = d phi_j / d xi_k at node i
      E    4 x [Np][Np]  int_{F_f} phi_i phi_j, unit-area face f
    """
    labs = lattice(q)
    Np = len(labs)
    A = _multi_indices(q, 4)
    assert len(A) == Np
    pts = [tuple(Fraction(b, q) for b in bary_of_label(q, lab)) for lab in labs]

    def mono(a, lam):
        v = Fraction(1)
        for ai, li in zip(a, lam):
            v *= li ** ai
        return v

    V = [[mono(a, pts[n]) for a in A] for n in range(Np)]
    C = _frac_inv(V)
    # Gram matrix of monomials over the unit-volume tetrahedron
    G = [[_dirichlet(tuple(x + y for x, y in zip(a, b)), 3) for b in A] for a in A]
    M = _matmul(_matmul(_transpose(C), G), C)
    # derivatives: d lambda^a / d xi_k = a_k lambda^(a-e_k) - a_0 lambda^(a-e_0)
    D = []
    for k in (1, 2, 3):
        dV = []
        for n in range(Np):
            row = []
            for a in A:
                val = Fraction(0)
                if a[k] > 0:
                    b = list(a)
                    b[k] -= 1
                    val += a[k] * mono(b, pts[n])
                if a[0] > 0:
                    b = list(a)
                    b[0] -= 1
                    val -= a[0] * mono(b, pts[n])
                row.append(val)
            dV.append(row)
        D.append(_matmul(dV, C))
    # face mass matrices: on face f lambda_f = 0, the other three lambdas are
    # the face's barycentric coordinates
    E = []
    for f in range(4):
        Gf = [[Fraction(0)] * Np for _ in range(Np)]
        for ia, a in enumerate(A):
            if a[f] != 0:
                continue
            for ib, b in enumerate(A):
                if b[f] != 0:
                    continue
                s = tuple(x + y for i, (x, y) in enumerate(zip(a, b)) if i != f)
                Gf[ia][ib] = _dirichlet(s, 2)
        E.append(_matmul(_matmul(_transpose(C), Gf), C))
    return dict(V=V, C=C, M=M, D=D, E=E, A=A)


def _to_np(F):
    return np.array([[float(x) for x in row] for row in F], dtype=np.float64)


@lru_cache(maxsize=None)
def matrices(q: int):
    """Float64 reference matrices.

    Returns dict(M [Np,Np], Minv, D [3,Np,Np], LIFT [Np, 4*Nfp], Ef [4,Nfp,Nfp],
    fmask [4,Nfp]).  LIFT = M^-1 [E_0|E_1|E_2|E_3] restricted to face-node
    columns, unit-volume element and unit-area faces.
    """
    ex = exact_matrices(q)
    fm = face_nodes(q)
    Np = np_count(q)
    Minv_ex = _frac_inv(ex["M"])
    cols = []
    for f in range(4):
        for n in fm[f]:
            cols.append([ex["E"][f][i][n] for i in range(Np)])
    Ecat = _transpose(cols)  # [Np][4 Nfp]
    LIFT = _matmul(Minv_ex, Ecat)
    Ef = np.array([[[float(ex["E"][f][i][j]) for j in fm[f]] for i in fm[f]] for f in range(4)])
    return dict(M=_to_np(ex["M"]), Minv=_to_np(Minv_ex),
                D=np.stack([_to_np(d) for d in ex["D"]]),
                LIFT=_to_np(LIFT), Ef=Ef, fmask=np.array(fm, dtype=np.int64))
