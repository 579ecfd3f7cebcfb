"""Reference P_q triangle for the 2-D nodal DG space (Section 5.2.2, DG
discretisation on triangles; the transverse-magnetic setting of Section 5.2.1).

Built like the tetrahedron in ``refelem``, in exact rational arithmetic:

* nodes: equispaced lattice xi = (i, j)/q, j slowest, i fastest;
* basis for P_q: homogeneous barycentric monomials lambda^a, |a| = q;
* integrals: the Dirichlet moment formula on a simplex;
* nodal mass, differentiation and lift matrices for a unit-area element
  with unit-length edges (the affine scalings are applied in the operator).

Local edge f is opposite local vertex f; lambda_0 = 1 - xi1 - xi2,
lambda_k = xi_k.  Edge nodes are listed in element node order.
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache

import numpy as np

from .refelem import _dirichlet, _frac_inv, _matmul, _multi_indices, _transpose


def np_count(q: int) -> int:
    return (q + 1) * (q + 2) // 2


def nfp_count(q: int) -> int:
    return q + 1


def lattice(q: int):
    """Integer node labels (i, j), j slowest, i fastest."""
    return [(i, j) for j in range(q + 1) for i in range(q + 1 - j)]


def bary_of_label(q: int, lab):
    i, j = lab
    return (q - i - j, i, j)


def nodes(q: int) -> np.ndarray:
    """Reference node coordinates xi [Np, 2] (float64)."""
    return np.array(lattice(q), dtype=np.float64) / q


def face_nodes(q: int):
    """For each local edge f, the element-node indices with lambda_f = 0."""
    labs = lattice(q)
    return [[n for n, lab in enumerate(labs) if bary_of_label(q, lab)[f] == 0] for f in range(3)]


def _mono(a, lam):
    v = Fraction(1)
    for ai, li in zip(a, lam):
        v *= li ** ai
    return v


@lru_cache(maxsize=None)
def exact_matrices(q: int):
    """Exact (Fraction) reference matrices for degree q: V, C = V^-1 (nodal
    basis phi_n = sum_a C[a][n] lambda^a), M (unit-area element), D (2 x
    [Np][Np], D_k[i][j] = d phi_j / d xi_k at node i), E (3 x [Np][Np], the
    mass matrix of unit-length edge f)."""
    labs = lattice(q)
    Np = len(labs)
    A = _multi_indices(q, 3)
    assert len(A) == Np
    pts = [tuple(Fraction(b, q) for b in bary_of_label(q, lab)) for lab in labs]
    V = [[_mono(a, pts[n]) for a in A] for n in range(Np)]
    C = _frac_inv(V)
    G = [[_dirichlet(tuple(x + y for x, y in zip(a, b)), 2) for b in A] for a in A]
    M = _matmul(_matmul(_transpose(C), G), C)
    D = []
    for k in (1, 2):
        dV = []
        for n in range(Np):
            row = []
            for a in A:
                val = Fraction(0)
                if a[k] > 0:
                    b = list(a)
                    b[k] -= 1
                    val += a[k] * _mono(b, pts[n])
                if a[0] > 0:
                    b = list(a)
                    b[0] -= 1
                    val -= a[0] * _mono(b, pts[n])
                row.append(val)
            dV.append(row)
        D.append(_matmul(dV, C))
    E = []
    for f in range(3):
        Gf = [[Fraction(0)] * Np for _ in range(Np)]
        for ia, a in enumerate(A):
            if a[f] != 0:
                continue
            for ib, b in enumerate(A):
                if b[f] != 0:
                    continue
                s = tuple(x + y for i, (x, y) in enumerate(zip(a, b)) if i != f)
                Gf[ia][ib] = _dirichlet(s, 1)
        E.append(_matmul(_matmul(_transpose(C), Gf), C))
    return dict(V=V, C=C, M=M, D=D, E=E, A=A)


def _to_np(F):
    return np.array([[float(x) for x in row] for row in F], dtype=np.float64)


@lru_cache(maxsize=None)
def matrices(q: int):
    """Float64 reference matrices: M, Minv, D [2,Np,Np], LIFT [Np, 3*Nfp]
    (M^-1 times the edge mass columns of the edge nodes), fmask [3,Nfp]."""
    ex = exact_matrices(q)
    fm = face_nodes(q)
    Np = np_count(q)
    Minv_ex = _frac_inv(ex["M"])
    cols = [[ex["E"][f][i][n] for i in range(Np)] for f in range(3) for n in fm[f]]
    LIFT = _matmul(Minv_ex, _transpose(cols))
    return dict(M=_to_np(ex["M"]), Minv=_to_np(Minv_ex), D=np.stack([_to_np(d) for d in ex["D"]]),
                LIFT=_to_np(LIFT), fmask=np.array(fm, dtype=np.int64))


def basis_at(q: int, xi: np.ndarray) -> np.ndarray:
    """Values of the nodal basis at reference points xi [P, 2]: [P, Np]."""
    ex = exact_matrices(q)
    C = _to_np(ex["C"])
    lam = np.stack([1.0 - xi[:, 0] - xi[:, 1], xi[:, 0], xi[:, 1]], axis=1)
    mono = np.stack([np.prod(lam ** np.array(a, dtype=np.float64), axis=1) for a in ex["A"]], axis=1)
    return mono @ C
