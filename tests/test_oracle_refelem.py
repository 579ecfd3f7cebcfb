"""Pins of the oracle's reference element against independent computations:
exact differentiation of polynomials, a collapsed Gauss quadrature for the
volume and face mass matrices (the oracle uses Dirichlet moments), and the
lift identity M LIFT = [E_0 .. E_3]."""
import itertools

import numpy as np
import pytest

from oracle import refelem


def monomials(q):
    return [(a, b, c) for a in range(q + 1) for b in range(q + 1) for c in range(q + 1) if a + b + c <= q]


def eval_mono(e, x):
    return x[..., 0] ** e[0] * x[..., 1] ** e[1] * x[..., 2] ** e[2]


def lagrange_at(q, pts):
    """Nodal basis values at pts via a Cartesian monomial Vandermonde."""
    nodes = refelem.nodes(q)
    ms = monomials(q)
    V = np.stack([eval_mono(e, nodes) for e in ms], axis=1)
    W = np.stack([eval_mono(e, pts) for e in ms], axis=1)
    return W @ np.linalg.inv(V)  # [npts, Np]


def tet_quadrature(n):
    """Stroud conical product rule on the unit tetrahedron (Duffy collapse)."""
    x, w = np.polynomial.legendre.leggauss(n)
    x = 0.5 * (x + 1)
    w = 0.5 * w
    pts, wts = [], []
    for (u, wu), (v, wv), (s, ws) in itertools.product(zip(x, w), zip(x, w), zip(x, w)):
        pts.append((u, v * (1 - u), s * (1 - u) * (1 - v)))
        wts.append(wu * wv * ws * (1 - u) ** 2 * (1 - v))
    return np.array(pts), np.array(wts)


def tri_quadrature(n):
    x, w = np.polynomial.legendre.leggauss(n)
    x = 0.5 * (x + 1)
    w = 0.5 * w
    pts, wts = [], []
    for (u, wu), (v, wv) in itertools.product(zip(x, w), zip(x, w)):
        pts.append((u, v * (1 - u)))
        wts.append(wu * wv * (1 - u))
    return np.array(pts), np.array(wts)


FACE_VERTS = {0: [(1, 0, 0), (0, 1, 0), (0, 0, 1)], 1: [(0, 0, 0), (0, 1, 0), (0, 0, 1)],
              2: [(0, 0, 0), (1, 0, 0), (0, 0, 1)], 3: [(0, 0, 0), (1, 0, 0), (0, 1, 0)]}


@pytest.mark.parametrize("q", [1, 2, 3])
def test_node_count_and_order(q):
    xi = refelem.nodes(q)
    assert xi.shape == (refelem.np_count(q), 3)
    # k slowest, then j, i fastest
    lab = np.rint(xi * q).astype(int)
    key = lab[:, 2] * 100 + lab[:, 1] * 10 + lab[:, 0]
    assert np.all(np.diff(key) > 0)
    fm = refelem.face_nodes(q)
    assert all(len(f) == refelem.nfp_count(q) for f in fm)
    assert np.allclose(xi[fm[1], 0], 0) and np.allclose(xi[fm[2], 1], 0) and np.allclose(xi[fm[3], 2], 0)
    assert np.allclose(xi[fm[0]].sum(1), 1)


@pytest.mark.parametrize("q", [1, 2, 3])
def test_differentiation_exact_on_polynomials(q):
    m = refelem.matrices(q)
    xi = refelem.nodes(q)
    for e in monomials(q):
        f = eval_mono(e, xi)
        for k in range(3):
            de = list(e)
            coef = de[k]
            de[k] = max(de[k] - 1, 0)
            exact = coef * eval_mono(tuple(de), xi)
            assert np.max(np.abs(m["D"][k] @ f - exact)) < 1e-12


@pytest.mark.parametrize("q", [1, 2, 3])
def test_mass_matrix_against_quadrature(q):
    m = refelem.matrices(q)
    pts, wts = tet_quadrature(q + 3)
    L = lagrange_at(q, pts)
    Mq = 6.0 * (L * wts[:, None]).T @ L  # unit-volume element: |T_hat| = 1/6
    assert np.max(np.abs(Mq - m["M"])) < 1e-13
    assert abs(m["M"].sum() - 1.0) < 1e-14


@pytest.mark.parametrize("q", [1, 2, 3])
def test_face_mass_and_lift_against_quadrature(q):
    m = refelem.matrices(q)
    fm = refelem.face_nodes(q)
    Nfp = refelem.nfp_count(q)
    pts, wts = tri_quadrature(q + 3)
    for f in range(4):
        a, b, c = (np.array(v, dtype=float) for v in FACE_VERTS[f])
        X = a[None] + pts[:, 0:1] * (b - a)[None] + pts[:, 1:2] * (c - a)[None]
        L = lagrange_at(q, X)
        Ef = 2.0 * (L * wts[:, None]).T @ L  # unit-area face: |tri_hat| = 1/2
        # basis functions of nodes off the face vanish on it
        off = [n for n in range(L.shape[1]) if n not in fm[f]]
        assert np.max(np.abs(L[:, off])) < 1e-12
        assert np.max(np.abs(Ef[np.ix_(fm[f], fm[f])] - m["Ef"][f])) < 1e-13
        # lift identity: M LIFT_f = E_f restricted to face-node columns
        ML = m["M"] @ m["LIFT"][:, f * Nfp:(f + 1) * Nfp]
        assert np.max(np.abs(ML - Ef[:, fm[f]])) < 1e-13
