"""Pins of the oracle's DG operator.

* K^T = S K S (the discrete form of the adjoint relation between the forward
  and backward Maxwell operators, eq. (3.x) after the weak formulation), which
  makes P* = S P S exact for any RK polynomial;
* centred flux with PEC walls and sigma = 0 is skew: K + K^T = 0 (energy
  conservation of the semi-discrete scheme);
* the upwind dissipation equals its closed form (jumps on interior faces,
  tangential traces on PEC / impedance faces, sigma |E|^2);
* consistency: a continuous polynomial field of degree <= q is mapped to its
  exact curl on elements without boundary faces.
"""
import numpy as np
import pytest

from paper_2106_02858_amd import inputs
from oracle import dg, mesh as omesh, refelem
from tests._problems import hetero_problem


def K_and_S(p):
    B = dg.assemble_B(p)
    M = dg.mass_matrix(p)
    K = -(M @ B)
    s = np.ones((p.K, 6, p.Np))
    s[:, 3:6] = -1
    return K, s.ravel()


@pytest.mark.parametrize("q", [1, 2, 3])
def test_KT_equals_SKS(q):
    p = hetero_problem(n=2 if q < 3 else 1, q=q, seed=q)
    K, s = K_and_S(p)
    SKS = K.multiply(s[:, None]).multiply(s[None, :])
    err = abs(K.T - SKS).max()
    assert err <= 1e-14 * abs(K).max()


@pytest.mark.parametrize("q", [1, 2])
def test_central_pec_skew(q):
    p = hetero_problem(n=2, q=q, seed=5, alpha=0.0, sigma=False, tags=inputs.TAG_PEC)
    K, _ = K_and_S(p)
    assert abs(K + K.T).max() <= 1e-14 * abs(K).max()


def face_integral(p, f, a, b):
    """int over local face f of every element of a . b (a, b: [K, Nfp, 3])."""
    Ef = p.ref["Ef"][f]
    return p.geo.area[:, f] * np.einsum("eic,ij,ejc->e", a, Ef, b)


@pytest.mark.parametrize("q", [1, 2, 3])
def test_upwind_dissipation_closed_form(q):
    p = hetero_problem(n=2 if q < 3 else 1, q=q, seed=10 + q)
    rng = np.random.default_rng(1)
    U = rng.standard_normal((p.K, 6, p.Np))
    rate = dg.inner(p, dg.apply_B(p, U), U)  # d/dt (1/2)||U||^2
    geo = p.geo
    fm = p.ref["fmask"]
    Z = np.sqrt(p.mu / p.eps)
    total = 0.0
    for f in range(4):
        n = geo.normal[:, f][:, None, :]
        E = np.transpose(U[:, 0:3][:, :, fm[f]], (0, 2, 1))
        H = np.transpose(U[:, 3:6][:, :, fm[f]], (0, 2, 1))
        tau = lambda X: X - np.sum(X * n, -1, keepdims=True) * n
        Et, Ht = tau(E), tau(H)
        imp = geo.tag[:, f] == omesh.TAG_IMPEDANCE
        pec = geo.tag[:, f] == omesh.TAG_PEC
        total -= np.sum((face_integral(p, f, Et, Et) / (2 * Z) + Z * face_integral(p, f, Ht, Ht) / 2)[imp])
        total -= np.sum((face_integral(p, f, Et, Et) / Z)[pec])
        inter = geo.nbr[:, f] >= 0
        e2 = geo.nbr[:, f].clip(min=0)
        node2 = geo.nbr_node[:, f].clip(min=0)
        E2 = np.transpose(U[e2][:, 0:3], (0, 2, 1))[np.arange(p.K)[:, None], node2]
        H2 = np.transpose(U[e2][:, 3:6], (0, 2, 1))[np.arange(p.K)[:, None], node2]
        dEt, dHt = tau(E2 - E), tau(H2 - H)
        Z2 = Z[e2]
        # each interior face is visited from both sides: half weight
        contrib = 0.5 * (face_integral(p, f, dEt, dEt) / (Z + Z2) + face_integral(p, f, dHt, dHt) / (1 / Z + 1 / Z2))
        total -= np.sum(contrib[inter])
    E = U[:, 0:3]
    ME = np.einsum("ij,ecj->eci", p.ref["M"], E)
    total -= np.sum(p.sigma[:, None, None] * p.geo.vol[:, None, None] * E * ME)
    assert abs(rate - total) <= 1e-12 * abs(total)
    assert rate < 0


@pytest.mark.parametrize("q", [1, 2, 3])
def test_polynomial_consistency(q):
    """For a continuous field of degree q, interior elements see the exact
    -curl H / eps and curl E / mu (all jumps vanish)."""
    p = hetero_problem(n=3 if q < 3 else 2, q=q, seed=3, source=False)
    x = p.geo.x
    rng = np.random.default_rng(7)
    exps = [(a, b, c) for a in range(q + 1) for b in range(q + 1) for c in range(q + 1) if a + b + c <= q]
    coef = rng.standard_normal((6, len(exps)))
    U = np.zeros((p.K, 6, p.Np))
    grad = np.zeros((p.K, 6, 3, p.Np))
    for m, e in enumerate(exps):
        val = x[..., 0] ** e[0] * x[..., 1] ** e[1] * x[..., 2] ** e[2]
        for d in range(3):
            de = list(e)
            c = de[d]
            de[d] = max(de[d] - 1, 0)
            dv = c * x[..., 0] ** de[0] * x[..., 1] ** de[1] * x[..., 2] ** de[2]
            grad[:, :, d] += coef[:, m][None, :, None] * dv[:, None, :]
        U += coef[:, m][None, :, None] * val[:, None, :]

    def curl(g):
        return np.stack([g[:, 2, 1] - g[:, 1, 2], g[:, 0, 2] - g[:, 2, 0], g[:, 1, 0] - g[:, 0, 1]], 1)

    r = dg.apply_B(p, U)
    interior = np.all(p.geo.nbr >= 0, axis=1)
    assert interior.sum() > 0
    ex_E = (-curl(grad[:, 3:6]) - p.sigma[:, None, None] * U[:, 0:3]) / p.eps[:, None, None]
    ex_H = curl(grad[:, 0:3]) / p.mu[:, None, None]
    scale = np.abs(ex_E).max() + np.abs(ex_H).max()
    assert np.max(np.abs(r[interior, 0:3] - ex_E[interior])) < 1e-11 * scale
    assert np.max(np.abs(r[interior, 3:6] - ex_H[interior])) < 1e-11 * scale


def test_mesh_geometry_basic():
    xyz, tet, tags = inputs.cube_mesh(3)
    g = omesh.build(xyz, tet, tags, 2)
    assert abs(g.vol.sum() - 1.0) < 1e-14
    # Kuhn tets: insphere diameter a / (1 + sqrt 2)
    assert np.allclose(g.rho, (1 / 3) / (1 + np.sqrt(2)))
    # outward normals of matched faces are opposite
    e, f = np.nonzero(g.nbr >= 0)
    e2 = g.nbr[e, f]
    dots = []
    for a, b, c in zip(e, f, e2):
        f2 = np.nonzero(g.nbr[c] == a)[0][0]
        dots.append(np.dot(g.normal[a, b], g.normal[c, f2]))
    assert np.allclose(dots, -1.0)
    # closed surface: sum of area-weighted normals vanishes per element
    assert np.max(np.abs(np.einsum("ef,efc->ec", g.area, g.normal))) < 1e-14
