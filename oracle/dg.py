"""Upwind nodal DG semi-discretisation of the time-domain Maxwell system
(Section 5.2; the paper's 2-D TM scheme written for 3-D tetrahedra).

Field convention of eq. (1.2):  eps dE/dt + sigma E + curl H = J,
mu dH/dt - curl E = 0.  On an element K with outward normal n, neighbour
(or ghost) state "+", own state "-", Delta X = X+ - X-, X_tau = X - (n.X) n,
Z = sqrt(mu/eps), Y = 1/Z, the strong form used here is

  eps dE/dt = -curl H - sigma E + J + L[(alpha dE_tau - Z+ n x dH)/(Z- + Z+)]
  mu  dH/dt = +curl E             + L[(alpha dH_tau + Y+ n x dE)/(Y- + Y+)]

(the exact Riemann flux for alpha = 1; alpha = 0 gives the centred flux),
where L[g] = M_K^-1 int_dK g phi.  Ghost states: PEC  E+ = -E-, H+ = H-;
impedance (dissipative Silver-Mueller, E x n - Z H_tau = G)  E+ = n x G,
H+ = 0, always with alpha = 1.  Z+ = Z- on boundary faces.

Dof layout inside the oracle: U[K, 6, Np], components (Ex,Ey,Ez,Hx,Hy,Hz).
Phi(t, U) = Re(JJ e^{i omega t}) + B U with B = -M^-1 K (eq. 5.x, ODE system).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import mesh as omesh
from . import refelem


@dataclass
class Problem:
    geo: omesh.Geometry
    ref: dict
    eps: np.ndarray
    mu: np.ndarray
    sigma: np.ndarray
    omega: float
    j: np.ndarray | None      # complex [K, Np, 3] nodal current density
    g: np.ndarray | None      # complex [K, 4, Nfp, 3] impedance boundary data
    alpha: float = 1.0

    dim = 3
    ncomp = 6

    @property
    def K(self):
        return self.geo.K

    @property
    def Np(self):
        return self.geo.Np

    @property
    def ndof(self):
        return self.geo.K * 6 * self.geo.Np


def make_problem(xyz, tet, face_tag, q, eps, mu, sigma=None, omega=2 * np.pi, j=None, g=None,
                 alpha=1.0) -> Problem:
    geo = omesh.build(xyz, tet, face_tag, q)
    K = geo.K
    eps = np.asarray(eps, dtype=np.float64).reshape(K)
    mu = np.asarray(mu, dtype=np.float64).reshape(K)
    sigma = np.zeros(K) if sigma is None else np.asarray(sigma, dtype=np.float64).reshape(K)
    if j is not None:
        j = np.asarray(j, dtype=np.complex128).reshape(K, geo.Np, 3)
    if g is not None:
        g = np.asarray(g, dtype=np.complex128).reshape(K, 4, geo.Nfp, 3)
    return Problem(geo, refelem.matrices(q), eps, mu, sigma, float(omega), j, g, float(alpha))


def _cross(a, b):
    return np.cross(a, b, axis=-1)


def apply_B(p: Problem, U: np.ndarray) -> np.ndarray:
    """B U: the homogeneous DG right-hand side (no J, no G)."""
    return _rhs(p, U, None)


def source(p: Problem, t: float) -> np.ndarray:
    """Re(JJ e^{i omega t}): current density and impedance boundary data."""
    out = np.zeros((p.K, 6, p.Np))
    ph = np.exp(1j * p.omega * t)
    if p.j is not None:
        jt = np.real(p.j * ph)  # [K,Np,3]
        out[:, 0:3, :] += np.transpose(jt, (0, 2, 1)) / p.eps[:, None, None]
    if p.g is not None:
        out += _boundary_source(p, np.real(p.g * ph))
    return out


def phi(p: Problem, t: float, U: np.ndarray, with_source: bool = True) -> np.ndarray:
    """Phi(t, U) of the semi-discrete ODE system (Section 5.2)."""
    r = apply_B(p, U)
    if with_source:
        r = r + source(p, t)
    return r


def _lift(p: Problem, fluxE, fluxH):
    """L[.] with face scaling, divided by eps / mu.  flux*: [K,4,Nfp,3]."""
    geo, ref = p.geo, p.ref
    K, Nfp = geo.K, geo.Nfp
    fs = geo.fscale[:, :, None, None]
    fE = (fluxE * fs).reshape(K, 4 * Nfp, 3)
    fH = (fluxH * fs).reshape(K, 4 * Nfp, 3)
    LE = np.einsum("ik,ekc->eci", ref["LIFT"], fE, optimize=True)
    LH = np.einsum("ik,ekc->eci", ref["LIFT"], fH, optimize=True)
    return LE, LH


def _boundary_source(p: Problem, Gt: np.ndarray) -> np.ndarray:
    """Flux terms driven by the ghost E+ = n x G on impedance faces."""
    geo = p.geo
    n = geo.normal[:, :, None, :]
    imp = (geo.tag == omesh.TAG_IMPEDANCE)[:, :, None, None]
    nG = _cross(np.broadcast_to(n, Gt.shape), Gt)
    Z = np.sqrt(p.mu / p.eps)[:, None, None, None]
    fluxE = np.where(imp, nG / (2 * Z), 0.0)
    fluxH = np.where(imp, _cross(np.broadcast_to(n, Gt.shape), nG) / 2.0, 0.0)
    LE, LH = _lift(p, fluxE, fluxH)
    out = np.zeros((p.K, 6, p.Np))
    out[:, 0:3] = LE / p.eps[:, None, None]
    out[:, 3:6] = LH / p.mu[:, None, None]
    return out


def _rhs(p: Problem, U: np.ndarray, _unused) -> np.ndarray:
    geo, ref = p.geo, p.ref
    K, Np, Nfp = geo.K, geo.Np, geo.Nfp
    U = U.reshape(K, 6, Np)
    # volume term: reference derivatives, then physical gradient
    dref = np.einsum("aij,ecj->ecai", ref["D"], U, optimize=True)   # [K,6,3,Np]
    grad = np.einsum("eak,ecai->ecki", geo.G, dref, optimize=True)  # [K,6,3(x_k),Np]
    E_g, H_g = grad[:, 0:3], grad[:, 3:6]

    def curl(gr):  # gr[e, comp, dir, node]
        return np.stack([gr[:, 2, 1] - gr[:, 1, 2],
                         gr[:, 0, 2] - gr[:, 2, 0],
                         gr[:, 1, 0] - gr[:, 0, 1]], axis=1)

    curlE = curl(E_g)
    curlH = curl(H_g)
    # face traces [K,4,Nfp,6]
    fm = ref["fmask"]
    Uf = np.transpose(U[:, :, fm], (0, 2, 3, 1))
    interior = geo.nbr >= 0
    nb = np.where(interior, geo.nbr, 0)
    # neighbour traces at the matching nodes: [K,4,Nfp,6]
    Up_int = U[nb[:, :, None], :, geo.nbr_node.clip(min=0)]
    Up = np.where(interior[:, :, None, None], Up_int, 0.0)
    pec = (geo.tag == omesh.TAG_PEC)[:, :, None, None]
    Up[..., 0:3] = np.where(pec, -Uf[..., 0:3], Up[..., 0:3])
    Up[..., 3:6] = np.where(pec, Uf[..., 3:6], Up[..., 3:6])
    # impedance ghost: zero (homogeneous part)
    dE = Up[..., 0:3] - Uf[..., 0:3]
    dH = Up[..., 3:6] - Uf[..., 3:6]
    n = np.broadcast_to(geo.normal[:, :, None, :], dE.shape)
    Zm = np.sqrt(p.mu / p.eps)
    Zp_face = np.where(interior, Zm[nb], Zm[:, None])
    Zmf = np.broadcast_to(Zm[:, None], (K, 4))
    Ym, Yp = 1.0 / Zmf, 1.0 / Zp_face
    alpha = np.where(geo.tag == omesh.TAG_IMPEDANCE, 1.0, p.alpha)[:, :, None, None]
    ndE = np.sum(n * dE, axis=-1, keepdims=True)
    ndH = np.sum(n * dH, axis=-1, keepdims=True)
    dE_tau = dE - ndE * n
    dH_tau = dH - ndH * n
    fluxE = (alpha * dE_tau - Zp_face[:, :, None, None] * _cross(n, dH)) / (Zmf + Zp_face)[:, :, None, None]
    fluxH = (alpha * dH_tau + Yp[:, :, None, None] * _cross(n, dE)) / (Ym + Yp)[:, :, None, None]
    LE, LH = _lift(p, fluxE, fluxH)
    out = np.empty((K, 6, Np))
    out[:, 0:3] = (-curlH - p.sigma[:, None, None] * U[:, 0:3] + LE) / p.eps[:, None, None]
    out[:, 3:6] = (curlE + LH) / p.mu[:, None, None]
    return out


# ---------------------------------------------------------------- inner product

def mass_weights(p: Problem) -> np.ndarray:
    """Per (element, component) weight |K| eps_K (E rows) or |K| mu_K (H rows)."""
    w = np.empty((p.K, 6))
    w[:, 0:3] = (p.geo.vol * p.eps)[:, None]
    w[:, 3:6] = (p.geo.vol * p.mu)[:, None]
    return w


def inner(p: Problem, U: np.ndarray, V: np.ndarray):
    """(U, V)_{eps,mu} = V^T M U with the block-diagonal DG mass (Section 2.2)."""
    U = U.reshape(p.K, 6, p.Np)
    V = V.reshape(p.K, 6, p.Np)
    MV = np.einsum("ij,ecj->eci", p.ref["M"], V)
    w = mass_weights(p)
    return np.sum(w[:, :, None] * np.conj(MV) * U) if np.iscomplexobj(V) else np.sum(w[:, :, None] * MV * U)


def norm(p: Problem, U: np.ndarray) -> float:
    return float(np.sqrt(np.real(inner(p, U, U))))


def energy(p: Problem, U: np.ndarray) -> float:
    return 0.5 * norm(p, U) ** 2


def mass_matrix(p: Problem) -> sp.csr_matrix:
    w = mass_weights(p)
    blocks = [sp.csr_matrix(w[e, c] * p.ref["M"]) for e in range(p.K) for c in range(6)]
    return sp.block_diag(blocks, format="csr")


def flip_H(U: np.ndarray) -> np.ndarray:
    """S U with S = diag(I_E, -I_H): the magnetic sign flip that turns the
    forward propagator into its adjoint (Section 4.1.2)."""
    V = np.array(U, copy=True)
    V[:, 3:6] *= -1.0
    return V


# ---------------------------------------------------------------- probed matrix

def _distance2_coloring(geo: omesh.Geometry):
    K = geo.K
    nbrs = [set(int(x) for x in geo.nbr[e] if x >= 0) for e in range(K)]
    color = -np.ones(K, dtype=np.int64)
    for e in range(K):
        used = set()
        ring = set(nbrs[e]) | {e}
        for a in list(nbrs[e]):
            ring |= nbrs[a]
        for a in ring:
            if color[a] >= 0:
                used.add(int(color[a]))
        c = 0
        while c in used:
            c += 1
        color[e] = c
    return color, nbrs


def assemble_B(p: Problem) -> sp.csr_matrix:
    """The matrix of U -> apply_B(U), by probing with distance-2 colouring.

    Column (e, c, j) has its non-zeros in rows of e and its face neighbours;
    elements of one colour have disjoint row supports, so one probe per
    (colour, local dof) recovers all their columns at once."""
    geo = p.geo
    K, Np = geo.K, geo.Np
    color, nbrs = _distance2_coloring(geo)
    rows, cols, vals = [], [], []
    nd = 6 * Np
    for c in range(int(color.max()) + 1):
        es = np.nonzero(color == c)[0]
        for ld in range(nd):
            x = np.zeros((K, nd))
            x[es, ld] = 1.0
            y = apply_B(p, x.reshape(K, 6, Np)).reshape(K, nd)
            for e in es:
                for r in [e] + sorted(nbrs[e]):
                    nz = np.nonzero(y[r])[0]
                    rows.extend((r * nd + nz).tolist())
                    cols.extend([e * nd + ld] * len(nz))
                    vals.extend(y[r, nz].tolist())
    n = K * nd
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def source_vector(p: Problem) -> np.ndarray:
    """Complex JJ with Re(JJ e^{i omega t}) = source(t) (flattened)."""
    c = source(p, 0.0)
    s = source(p, np.pi / (2 * p.omega))  # Re(JJ e^{i pi/2}) = -Im JJ
    return (c - 1j * s).reshape(-1)
