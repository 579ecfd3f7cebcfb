"""Upwind nodal DG semi-discretisation of the 2-D transverse-magnetic system
(Section 5.2.1, two-dimensional setting; Section 5.2.2, DG discretisation).

Fields: e (the out-of-plane electric component) and h = (h1, h2).  With
scurl h = d1 h2 - d2 h1 and vcurl e = (d2 e, -d1 e) the system is

  eps de/dt + sigma e + scurl h = j,     mu dh/dt - vcurl e = 0,

the 3-D system of eq. (1.2) for fields that do not depend on x3.  The scheme
here is the 3-D oracle's strong form restricted to such fields (normal
n = (n1, n2, 0), E = (0, 0, e) always tangential): with "+" the neighbour or
ghost state, "-" the own state, d = (+) - (-), n x dh = n1 dh2 - n2 dh1,
n x de = (n2 de, -n1 de),

  eps de/dt = -scurl h - sigma e + j + L[(alpha de - Z+ n x dh)/(Z- + Z+)]
  mu  dh/dt = +vcurl e             + L[(alpha dh_tau + Y+ n x de)/(Y- + Y+)]

with L[g] = M_K^-1 int_dK g phi.  Ghosts: PEC e+ = -e-, h+ = h-; impedance
(e + Z h x n = G, the characteristic entering the domain prescribed)
e+ = G, h+ = 0 with alpha = 1.  For equal impedances on both sides these are
the printed 2-D upwind fluxes with the average read as half the sum.  alpha
scales the jump penalty on interior and PEC edges: 1 is the exact Riemann
(upwind) flux, 0 the centred flux, 2 twice the upwind penalty.

Dof layout: U[K, 3, Np], components (e, h1, h2).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import dg as dg3
from . import mesh2d
from . import refelem2d


@dataclass
class Problem2D:
    geo: mesh2d.Geometry2D
    ref: dict
    eps: np.ndarray
    mu: np.ndarray
    sigma: np.ndarray
    omega: float
    j: np.ndarray | None      # complex [K, Np] nodal current density
    g: np.ndarray | None      # complex [K, 3, Nfp] impedance boundary data G
    alpha: float = 1.0

    dim = 2
    ncomp = 3

    @property
    def K(self):
        return self.geo.K

    @property
    def Np(self):
        return self.geo.Np

    @property
    def ndof(self):
        return self.geo.K * 3 * self.geo.Np


def make_problem(xy, tri, edge_tag, q, eps, mu, sigma=None, omega=2 * np.pi, j=None, g=None,
                 alpha=1.0) -> Problem2D:
    geo = mesh2d.build(xy, tri, edge_tag, q)
    K = geo.K
    eps = np.asarray(eps, dtype=np.float64).reshape(K)
    mu = np.asarray(mu, dtype=np.float64).reshape(K)
    sigma = np.zeros(K) if sigma is None else np.asarray(sigma, dtype=np.float64).reshape(K)
    if j is not None:
        j = np.asarray(j, dtype=np.complex128).reshape(K, geo.Np)
    if g is not None:
        g = np.asarray(g, dtype=np.complex128).reshape(K, 3, geo.Nfp)
    return Problem2D(geo, refelem2d.matrices(q), eps, mu, sigma, float(omega), j, g, float(alpha))


def _lift(p: Problem2D, flux):
    """L[.] with edge scaling.  flux: [K, 3 edges, Nfp, c] -> [K, c, Np]."""
    K, Nfp = p.geo.K, p.geo.Nfp
    f = (flux * p.geo.fscale[:, :, None, None]).reshape(K, 3 * Nfp, flux.shape[-1])
    return np.einsum("ik,ekc->eci", p.ref["LIFT"], f)


def _rhs(p: Problem2D, U: np.ndarray, ghost_e: np.ndarray | None) -> np.ndarray:
    """B U (ghost_e None) or the impedance-data term alone (U ignored,
    ghost_e = G at the edge nodes)."""
    geo, ref = p.geo, p.ref
    K, Np, Nfp = geo.K, geo.Np, geo.Nfp
    n = np.broadcast_to(geo.normal[:, :, None, :], (K, 3, Nfp, 2))
    Zm = np.sqrt(p.mu / p.eps)
    interior = geo.nbr >= 0
    nb = np.where(interior, geo.nbr, 0)
    Zp = np.where(interior, Zm[nb], Zm[:, None])
    Zmf = np.broadcast_to(Zm[:, None], (K, 3))
    Ym, Yp = 1.0 / Zmf, 1.0 / Zp
    imp = geo.tag == mesh2d.TAG_IMPEDANCE
    alpha = np.where(imp, 1.0, p.alpha)[:, :, None]
    if ghost_e is None:
        U = U.reshape(K, 3, Np)
        dref = np.einsum("aij,ecj->ecai", ref["D"], U)        # [K,3,2,Np]
        grad = np.einsum("eak,ecai->ecki", geo.G, dref)       # [K,3,2(x_k),Np]
        scurl_h = grad[:, 2, 0] - grad[:, 1, 1]
        vcurl_e = np.stack([grad[:, 0, 1], -grad[:, 0, 0]], axis=1)
        Uf = np.transpose(U[:, :, ref["fmask"]], (0, 2, 3, 1))  # [K,3 edges,Nfp,3 comps]
        Up = U[nb[:, :, None], :, geo.nbr_node.clip(min=0)]     # [K,3,Nfp,3]
        Up = np.where(interior[:, :, None, None], Up, 0.0)
        pec = (geo.tag == mesh2d.TAG_PEC)[:, :, None]
        Up[..., 0] = np.where(pec, -Uf[..., 0], Up[..., 0])
        Up[..., 1:3] = np.where(pec[..., None], Uf[..., 1:3], Up[..., 1:3])
        de = Up[..., 0] - Uf[..., 0]
        dh = Up[..., 1:3] - Uf[..., 1:3]
    else:
        de = np.where(imp[:, :, None], ghost_e, 0.0)
        dh = np.zeros((K, 3, Nfp, 2))
    n_x_dh = n[..., 0] * dh[..., 1] - n[..., 1] * dh[..., 0]
    n_x_de = np.stack([n[..., 1] * de, -n[..., 0] * de], axis=-1)
    dh_tau = dh - np.sum(n * dh, axis=-1, keepdims=True) * n
    flux_e = (alpha * de - Zp[:, :, None] * n_x_dh) / (Zmf + Zp)[:, :, None]
    flux_h = (alpha[..., None] * dh_tau + Yp[:, :, None, None] * n_x_de) / (Ym + Yp)[:, :, None, None]
    Le = _lift(p, flux_e[..., None])[:, 0]
    Lh = _lift(p, flux_h)
    out = np.empty((K, 3, Np))
    if ghost_e is None:
        out[:, 0] = (-scurl_h - p.sigma[:, None] * U[:, 0] + Le) / p.eps[:, None]
        out[:, 1:3] = (vcurl_e + Lh) / p.mu[:, None, None]
    else:
        out[:, 0] = Le / p.eps[:, None]
        out[:, 1:3] = Lh / p.mu[:, None, None]
    return out


def apply_B(p: Problem2D, U: np.ndarray) -> np.ndarray:
    """B U: the homogeneous DG right-hand side (no j, no G)."""
    return _rhs(p, U, None)


def source(p: Problem2D, t: float) -> np.ndarray:
    """Re(JJ e^{i omega t}): current density and impedance boundary data."""
    out = np.zeros((p.K, 3, p.Np))
    ph = np.exp(1j * p.omega * t)
    if p.j is not None:
        out[:, 0] += np.real(p.j * ph) / p.eps[:, None]
    if p.g is not None:
        out += _rhs(p, None, np.real(p.g * ph))
    return out


def phi(p: Problem2D, t: float, U: np.ndarray, with_source: bool = True) -> np.ndarray:
    """Phi(t, U) of the semi-discrete ODE system (Section 5.2.2)."""
    r = apply_B(p, U)
    if with_source:
        r = r + source(p, t)
    return r


def mass_weights(p: Problem2D) -> np.ndarray:
    """Per (element, component) weight |K| eps_K (e) or |K| mu_K (h)."""
    w = np.empty((p.K, 3))
    w[:, 0] = p.geo.vol * p.eps
    w[:, 1:3] = (p.geo.vol * p.mu)[:, None]
    return w


def inner(p: Problem2D, U: np.ndarray, V: np.ndarray):
    """(U, V)_{eps,mu} = V^H M U with the block-diagonal DG mass."""
    U = U.reshape(p.K, 3, p.Np)
    V = V.reshape(p.K, 3, p.Np)
    MV = np.einsum("ij,ecj->eci", p.ref["M"], V)
    w = mass_weights(p)
    return np.sum(w[:, :, None] * np.conj(MV) * U) if np.iscomplexobj(V) else np.sum(w[:, :, None] * MV * U)


def norm(p: Problem2D, U: np.ndarray) -> float:
    return float(np.sqrt(np.real(inner(p, U, U))))


def mass_matrix(p: Problem2D) -> sp.csr_matrix:
    w = mass_weights(p)
    blocks = [sp.csr_matrix(w[e, c] * p.ref["M"]) for e in range(p.K) for c in range(3)]
    return sp.block_diag(blocks, format="csr")


def flip_H(U: np.ndarray) -> np.ndarray:
    """S U with S = diag(1, -1, -1): the magnetic sign flip of P* = S P S."""
    V = np.array(U, copy=True)
    V[:, 1:3] *= -1.0
    return V


def assemble_B(p: Problem2D) -> sp.csr_matrix:
    """The matrix of U -> apply_B(U), probed one (colour, local dof) at a time
    with a distance-2 colouring of the element graph: the probe's response in
    element r belongs to the one probed element in r's neighbourhood."""
    K, Np = p.K, p.Np
    color, nbrs = dg3._distance2_coloring(p.geo)
    rows, cols, vals = [], [], []
    nd = 3 * Np
    for c in range(int(color.max()) + 1):
        es = np.nonzero(color == c)[0]
        owner = -np.ones(K, dtype=np.int64)
        owner[es] = es
        for f in range(3):
            nb = p.geo.nbr[es, f]
            owner[nb[nb >= 0]] = es[nb >= 0]
        for ld in range(nd):
            x = np.zeros((K, nd))
            x[es, ld] = 1.0
            y = apply_B(p, x.reshape(K, 3, Np)).reshape(-1)
            nz = np.nonzero(y)[0]
            assert np.all(owner[nz // nd] >= 0)
            rows.append(nz)
            cols.append(owner[nz // nd] * nd + ld)
            vals.append(y[nz])
    n = K * nd
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def source_vector(p: Problem2D) -> np.ndarray:
    """Complex JJ with Re(JJ e^{i omega t}) = source(t) (flattened)."""
    c = source(p, 0.0)
    s = source(p, np.pi / (2 * p.omega))
    return (c - 1j * s).reshape(-1)
