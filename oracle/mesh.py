"""Mesh connectivity and affine geometry for the DG oracle (Section 5.2:
conforming simplicial mesh, face sets F_int / F_P / F_I, outward normals).

Plain and direct: faces are matched through their sorted vertex triples,
face nodes are matched through their physical coordinates, normals come
from cross products oriented away from the opposite vertex.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import refelem

TAG_INTERIOR = 0
TAG_PEC = 1
TAG_IMPEDANCE = 2


@dataclass
class Geometry:
    q: int
    K: int
    Np: int
    Nfp: int
    x: np.ndarray          # [K, Np, 3] node coordinates
    vol: np.ndarray        # [K]
    G: np.ndarray          # [K, 3, 3]  G[e, a, k] = d xi_a / d x_k
    normal: np.ndarray     # [K, 4, 3]  outward unit normals
    area: np.ndarray       # [K, 4]
    fscale: np.ndarray     # [K, 4]  area / volume
    nbr: np.ndarray        # [K, 4]  neighbour element or -1
    nbr_node: np.ndarray   # [K, 4, Nfp] element-node index in the neighbour
    tag: np.ndarray        # [K, 4]  0 interior, 1 PEC, 2 impedance
    rho: np.ndarray        # [K] insphere diameter 6|K| / area(dK)


def build(xyz: np.ndarray, tet: np.ndarray, face_tag: np.ndarray, q: int) -> Geometry:
    xyz = np.asarray(xyz, dtype=np.float64)
    tet = np.asarray(tet, dtype=np.int64)
    K = tet.shape[0]
    v = xyz[tet]  # [K,4,3]
    Jm = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]], axis=2)  # columns
    det = np.linalg.det(Jm)
    if np.any(np.abs(det) < 1e-300):
        raise ValueError("degenerate tetrahedron")
    vol = np.abs(det) / 6.0
    G = np.linalg.inv(Jm)  # rows: grad xi_a
    # faces: face f is opposite local vertex f
    normal = np.zeros((K, 4, 3))
    area = np.zeros((K, 4))
    for f in range(4):
        o = [a for a in range(4) if a != f]
        p0, p1, p2 = v[:, o[0]], v[:, o[1]], v[:, o[2]]
        cr = np.cross(p1 - p0, p2 - p0)
        a2 = np.linalg.norm(cr, axis=1)
        nvec = cr / a2[:, None]
        away = np.sum(nvec * (v[:, f] - p0), axis=1)
        nvec[away > 0] *= -1.0
        normal[:, f] = nvec
        area[:, f] = 0.5 * a2
    fscale = area / vol[:, None]
    rho = 6.0 * vol / area.sum(axis=1)
    # nodes
    xi = refelem.nodes(q)
    x = v[:, 0][:, None, :] + np.einsum("kab,nb->kna", Jm, xi)
    Np = xi.shape[0]
    fm = refelem.face_nodes(q)
    Nfp = len(fm[0])
    # face matching through sorted vertex triples
    owner = {}
    nbr = -np.ones((K, 4), dtype=np.int64)
    nbr_face = -np.ones((K, 4), dtype=np.int64)
    for e in range(K):
        for f in range(4):
            key = tuple(sorted(int(tet[e, a]) for a in range(4) if a != f))
            if key in owner:
                e2, f2 = owner.pop(key)
                if e2 == -2:
                    raise ValueError("non-conforming mesh: face shared by more than two tets")
                nbr[e, f], nbr_face[e, f] = e2, f2
                nbr[e2, f2], nbr_face[e2, f2] = e, f
            else:
                owner[key] = (e, f)
    tag = np.asarray(face_tag, dtype=np.int64).copy()
    interior = nbr >= 0
    tag[interior] = TAG_INTERIOR
    if np.any(tag[~interior] == TAG_INTERIOR):
        raise ValueError("untagged boundary face")
    # face-node matching through physical coordinates
    nbr_node = -np.ones((K, 4, Nfp), dtype=np.int64)
    for f in range(4):
        es = np.nonzero(interior[:, f])[0]
        if es.size == 0:
            continue
        mine = x[es][:, fm[f], :]  # [n, Nfp, 3]
        e2 = nbr[es, f]
        f2 = nbr_face[es, f]
        theirs_idx = np.array(fm)[f2]  # [n, Nfp]
        theirs = x[e2[:, None], theirs_idx]  # [n, Nfp, 3]
        d = np.linalg.norm(mine[:, :, None, :] - theirs[:, None, :, :], axis=-1)
        j = np.argmin(d, axis=2)
        if np.max(np.take_along_axis(d, j[:, :, None], axis=2)) > 1e-9:
            raise ValueError("face nodes do not match")
        nbr_node[es, f] = np.take_along_axis(theirs_idx, j, axis=1)
    return Geometry(q, K, Np, Nfp, x, vol, G, normal, area, fscale, nbr, nbr_node, tag, rho)
