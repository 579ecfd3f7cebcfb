"""Triangle-mesh connectivity and affine geometry for the 2-D DG oracle
(Section 5.2: conforming triangulation, edge sets F_int / F_P / F_I, outward
normals, rho_K the diameter of the inscribed circle).

Edges are matched through their sorted vertex pairs, edge nodes through their
physical coordinates; normals are the edge directions turned a quarter turn
and oriented away from the opposite vertex.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import refelem2d

TAG_INTERIOR = 0
TAG_PEC = 1
TAG_IMPEDANCE = 2


@dataclass
class Geometry2D:
    q: int
    K: int
    Np: int
    Nfp: int
    x: np.ndarray          # [K, Np, 2] node coordinates
    vol: np.ndarray        # [K] triangle areas
    G: np.ndarray          # [K, 2, 2]  G[e, a, k] = d xi_a / d x_k
    normal: np.ndarray     # [K, 3, 2]  outward unit normals
    length: np.ndarray     # [K, 3]
    fscale: np.ndarray     # [K, 3]  length / area
    nbr: np.ndarray        # [K, 3]  neighbour element or -1
    nbr_node: np.ndarray   # [K, 3, Nfp] element-node index in the neighbour
    tag: np.ndarray        # [K, 3]  0 interior, 1 PEC, 2 impedance
    rho: np.ndarray        # [K] inscribed-circle diameter 4|K| / perimeter


def build(xy: np.ndarray, tri: np.ndarray, edge_tag: np.ndarray, q: int) -> Geometry2D:
    xy = np.asarray(xy, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.int64)
    K = tri.shape[0]
    v = xy[tri]  # [K,3,2]
    Jm = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]], axis=2)  # columns
    det = np.linalg.det(Jm)
    if np.any(np.abs(det) < 1e-300):
        raise ValueError("degenerate triangle")
    vol = np.abs(det) / 2.0
    G = np.linalg.inv(Jm)
    normal = np.zeros((K, 3, 2))
    length = np.zeros((K, 3))
    for f in range(3):
        a, b = [k for k in range(3) if k != f]
        t = v[:, b] - v[:, a]
        L = np.linalg.norm(t, axis=1)
        nvec = np.stack([t[:, 1], -t[:, 0]], axis=1) / L[:, None]
        away = np.sum(nvec * (v[:, f] - v[:, a]), axis=1)
        nvec[away > 0] *= -1.0
        normal[:, f] = nvec
        length[:, f] = L
    fscale = length / vol[:, None]
    rho = 4.0 * vol / length.sum(axis=1)
    xi = refelem2d.nodes(q)
    x = v[:, 0][:, None, :] + np.einsum("kab,nb->kna", Jm, xi)
    Np = xi.shape[0]
    fm = refelem2d.face_nodes(q)
    Nfp = len(fm[0])
    owner = {}
    nbr = -np.ones((K, 3), dtype=np.int64)
    nbr_face = -np.ones((K, 3), dtype=np.int64)
    for e in range(K):
        for f in range(3):
            key = tuple(sorted(int(tri[e, k]) for k in range(3) if k != f))
            if key in owner:
                e2, f2 = owner.pop(key)
                nbr[e, f], nbr_face[e, f] = e2, f2
                nbr[e2, f2], nbr_face[e2, f2] = e, f
            else:
                owner[key] = (e, f)
    tag = np.asarray(edge_tag, dtype=np.int64).copy()
    interior = nbr >= 0
    tag[interior] = TAG_INTERIOR
    if np.any(tag[~interior] == TAG_INTERIOR):
        raise ValueError("untagged boundary edge")
    nbr_node = -np.ones((K, 3, Nfp), dtype=np.int64)
    for f in range(3):
        es = np.nonzero(interior[:, f])[0]
        if es.size == 0:
            continue
        mine = x[es][:, fm[f], :]
        theirs_idx = np.array(fm)[nbr_face[es, f]]
        theirs = x[nbr[es, f][:, None], theirs_idx]
        d = np.linalg.norm(mine[:, :, None, :] - theirs[:, None, :, :], axis=-1)
        j = np.argmin(d, axis=2)
        if np.max(np.take_along_axis(d, j[:, :, None], axis=2)) > 1e-9:
            raise ValueError("edge nodes do not match")
        nbr_node[es, f] = np.take_along_axis(theirs_idx, j, axis=1)
    return Geometry2D(q, K, Np, Nfp, x, vol, G, normal, length, fscale, nbr, nbr_node, tag, rho)
