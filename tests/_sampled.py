"""Oracle right-hand side at sampled elements of a mesh too large for the
oracle: each sampled element is evaluated on the submesh of it and its face
neighbours, with its global boundary tags, where its right-hand side equals
the one on the full mesh."""
import numpy as np

from oracle import dg
from paper_2106_02858_amd import inputs

FACE_VERTS = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])  # face f opposite vertex f


def face_neighbours(tet, elems):
    """Global face neighbour (or -1) of every face of the elements `elems`.
    A face is keyed by its sorted vertex triple (a, b, c) as the pair
    (a nv + b, c), which stays within int64 for any vertex count below 3e9."""
    nv = int(tet.max()) + 1
    f = np.sort(tet[:, FACE_VERTS], axis=2).astype(np.int64)           # [K][4][3]
    k1 = (f[..., 0] * nv + f[..., 1]).ravel()
    k2 = f[..., 2].ravel()
    order = np.lexsort((k2, k1))                                         # by k1, then k2
    s1 = k1[order]
    out = -np.ones((len(elems), 4), dtype=np.int64)
    for i, e in enumerate(elems):
        for fi in range(4):
            a, c = k1[4 * e + fi], k2[4 * e + fi]
            lo = np.searchsorted(s1, a, side="left")
            hi = np.searchsorted(s1, a, side="right")
            for j in order[lo:hi]:
                if k2[j] == c and j // 4 != e:
                    out[i, fi] = j // 4
    return out


def sampled_oracle_rhs(w, nodes, U, samples, t, with_source=True):
    """Oracle right-hand side at the sampled elements.  U needs only to
    support U[element indices] (an array, or a function of the indices)."""
    nb = face_neighbours(w.tet, samples)
    elems = np.unique(np.concatenate([samples, nb[nb >= 0]]))
    pos = {int(e): i for i, e in enumerate(elems)}
    sub_tet_g = w.tet[elems]
    verts, inv = np.unique(sub_tet_g.ravel(), return_inverse=True)
    sub_tet = inv.reshape(-1, 4)
    sub_xyz = w.xyz[verts]
    # tags: global boundary tags; interior faces whose neighbour is outside the
    # submesh become impedance faces (those elements are not compared)
    all_nb = face_neighbours(w.tet, elems)
    tags = np.array(w.tags[elems], copy=True)
    for i in range(len(elems)):
        for f in range(4):
            g = all_nb[i, f]
            if g >= 0:
                tags[i, f] = 0 if int(g) in pos else inputs.TAG_IMPEDANCE
    j = inputs.gaussian_current(nodes[elems], w.centre, w.width, w.pol) if with_source else None
    op = dg.make_problem(sub_xyz, sub_tet, tags, w.q, w.eps[elems], w.mu[elems], w.sigma[elems],
                         omega=w.omega, j=j)
    if nodes is not None:
        assert np.max(np.abs(op.geo.x - nodes[elems])) < 1e-14  # same nodes, same order
    ref = dg.phi(op, t, U(elems) if callable(U) else U[elems], with_source=with_source)
    return ref[[pos[int(e)] for e in samples]]


def sample_elements(w, rng, extra=()):
    K = w.K
    s = set(int(x) for x in rng.choice(K, 40, replace=False))
    s.update([0, K - 1, K - 2] + [int(x) for x in extra])
    bnd = np.nonzero((w.tags != 0).any(axis=1))[0]
    s.update(int(x) for x in rng.choice(bnd, 6, replace=False))
    return np.array(sorted(s))
