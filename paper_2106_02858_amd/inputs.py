"""Seeded synthetic inputs for the CMCG Maxwell solver.

This module only *generates problem data* -- meshes, material coefficients,
source descriptions -- with numpy's PCG64 generator.  It contains none of the
method's arithmetic (no DG operator, no time stepping, no CG), so both the
HIP library and the CPU oracle may consume what it produces.

Workloads (3-D stand-ins for the paper's 2-D experiments, Section 6):

* ``cube_mesh(n)``: the unit cube split into n^3 cubes, each cut into the six
  Kuhn tetrahedra (o, o+a e_p1, o+a(e_p1+e_p2), o+a(1,1,1)), one per
  permutation p of the axes in lexicographic order.  Cube index
  c = i + n (j + n k), x fastest; tet index = 6 c + permutation index.
  The split is conforming under translation.
* Face tags follow the library convention: local face f is opposite local
  vertex f; tag 0 = interior, 1 = PEC, 2 = impedance (Silver-Mueller).
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

TAG_INTERIOR = 0
TAG_PEC = 1
TAG_IMPEDANCE = 2

_PERMS = list(itertools.permutations(range(3)))  # lexicographic order


def cube_mesh(n: int, boundary_tag: int = TAG_IMPEDANCE):
    """Kuhn split of [0,1]^3 into 6 n^3 tetrahedra.

    Returns (xyz [nv,3] float64, tet [K,4] int64, face_tag [K,4] int8).
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    nv1 = n + 1
    ii, jj, kk = np.meshgrid(np.arange(nv1), np.arange(nv1), np.arange(nv1), indexing="ij")
    # vertex index v = i + (n+1)(j + (n+1) k): x fastest
    lat = np.stack([ii.transpose(2, 1, 0).ravel(), jj.transpose(2, 1, 0).ravel(),
                    kk.transpose(2, 1, 0).ravel()], axis=1)
    xyz = lat.astype(np.float64) / n

    def vid(i, j, k):
        return i + nv1 * (j + nv1 * k)

    ci, cj, ck = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ci = ci.transpose(2, 1, 0).ravel()
    cj = cj.transpose(2, 1, 0).ravel()
    ck = ck.transpose(2, 1, 0).ravel()
    ncube = n ** 3
    tet = np.empty((ncube, 6, 4), dtype=np.int64)
    for p, perm in enumerate(_PERMS):
        off = np.zeros((ncube, 3), dtype=np.int64)
        corners = [off.copy()]
        for ax in perm:
            off = off.copy()
            off[:, ax] += 1
            corners.append(off)
        for v in range(4):
            tet[:, p, v] = vid(ci + corners[v][:, 0], cj + corners[v][:, 1], ck + corners[v][:, 2])
    tet = tet.reshape(-1, 4)
    tags = boundary_tags(lat, tet, n, boundary_tag)
    return xyz, tet, tags


def graded_cube_mesh(xs, ys, zs, boundary_tag: int = TAG_IMPEDANCE):
    """Kuhn split of the tensor-product grid xs x ys x zs (increasing vertex
    coordinates per axis) into 6 (len(xs)-1)(len(ys)-1)(len(zs)-1) tetrahedra,
    cells and tetrahedra numbered as in cube_mesh.  A grid with a few narrow
    cells is a conforming, locally refined mesh (the narrow cells' elements
    have small insphere diameters).  Returns (xyz, tet, face_tag)."""
    xs, ys, zs = (np.asarray(a, dtype=np.float64) for a in (xs, ys, zs))
    if min(len(xs), len(ys), len(zs)) < 2 or any(np.any(np.diff(a) <= 0) for a in (xs, ys, zs)):
        raise ValueError("coordinates must be increasing, at least two per axis")
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1
    ii, jj, kk = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1), indexing="ij")
    lat = np.stack([ii.transpose(2, 1, 0).ravel(), jj.transpose(2, 1, 0).ravel(),
                    kk.transpose(2, 1, 0).ravel()], axis=1)
    xyz = np.stack([xs[lat[:, 0]], ys[lat[:, 1]], zs[lat[:, 2]]], axis=1)

    def vid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ci, cj, ck = (a.transpose(2, 1, 0).ravel() for a in (ci, cj, ck))
    ncube = nx * ny * nz
    tet = np.empty((ncube, 6, 4), dtype=np.int64)
    for p, perm in enumerate(_PERMS):
        off = np.zeros((ncube, 3), dtype=np.int64)
        corners = [off.copy()]
        for ax in perm:
            off = off.copy()
            off[:, ax] += 1
            corners.append(off)
        for v in range(4):
            tet[:, p, v] = vid(ci + corners[v][:, 0], cj + corners[v][:, 1], ck + corners[v][:, 2])
    tet = tet.reshape(-1, 4)
    K = tet.shape[0]
    tags = np.zeros((K, 4), dtype=np.int8)
    ext = np.array([nx, ny, nz])
    for f in range(4):
        pts = lat[tet[:, [v for v in range(4) if v != f]]]
        on = np.zeros(K, dtype=bool)
        for ax in range(3):
            c = pts[:, :, ax]
            on |= np.all(c == 0, axis=1) | np.all(c == ext[ax], axis=1)
        tags[on, f] = boundary_tag
    return xyz, tet, tags


def refined_cube_mesh(n: int, r: int, boundary_tag: int = TAG_IMPEDANCE):
    """[0,1]^3 with n uniform cells per axis, the middle cell of every axis
    split into r: a small central region of cells r times finer (and slabs of
    thin elements through it), the rest at spacing 1/n."""
    if n < 1 or r < 1:
        raise ValueError("n, r must be >= 1")
    c = n // 2
    axis = np.concatenate([np.arange(c) / n, (c + np.arange(r) / r) / n, np.arange(c + 1, n + 1) / n])
    return graded_cube_mesh(axis, axis, axis, boundary_tag)


def boundary_tags(lat: np.ndarray, tet: np.ndarray, n: int, boundary_tag: int) -> np.ndarray:
    """Tag faces whose three vertices lie on one side of the cube's boundary."""
    K = tet.shape[0]
    tags = np.zeros((K, 4), dtype=np.int8)
    for f in range(4):
        others = [v for v in range(4) if v != f]
        pts = lat[tet[:, others]]  # [K,3 verts,3 coords]
        on = np.zeros(K, dtype=bool)
        for ax in range(3):
            c = pts[:, :, ax]
            on |= np.all(c == 0, axis=1) | np.all(c == n, axis=1)
        tags[on, f] = boundary_tag
    return tags


def tet_centroid_lattice4(lat_xyz_times_n: np.ndarray, tet: np.ndarray) -> np.ndarray:
    """4 n * centroid as exact integers (sum of lattice coordinates)."""
    return lat_xyz_times_n[tet].sum(axis=1)


def gaussian_current(nodes: np.ndarray, centre, width: float, pol: int) -> np.ndarray:
    """Nodal samples of j(x) = e_pol exp(-|x-centre|^2/width^2).

    ``nodes`` is [K, Np, 3]; returns j_re [K, Np, 3] (j_im = 0).
    """
    d2 = np.sum((nodes - np.asarray(centre, dtype=np.float64)) ** 2, axis=-1)
    j = np.zeros(nodes.shape, dtype=np.float64)
    j[..., pol] = np.exp(-d2 / (width * width))
    return j


@dataclass
class Workload:
    """A seeded problem description (mesh + coefficients + source recipe)."""
    name: str
    n: int
    q: int
    omega: float
    eps: np.ndarray          # [K]
    mu: np.ndarray           # [K]
    sigma: np.ndarray        # [K]
    centre: np.ndarray       # [3]
    width: float
    pol: int
    boundary_tag: int = TAG_IMPEDANCE
    xyz: np.ndarray = field(default=None, repr=False)
    tet: np.ndarray = field(default=None, repr=False)
    tags: np.ndarray = field(default=None, repr=False)

    @property
    def K(self) -> int:
        return self.tet.shape[0]


def _mesh(n, boundary_tag):
    return cube_mesh(n, boundary_tag)


def plain_fp64(n: int = 6, q: int = 1, boundary_tag: int = TAG_IMPEDANCE) -> Workload:
    """Unit cube, eps=mu=1, omega=2 pi, Gaussian e_z source width 0.1 at the centre.

    n=6, q=1 is the 1296-tet plain FP64 configuration."""
    xyz, tet, tags = _mesh(n, boundary_tag)
    K = tet.shape[0]
    return Workload("plain_fp64", n, q, 2 * math.pi, np.ones(K), np.ones(K), np.zeros(K),
                    np.array([0.5, 0.5, 0.5]), 0.1, 2, boundary_tag, xyz, tet, tags)


def large_single(n: int = 20, q: int = 3, seed: int = 2, boundary_tag: int = TAG_IMPEDANCE) -> Workload:
    """eps per cube from {1,2,4} (seeded), omega = 4 pi, Gaussian width 0.05 at a
    seeded point of [0.3,0.7]^3, e_z polarisation.  n=20, q=3 is the
    48000-tet P3 FP32-vs-FP64 configuration; boundary_tag = TAG_PEC makes the
    same medium a closed cavity (no dissipation through the walls)."""
    rng = np.random.default_rng(seed)
    eps_cube = np.array([1.0, 2.0, 4.0])[rng.integers(0, 3, n ** 3)]
    centre = rng.uniform(0.3, 0.7, 3)
    xyz, tet, tags = _mesh(n, boundary_tag)
    K = tet.shape[0]
    eps = np.repeat(eps_cube, 6)
    return Workload("large_single", n, q, 4 * math.pi, eps, np.ones(K), np.zeros(K),
                    centre, 0.05, 2, boundary_tag, xyz, tet, tags)


def batched_members(n: int = 12, q: int = 2, B: int = 64, seed: int = 3):
    """Per-member (omega, centre, polarisation) for the batched configuration
    (10368-tet P2 mesh at n=12, eps=mu=1, width 0.1)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(B):
        omega = rng.uniform(2 * math.pi, 6 * math.pi)
        centre = rng.uniform(0.2, 0.8, 3)
        pol = int(rng.integers(0, 3))
        out.append((omega, centre, pol))
    xyz, tet, tags = _mesh(n, TAG_IMPEDANCE)
    K = tet.shape[0]
    members = [Workload(f"batched_{b}", n, q, om, np.ones(K), np.ones(K), np.zeros(K),
                        c, 0.1, p, TAG_IMPEDANCE, xyz, tet, tags)
               for b, (om, c, p) in enumerate(out)]
    return members


def serving_stream(n_requests: int = 2000, rate: float = 20.0, seed: int = 4,
                   sizes=(8, 12, 16, 24), orders=(1, 2, 3)):
    """Poisson arrival stream of request recipes (no meshes built here)."""
    rng = np.random.default_rng(seed)
    reqs = []
    t = 0.0
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate)
        n = int(sizes[rng.integers(0, len(sizes))])
        q = int(orders[rng.integers(0, len(orders))])
        omega = rng.uniform(2 * math.pi, 8 * math.pi)
        centre = rng.uniform(0.2, 0.8, 3)
        pol = int(rng.integers(0, 3))
        sub = int(rng.integers(0, 2 ** 31))
        reqs.append(dict(id=r, arrival=t, n=n, q=q, omega=omega, centre=centre, pol=pol,
                         width=0.1, subseed=sub))
    return reqs


def serving_request_workload(req) -> Workload:
    rng = np.random.default_rng(req["subseed"])
    n = req["n"]
    eps_cube = np.array([1.0, 2.0, 4.0])[rng.integers(0, 3, n ** 3)]
    xyz, tet, tags = _mesh(n, TAG_IMPEDANCE)
    K = tet.shape[0]
    return Workload(f"req_{req['id']}", n, req["q"], req["omega"], np.repeat(eps_cube, 6),
                    np.ones(K), np.zeros(K), np.asarray(req["centre"]), req["width"],
                    req["pol"], TAG_IMPEDANCE, xyz, tet, tags)


def scatterer(n: int = 64, q: int = 2) -> Workload:
    """Dielectric sphere eps=4 (radius 0.25 at the centre; a tet is inside when
    its centroid is strictly inside), background eps=mu=1, omega = 8 pi,
    Gaussian e_z source at (0.15,0.5,0.5) width 0.03."""
    xyz, tet, tags = _mesh(n, TAG_IMPEDANCE)
    lat = np.rint(xyz * n).astype(np.int64)
    c4 = lat[tet].sum(axis=1)  # = 4 n centroid, exact
    d = c4 - 2 * n  # 4n (centroid - 1/2)
    inside = np.sum(d * d, axis=1) < (n * n)  # |4n(c-1/2)|^2 < (4n/4)^2
    K = tet.shape[0]
    eps = np.where(inside, 4.0, 1.0)
    return Workload("scatterer", n, q, 8 * math.pi, eps, np.ones(K), np.zeros(K),
                    np.array([0.15, 0.5, 0.5]), 0.03, 2, TAG_IMPEDANCE, xyz, tet, tags)


# ------------------------------------------------------------------ 2-D (TM)
#
# The paper's own experiments are two-dimensional (Section 6).  An "nx x ny
# Cartesian mesh" of a rectangle is the grid of nx x ny cells, each divided
# into four triangles by joining its corners to its barycentre.  Triangles are
# counter-clockwise; local edge f is opposite local vertex f; the barycentre is
# local vertex 0, so edge 0 is the cell side.  Cell c = i + nx j (x fastest)
# holds triangles 4c .. 4c+3 for its bottom, right, top and left sides.

SIDE_BOTTOM, SIDE_RIGHT, SIDE_TOP, SIDE_LEFT = range(4)


def cartesian_triangles(nx: int, ny: int, x0: float = 0.0, y0: float = 0.0, lx: float = 1.0,
                        ly: float = 1.0, side_tags=(TAG_IMPEDANCE,) * 4):
    """Returns (xy [nv,2] float64, tri [4 nx ny, 3] int64, edge_tag [K,3] int8);
    side_tags gives the tag of the bottom, right, top and left sides."""
    if nx < 1 or ny < 1:
        raise ValueError("nx, ny must be >= 1")
    gi, gj = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="xy")
    corners = np.stack([x0 + lx * gi.ravel() / nx, y0 + ly * gj.ravel() / ny], axis=1)
    ci, cj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    ci, cj = ci.ravel(), cj.ravel()
    centres = np.stack([x0 + lx * (ci + 0.5) / nx, y0 + ly * (cj + 0.5) / ny], axis=1)
    xy = np.concatenate([corners, centres])
    ncorner = corners.shape[0]

    def vid(i, j):
        return i + (nx + 1) * j

    p0, p1, p2, p3 = vid(ci, cj), vid(ci + 1, cj), vid(ci + 1, cj + 1), vid(ci, cj + 1)
    c = ncorner + np.arange(nx * ny)
    tri = np.stack([np.stack([c, p0, p1], 1), np.stack([c, p1, p2], 1),
                    np.stack([c, p2, p3], 1), np.stack([c, p3, p0], 1)], axis=1).reshape(-1, 3)
    tags = np.zeros((tri.shape[0], 3), dtype=np.int8)
    side = np.tile(np.arange(4), nx * ny)
    on = np.stack([cj == 0, ci == nx - 1, cj == ny - 1, ci == 0], axis=1)  # [cells, side]
    on = on.reshape(-1)
    tags[on, 0] = np.asarray(side_tags, dtype=np.int8)[side[on]]
    return xy, tri.astype(np.int64), tags


@dataclass
class Workload2D:
    """A 2-D TM problem: mesh, coefficients and the recipe of its data.

    source kinds: "constant" (j = 1), "gaussian" (j = exp(-|x-c|^2/s^2)),
    "planewave" (impedance data of the plane wave exp(i omega d.x),
    d = (cos theta, sin theta)), "none"."""
    name: str
    q: int
    omega: float
    eps: np.ndarray
    mu: np.ndarray
    sigma: np.ndarray
    xy: np.ndarray = field(repr=False)
    tri: np.ndarray = field(repr=False)
    tags: np.ndarray = field(repr=False)
    source: str = "none"
    centre: np.ndarray = None
    width: float = 0.0
    theta: float = 0.0

    @property
    def K(self) -> int:
        return self.tri.shape[0]


def cavity2d(n: int = 32, q: int = 1, omega_r: float = 3 * math.sqrt(2) * math.pi,
             delta: float = 1.0 / 8.0) -> Workload2D:
    """Closed PEC cavity (0,1)^2 on an n x n Cartesian mesh, eps = mu = 1,
    j = 1, omega = omega_r + sqrt(2) pi delta (the cavity experiment)."""
    xy, tri, tags = cartesian_triangles(n, n, side_tags=(TAG_PEC,) * 4)
    K = tri.shape[0]
    om = omega_r + math.sqrt(2) * math.pi * delta
    return Workload2D(f"cavity2d_n{n}_q{q}", q, om, np.ones(K), np.ones(K), np.zeros(K), xy, tri, tags,
                      "constant")


def planewave2d(n: int = 32, q: int = 1, omega: float = 10 * math.pi,
                theta: float = math.pi / 4) -> Workload2D:
    """Plane wave in (0,1)^2 with impedance walls on every side, eps = mu = 1,
    j = 0, on an n x n Cartesian mesh (the free-space experiment)."""
    xy, tri, tags = cartesian_triangles(n, n, side_tags=(TAG_IMPEDANCE,) * 4)
    K = tri.shape[0]
    return Workload2D(f"planewave2d_n{n}_q{q}", q, omega, np.ones(K), np.ones(K), np.zeros(K), xy, tri,
                      tags, "planewave", theta=theta)


def trap2d(n: int = 30, q: int = 3, shape: str = "square") -> Workload2D:
    """Dipole in a trapping body G inside Omega = (-1,1)^2 with impedance
    walls: eps = 4 in G (a triangle is inside when its centroid is), else 1,
    mu = 1, j = exp(-|x-c|^2/s^2) with s = 0.05.
      shape "square": G = [-1/2,1/2]^2, c = (1/4, 0), omega = 10 pi;
      shape "disk":   G = {|x| < 1/2}, c = (sqrt2/4, 1/2 - sqrt2/4), omega = 20 pi.
    The paper meshes these with GMSH (3636 and 22294 triangles); the n x n
    Cartesian mesh of (-1,1)^2 stands in for them (n = 30: 3600 triangles,
    n = 75: 22500)."""
    xy, tri, tags = cartesian_triangles(n, n, -1.0, -1.0, 2.0, 2.0)
    K = tri.shape[0]
    cen = xy[tri].mean(axis=1)
    if shape == "square":
        inside = np.all(np.abs(cen) < 0.5, axis=1)
        c, om = np.array([0.25, 0.0]), 10 * math.pi
    elif shape == "disk":
        inside = np.sum(cen * cen, axis=1) < 0.25
        c, om = np.array([math.sqrt(2) / 4, 0.5 - math.sqrt(2) / 4]), 20 * math.pi
    else:
        raise ValueError("shape must be 'square' or 'disk'")
    return Workload2D(f"trap2d_{shape}_n{n}_q{q}", q, om, np.where(inside, 4.0, 1.0), np.ones(K), np.zeros(K),
                      xy, tri, tags, "gaussian", centre=c, width=0.05)


def waveguide2d(nx: int = 64, q: int = 1, omega: float = 2 * math.pi, theta: float = math.pi / 6) -> Workload2D:
    """Half-open waveguide (0,4) x (0,1) on an nx x nx/4 Cartesian mesh: PEC on
    the bottom, top and left sides, impedance wall on the right with the data
    of the plane wave exp(i omega d.x), d = (cos theta, sin theta); eps = mu =
    1, j = 0 (the waveguide experiment)."""
    xy, tri, tags = cartesian_triangles(nx, nx // 4, 0.0, 0.0, 4.0, 1.0,
                                        side_tags=(TAG_PEC, TAG_IMPEDANCE, TAG_PEC, TAG_PEC))
    K = tri.shape[0]
    return Workload2D(f"waveguide2d_n{nx}_q{q}", q, omega, np.ones(K), np.ones(K), np.zeros(K), xy, tri, tags,
                      "wallwave", theta=theta)


def current_2d(w: Workload2D, nodes: np.ndarray) -> np.ndarray | None:
    """Nodal samples of the current density j at nodes [K, Np, 2] (real), or
    None for sources without a current."""
    if w.source == "constant":
        return np.ones(nodes.shape[:2])
    if w.source == "gaussian":
        d2 = np.sum((nodes - w.centre) ** 2, axis=-1)
        return np.exp(-d2 / (w.width * w.width))
    return None


SIDE_NORMALS = np.array([[0.0, -1.0], [1.0, 0.0], [0.0, 1.0], [-1.0, 0.0]])


def _wall_data(w: Workload2D, face_points: np.ndarray, fn, project: bool) -> np.ndarray:
    """fn(points [..., 2], outward normal [2]) on the impedance edges (edge 0
    of wall cells; the normal is that of the cell side), sampled at the edge
    nodes or L2-projected onto polynomials of degree Nfp - 1 on each edge
    (Gauss-Legendre, 16 points): [K, 3, Nfp] complex, zero elsewhere."""
    assert face_points.shape[0] == w.K
    out = np.zeros(face_points.shape[:3], dtype=np.complex128)
    wall = np.nonzero(w.tags[:, 0] == TAG_IMPEDANCE)[0]
    pts = face_points[wall, 0]                            # [nw, Nfp, 2]
    Nfp = pts.shape[1]
    if not project:
        for i, e in enumerate(wall):
            out[e, 0] = fn(pts[i], SIDE_NORMALS[e % 4])
        return out
    A = w.xy[w.tri[wall, 1]]
    B = w.xy[w.tri[wall, 2]]
    sg, wg = np.polynomial.legendre.leggauss(16)
    sg, wg = (sg + 1) / 2, wg / 2
    L2 = np.sum((B - A) ** 2, axis=1)
    s_nodes = np.einsum("wkc,wc->wk", pts - A[:, None, :], B - A) / L2[:, None]   # node positions on [0,1]
    for i, e in enumerate(wall):
        lag = np.ones((len(sg), Nfp))
        for k in range(Nfp):
            for l in range(Nfp):
                if l != k:
                    lag[:, k] *= (sg - s_nodes[i, l]) / (s_nodes[i, k] - s_nodes[i, l])
        G = fn(A[i] + sg[:, None] * (B[i] - A[i]), SIDE_NORMALS[e % 4])
        out[e, 0] = np.linalg.solve(lag.T @ (wg[:, None] * lag), lag.T @ (wg * G))
    return out


def planewave_boundary_data(w: Workload2D, face_points: np.ndarray, project: bool = True) -> np.ndarray:
    """Impedance data G = e + Z h x n of the plane wave e = exp(i omega d.x),
    h = (sin theta, -cos theta) e, Z = 1 (so G = e (1 + d.n)), on the wall
    edges of a Cartesian mesh; [K, 3, Nfp] complex nodal values at the edge
    nodes face_points [K, 3, Nfp, 2], zero off the impedance edges.
    project=True returns the L2 projection on each edge (exact edge integrals
    of the data against the edge basis), project=False samples the nodes."""
    d = np.array([math.cos(w.theta), math.sin(w.theta)])
    return _wall_data(w, face_points, lambda x, n: np.exp(1j * w.omega * (x @ d)) * (1.0 + n @ d), project)


def waveguide_boundary_data(w: Workload2D, face_points: np.ndarray, project: bool = True) -> np.ndarray:
    """Impedance data of the waveguide's right wall: the printed data xi =
    exp(i omega d.x) is read as the Robin data of d_n e + i omega e, so the
    first-order data is G = xi / (i omega) (see planewave_boundary_data for
    the layout and `project`)."""
    d = np.array([math.cos(w.theta), math.sin(w.theta)])
    return _wall_data(w, face_points, lambda x, n: np.exp(1j * w.omega * (x @ d)) / (1j * w.omega), project)
