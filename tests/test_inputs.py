"""The seeded workload generators: mesh structure and sizes."""
import numpy as np

from paper_2106_02858_amd import inputs


def test_cube_mesh_counts_and_conformity():
    for n in (1, 2, 3):
        xyz, tet, tags = inputs.cube_mesh(n)
        assert tet.shape == (6 * n ** 3, 4)
        assert xyz.shape == ((n + 1) ** 3, 3)
        faces = {}
        for e in range(tet.shape[0]):
            for f in range(4):
                key = tuple(sorted(int(tet[e, a]) for a in range(4) if a != f))
                faces.setdefault(key, []).append((e, f))
        assert max(len(v) for v in faces.values()) == 2
        nb = sum(1 for v in faces.values() if len(v) == 1)
        assert nb == 12 * n * n  # 2 triangles per boundary square
        assert (tags > 0).sum() == nb
        # every tet has volume a^3 / 6
        v = xyz[tet]
        vol = np.abs(np.linalg.det(np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]], 2))) / 6
        assert np.allclose(vol, 1 / (6 * n ** 3))


def test_scatterer_sphere_count_exact():
    w = inputs.scatterer(64)
    assert w.K == 1572864
    assert int((w.eps == 4).sum()) == 103392


def test_large_single_seeded():
    a = inputs.large_single(n=4)
    b = inputs.large_single(n=4)
    assert np.array_equal(a.eps, b.eps) and np.array_equal(a.centre, b.centre)
    assert set(np.unique(a.eps)) <= {1.0, 2.0, 4.0}
    assert np.all((a.centre >= 0.3) & (a.centre <= 0.7))


def test_serving_stream():
    r = inputs.serving_stream(100)
    t = np.array([x["arrival"] for x in r])
    assert np.all(np.diff(t) > 0)
    assert {x["q"] for x in r} <= {1, 2, 3}


def test_cartesian_triangles_follow_the_paper_definition():
    """n x m cells, each cut into four counter-clockwise triangles through its
    barycentre; every wall edge is tagged with its side's tag and no other."""
    from paper_2106_02858_amd import inputs
    xy, tri, tags = inputs.cartesian_triangles(3, 2, 0.0, 0.0, 4.0, 1.0, side_tags=(1, 2, 1, 1))
    assert tri.shape == (24, 3) and xy.shape == (12 + 6, 2)
    v = xy[tri]
    area2 = (v[:, 1, 0] - v[:, 0, 0]) * (v[:, 2, 1] - v[:, 0, 1]) - (v[:, 1, 1] - v[:, 0, 1]) * (v[:, 2, 0] - v[:, 0, 0])
    assert np.all(area2 > 0) and abs(area2.sum() / 2 - 4.0) < 1e-14
    # vertex 0 is the cell barycentre; edge 0 (vertices 1, 2) is the cell side
    assert np.allclose(v[0::4, 0], v[:, 1].reshape(-1, 4, 2).mean(axis=1)) and np.all(tags[:, 1:] == 0)
    mid = 0.5 * (v[:, 1] + v[:, 2])
    side = np.arange(24) % 4
    on_wall = np.isclose(mid[:, 1], 0) | np.isclose(mid[:, 0], 4) | np.isclose(mid[:, 1], 1) | np.isclose(mid[:, 0], 0)
    on_wall &= (side == 0) & np.isclose(mid[:, 1], 0) | (side == 1) & np.isclose(mid[:, 0], 4) | \
        (side == 2) & np.isclose(mid[:, 1], 1) | (side == 3) & np.isclose(mid[:, 0], 0)
    assert np.array_equal(tags[:, 0] != 0, on_wall)
    assert np.all(tags[on_wall & (side == 1), 0] == 2) and np.all(tags[on_wall & (side != 1), 0] == 1)


def test_2d_workloads():
    import math
    from paper_2106_02858_amd import inputs
    w = inputs.cavity2d(32, 1, 3 * math.sqrt(2) * math.pi, 1 / 8)
    assert w.K == 4096 and abs(w.omega / (2 * math.pi) - 2.209707) < 1e-5   # the figure's data-file label
    assert np.all(w.tags[w.tags != 0] == inputs.TAG_PEC)
    d = inputs.trap2d(75, 3, "disk")
    cen = d.xy[d.tri].mean(axis=1)
    assert d.K == 22500 and np.array_equal(d.eps == 4.0, np.sum(cen ** 2, axis=1) < 0.25)
    assert abs(d.omega - 20 * math.pi) < 1e-12 and np.all(d.tags[d.tags != 0] == inputs.TAG_IMPEDANCE)
    g = inputs.waveguide2d(64, 1, 2 * math.pi)
    assert g.K == 64 * 16 * 4 and np.all(g.tags[g.tags[:, 0] == inputs.TAG_IMPEDANCE, 0] == inputs.TAG_IMPEDANCE)
    right = (np.arange(g.K) % 4 == 1) & (g.tags[:, 0] != 0)
    assert np.all(g.tags[right, 0] == inputs.TAG_IMPEDANCE) and np.all(g.tags[~right & (g.tags[:, 0] != 0), 0] == inputs.TAG_PEC)
