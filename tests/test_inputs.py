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
