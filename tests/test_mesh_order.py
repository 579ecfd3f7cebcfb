"""Locality order of elements (host-only library call, no GPU): it is a
permutation, it sorts centroids by their Morton key (checked against a
bit-by-bit interleave written here), and on a randomly numbered mesh it
brings face neighbours close in index again."""
import numpy as np
import pytest

from paper_2106_02858_amd import inputs


@pytest.fixture
def lib():
    """The library's host-only entry points need no GPU."""
    from paper_2106_02858_amd import cmcg
    return cmcg


def morton_key(c, lo, sc):
    """Bit-by-bit interleave of the 21-bit cell coordinates (x in bit 0)."""
    cell = [int((c[d] - lo[d]) * sc) for d in range(3)]
    k = 0
    for b in range(21):
        for d in range(3):
            k |= ((cell[d] >> b) & 1) << (3 * b + d)
    return k


def neighbour_spread(tet):
    """Mean |i - j| over pairs of elements sharing a face."""
    faces = {}
    for e, t in enumerate(tet):
        for f in range(4):
            key = tuple(sorted(np.delete(t, f)))
            faces.setdefault(key, []).append(e)
    d = [abs(a - b) for v in faces.values() if len(v) == 2 for a, b in [v]]
    return float(np.mean(d))


def test_locality_order_is_morton_sort(lib):
    xyz, tet, _ = inputs.cube_mesh(4)
    rng = np.random.default_rng(5)
    tet = tet[rng.permutation(tet.shape[0])]
    order = lib.cmcg_mesh_locality_order(xyz, tet)
    assert np.array_equal(np.sort(order), np.arange(tet.shape[0]))
    c = xyz[tet].mean(axis=1)
    lo, hi = c.min(axis=0), c.max(axis=0)
    sc = ((1 << 21) - 1) / np.max(hi - lo)
    keys = [morton_key(c[e], lo, sc) for e in order]
    assert all(a <= b for a, b in zip(keys, keys[1:]))


def test_locality_order_restores_neighbour_locality(lib):
    xyz, tet, _ = inputs.cube_mesh(6)
    rng = np.random.default_rng(6)
    shuffled = tet[rng.permutation(tet.shape[0])]
    order = lib.cmcg_mesh_locality_order(xyz, shuffled)
    s_rand, s_cube, s_morton = neighbour_spread(shuffled), neighbour_spread(tet), neighbour_spread(shuffled[order])
    print(f"mean neighbour index distance: random {s_rand:.0f}, cube order {s_cube:.0f}, Morton {s_morton:.0f}")
    assert s_morton < 0.15 * s_rand and s_morton < 1.5 * s_cube


def test_locality_order_errors(lib):
    xyz, tet, _ = inputs.cube_mesh(1)
    bad = tet.copy()
    bad[0, 0] = xyz.shape[0]
    with pytest.raises(lib.CmcgError) as e:
        lib.cmcg_mesh_locality_order(xyz, bad)
    assert e.value.code == lib.CMCG_ERR_ARG
    x2 = xyz.copy()
    x2[0, 0] = np.nan
    with pytest.raises(lib.CmcgError) as e:
        lib.cmcg_mesh_locality_order(x2, tet)
    assert e.value.code == lib.CMCG_ERR_ARG
