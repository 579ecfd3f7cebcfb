"""The C-ABI library loads and exports every function include/cmcg.h
declares; host-side mesh validation reports its errors (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2106_02858_amd", "libcmcg.so")


def declared():
    src = open(os.path.join(ROOT, "include", "cmcg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w\s\*]*?\b(cmcg_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def so():
    if not os.path.exists(LIB):
        pytest.fail("libcmcg.so not built: run __graft_entry__.build()")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(so):
    names = declared()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(so, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2106_02858_amd import cmcg
    assert sorted(cmcg.EXPORTED) == declared()


def test_mesh_validation_host_only():
    from paper_2106_02858_amd import cmcg, inputs
    xyz, tet, tags = inputs.cube_mesh(2)
    m = cmcg.cmcg_mesh_create(xyz, tet, tags)
    info = cmcg.cmcg_mesh_info(m)
    assert info["K"] == 48 and info["n_boundary"] == 48
    assert abs(info["min_rho"] - 0.5 / (1 + np.sqrt(2))) < 1e-15
    # degenerate tetrahedron
    bad = tet.copy()
    bad[0, 1] = bad[0, 0] + 0  # repeated vertex
    with pytest.raises(cmcg.CmcgError) as e:
        cmcg.cmcg_mesh_create(xyz, bad, tags)
    assert e.value.code in (cmcg.CMCG_ERR_MESH,)
    # vertex index out of range
    bad = tet.copy()
    bad[3, 2] = xyz.shape[0]
    with pytest.raises(cmcg.CmcgError) as e:
        cmcg.cmcg_mesh_create(xyz, bad, tags)
    assert e.value.code == cmcg.CMCG_ERR_ARG
    # untagged boundary face
    t2 = tags.copy()
    t2[t2 > 0][:1] = 0
    b = np.argwhere(tags > 0)[0]
    t2[b[0], b[1]] = 0
    with pytest.raises(cmcg.CmcgError) as e:
        cmcg.cmcg_mesh_create(xyz, tet, t2)
    assert e.value.code == cmcg.CMCG_ERR_MESH
    # a face shared by three tetrahedra
    extra = np.concatenate([tet, tet[:1]], axis=0)
    with pytest.raises(cmcg.CmcgError) as e:
        cmcg.cmcg_mesh_create(xyz, extra, np.concatenate([tags, tags[:1]]))
    assert e.value.code == cmcg.CMCG_ERR_MESH


def test_options_defaults():
    from paper_2106_02858_amd import cmcg
    o = cmcg.cmcg_options_default()
    assert o.tol == 1e-8 and o.max_iter == 1000 and o.use_graph == 1 and o.fixed_iters == 0


def test_mesh_edge_cases_host_only():
    from paper_2106_02858_amd import cmcg
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64)
    tags = np.full((1, 4), cmcg.CMCG_TAG_IMPEDANCE, dtype=np.int8)
    # a single tetrahedron: every face on the boundary
    m = cmcg.cmcg_mesh_create(xyz, np.array([[0, 1, 2, 3]]), tags)
    info = cmcg.cmcg_mesh_info(m)
    assert info["K"] == 1 and info["n_boundary"] == 4
    # the same tetrahedron with negative orientation is accepted (vertices reordered)
    m2 = cmcg.cmcg_mesh_create(xyz, np.array([[1, 0, 2, 3]]), tags)
    assert abs(cmcg.cmcg_mesh_info(m2)["min_rho"] - info["min_rho"]) < 1e-15
    # empty mesh, too few vertices
    with pytest.raises(cmcg.CmcgError) as e:
        cmcg.cmcg_mesh_create(xyz, np.zeros((0, 4), dtype=np.int64), np.zeros((0, 4), dtype=np.int8))
    assert e.value.code == cmcg.CMCG_ERR_ARG
    with pytest.raises(cmcg.CmcgError) as e:
        cmcg.cmcg_mesh_create(xyz[:3], np.array([[0, 1, 2, 2]]), tags)
    assert e.value.code == cmcg.CMCG_ERR_ARG
    # coplanar vertices: zero volume
    flat = xyz.copy()
    flat[3] = [1, 1, 0]
    with pytest.raises(cmcg.CmcgError) as e:
        cmcg.cmcg_mesh_create(flat, np.array([[0, 1, 2, 3]]), tags)
    assert e.value.code == cmcg.CMCG_ERR_MESH


def test_c_program_links_against_the_library():
    """The plain-C demo (built with the library) resolves libcmcg through its
    rpath: the ABI is usable from C without Python."""
    import subprocess
    exe = os.path.join(os.path.dirname(__file__), "c_abi", "solve_demo")
    if not os.path.exists(exe):
        pytest.skip("library not built")
    out = subprocess.run(["ldd", exe], capture_output=True, text=True).stdout
    assert "libcmcg.so" in out and "not found" not in out


def test_mesh2d_validation_host_only():
    """2-D triangle meshes: counts, inscribed-circle diameters, orientation
    independence and the error paths (host only, no device work)."""
    from paper_2106_02858_amd import cmcg, inputs
    xy, tri, tags = inputs.cartesian_triangles(3, 2, side_tags=(1, 2, 1, 2))
    m = cmcg.cmcg_mesh2d_create(xy, tri, tags)
    assert cmcg.cmcg_mesh_dim(m) == 2
    info = cmcg.cmcg_mesh_info(m)
    assert info["K"] == 24 and info["n_boundary"] == 2 * (3 + 2)
    h = min(1 / 3, 1 / 2)   # cells 1/3 x 1/2: the smallest inscribed circle sits in the flattest triangles
    assert 0 < info["min_rho"] < h
    # clockwise triangles are accepted (normals are oriented by the opposite vertex)
    cw = tri[:, [0, 2, 1]]
    cw_tags = tags[:, [0, 2, 1]]
    assert cmcg.cmcg_mesh_info(cmcg.cmcg_mesh2d_create(xy, cw, cw_tags))["min_rho"] == info["min_rho"]
    bad = tri.copy()
    bad[0, 1] = bad[0, 0]
    with pytest.raises(cmcg.CmcgError) as e:
        cmcg.cmcg_mesh2d_create(xy, bad, tags)
    assert e.value.code == cmcg.CMCG_ERR_MESH
    bad = tri.copy()
    bad[2, 2] = xy.shape[0]
    with pytest.raises(cmcg.CmcgError) as e:
        cmcg.cmcg_mesh2d_create(xy, bad, tags)
    assert e.value.code == cmcg.CMCG_ERR_ARG
    t2 = tags.copy()
    b = np.argwhere(tags > 0)[0]
    t2[b[0], b[1]] = 0
    with pytest.raises(cmcg.CmcgError) as e:
        cmcg.cmcg_mesh2d_create(xy, tri, t2)
    assert e.value.code == cmcg.CMCG_ERR_MESH
    with pytest.raises(cmcg.CmcgError) as e:   # an edge shared by three triangles
        cmcg.cmcg_mesh2d_create(xy, np.concatenate([tri, tri[:1]]), np.concatenate([tags, tags[:1]]))
    assert e.value.code == cmcg.CMCG_ERR_MESH
    flat = xy.copy()
    flat[:, 1] = 0.0                                 # every triangle degenerate
    with pytest.raises(cmcg.CmcgError) as e:
        cmcg.cmcg_mesh2d_create(flat, tri, tags)
    assert e.value.code == cmcg.CMCG_ERR_MESH
    with pytest.raises(cmcg.CmcgError) as e:         # no triangles
        cmcg.cmcg_mesh2d_create(xy, tri[:0], tags[:0])
    assert e.value.code == cmcg.CMCG_ERR_ARG
    nan = xy.copy()
    nan[tri[0, 2], 1] = np.nan                       # a non-finite vertex
    with pytest.raises(cmcg.CmcgError) as e:
        cmcg.cmcg_mesh2d_create(nan, tri, tags)
    assert e.value.code == cmcg.CMCG_ERR_MESH


def test_default_stream_does_not_start_torch():
    """With no stream given and torch not yet on the device, the binding uses
    the default stream and leaves torch alone (starting torch after the library
    has loaded its own HIP runtime fails); in a fresh interpreter."""
    import subprocess
    import sys
    code = ("import sys; from paper_2106_02858_amd import cmcg; "
            "assert cmcg._stream(None) is None; assert 'torch' not in sys.modules; print('ok')")
    root = __import__("os").path.dirname(__import__("os").path.dirname(__import__("os").path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=root, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stderr


def test_stage_variant_by_launch_size_host_only():
    """The default stage variant of P2/P3 (-1) resolves by the launch's size
    (workgroups of 10 elements over all members); an explicit choice wins."""
    from paper_2106_02858_amd import cmcg
    FP64, FP32 = cmcg.CMCG_FP64, cmcg.CMCG_FP32
    assert cmcg.cmcg_tune_get_stage(3, FP32) == -1 and cmcg.cmcg_tune_get_stage(1, FP32) == 0
    r = cmcg.cmcg_tune_resolve_stage
    assert r(3, FP32, 3072) == 9 and r(3, FP32, 48000) == 6 and r(3, FP32, 384000) == 4
    assert r(3, FP32, 3072, 64) == 4                  # 64 members: a large launch
    assert r(2, FP32, 3072) == 9 and r(2, FP32, 24576) == 5 and r(2, FP32, 82944) == 4
    assert r(2, FP32, 1572864) == 3 and r(2, FP32, 10368, 64) == 3
    assert r(3, FP64, 48000) == 8 and r(3, FP64, 384000) == 4 and r(2, FP64, 3072) == 9
    assert r(2, FP64, 10368) == 8 and r(2, FP64, 48000) == 4 and r(1, FP32, 48000) == 0
    cmcg.cmcg_tune_stage(3, FP32, 5)
    try:
        assert r(3, FP32, 3072) == 5 and r(3, FP32, 384000) == 5
    finally:
        cmcg.cmcg_tune_stage(3, FP32, -1)
    with pytest.raises(cmcg.CmcgError):
        cmcg.cmcg_tune_stage(3, FP32, -2)
    with pytest.raises(cmcg.CmcgError):
        r(3, FP32, 0)
