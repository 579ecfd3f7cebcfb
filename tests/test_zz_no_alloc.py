"""The allocation-free inner product (cmcg_debug_dot_noalloc) against the
allocating one (cmcg_debug_dot): same kernels and summation order, so the
values agree bit for bit.  Two calls in a row, the second on a smaller
problem (the fixed scratch array keeps the first call's partials and must not
leak them into the second), on tetrahedra and triangles, through the C-ABI."""
import numpy as np
import pytest

from paper_2106_02858_amd import inputs

pytestmark = pytest.mark.gpu


def dev(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def problem3d(lib, n, q, seed):
    xyz, tet, tags = inputs.cube_mesh(n)
    K = tet.shape[0]
    rng = np.random.default_rng(seed)
    m = lib.cmcg_mesh_create(xyz, tet, tags)
    s = lib.cmcg_space_create(m, q, lib.CMCG_FP64)
    p = lib.cmcg_problem_create(s, rng.choice([1.0, 2.0, 4.0], K), rng.choice([1.0, 1.5], K), None, 2 * np.pi,
                                None)
    return p, (K, 6, lib.cmcg_space_info(s)["Np"])


def problem2d(lib, n, q, seed):
    xy, tri, tags = inputs.cartesian_triangles(n, n)
    K = tri.shape[0]
    rng = np.random.default_rng(seed)
    m = lib.cmcg_mesh2d_create(xy, tri, tags)
    s = lib.cmcg_space_create(m, q, lib.CMCG_FP64)
    p = lib.cmcg_problem_create(s, rng.choice([1.0, 4.0], K), np.ones(K), None, 2 * np.pi, None)
    return p, (K, 3, lib.cmcg_space_info(s)["Np"])


@pytest.mark.parametrize("dim", [3, 2])
def test_noalloc_dot_equals_allocating_dot(lib, dim):
    import torch
    make = problem3d if dim == 3 else problem2d
    # first a large problem (1024 partials for 3-D: 6 K > 1024 x 256 rows),
    # then a small one that writes fewer partials than the first left behind
    sizes = ((24, 2), (2, 3)) if dim == 3 else ((40, 3), (3, 1))
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    for call, (n, q) in enumerate(sizes):
        p, shape = make(lib, n, q, seed=call)
        rng = np.random.default_rng(10 + call)
        U, V = dev(rng.standard_normal(shape)), dev(rng.standard_normal(shape))
        print(f"noalloc dot: dim={dim} call={call} shape={shape}", flush=True)
        lib.cmcg_debug_dot_noalloc(p, U, V, out[call:])
        torch.cuda.synchronize()
        ref = lib.cmcg_debug_dot(p, U, V)
        got = float(out[call].item())
        assert got == ref, (dim, call, got, ref)
        assert np.isfinite(got) and got != 0.0


def test_noalloc_dot_rejects_null_arguments(lib):
    import torch
    p, shape = problem3d(lib, 1, 1, 0)
    U = dev(np.zeros(shape))
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.CmcgError) as err:
        lib.cmcg_debug_dot_noalloc(p, U, None, out)
    assert err.value.code == lib.CMCG_ERR_ARG
