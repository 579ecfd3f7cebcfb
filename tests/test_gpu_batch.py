"""Batched solves (one launch per RK stage for all members): every member
equals the same problem solved alone, bit for bit (same per-member arithmetic
and reduction order), and matches the FP64 oracle at a fixed iteration
count."""
import math

import numpy as np
import pytest

from oracle import cmcg as ocmcg
from oracle import dg
from paper_2106_02858_amd import inputs
from tests._pairs import rel_norm_c

pytestmark = pytest.mark.gpu


def dev(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def filtered(lib, r, K, Np):
    import torch
    fr = torch.zeros((K, 6, Np), dtype=torch.float64, device="cuda")
    fi = torch.zeros_like(fr)
    lib.cmcg_result_filtered_device(r, fr, fi)
    return fr.cpu().numpy() + 1j * fi.cpu().numpy()


def initial(lib, r, K, Np):
    import torch
    u = torch.zeros((K, 6, Np), dtype=torch.float64, device="cuda")
    lib.cmcg_result_initial_device(r, u)
    return u.cpu().numpy()


def members(lib, n, q, precision, B, seed, hetero_eps=False):
    """B problems on one space: different omega, source centre and polarisation."""
    xyz, tet, tags = inputs.cube_mesh(n)
    K = tet.shape[0]
    m = lib.cmcg_mesh_create(xyz, tet, tags)
    s = lib.cmcg_space_create(m, q, precision)
    nodes = lib.cmcg_space_nodes(s)
    rng = np.random.default_rng(seed)
    probs, recipes = [], []
    for b in range(B):
        omega = rng.uniform(2 * math.pi, 6 * math.pi)
        centre = rng.uniform(0.3, 0.7, 3)
        pol = int(rng.integers(0, 3))
        eps = rng.choice([1.0, 2.0, 4.0], K) if hetero_eps else np.ones(K)
        j = inputs.gaussian_current(nodes, centre, 0.25, pol)
        probs.append(lib.cmcg_problem_create(s, eps, np.ones(K), None, omega, j))
        recipes.append((omega, centre, pol, eps))
    return s, probs, recipes, (xyz, tet, tags)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("q,n,hetero", [(1, 2, False), (2, 2, True), (3, 1, False)])
def test_batch_members_equal_single_solves(lib, q, n, precision, hetero):
    print(f"batch q={q} n={n} prec={precision} hetero={hetero}", flush=True)
    s, probs, _, _ = members(lib, n, q, precision, 4, seed=10 * q + precision, hetero_eps=hetero)
    info = lib.cmcg_space_info(s)
    K, Np = info["K"], info["Np"]
    o = lib.cmcg_options_default(tol=1e-8, max_iter=300)
    res = lib.cmcg_solve_batch(probs, o)
    steps = set()
    for p, r in zip(probs, res):
        single = lib.cmcg_solve(p, o)
        a, b = lib.cmcg_result_stats(r), lib.cmcg_result_stats(single)
        steps.add(a["steps"])
        assert a["iters"] == b["iters"] and a["periods"] == b["periods"] and a["steps"] == b["steps"]
        assert np.array_equal(lib.cmcg_result_history(r), lib.cmcg_result_history(single))
        assert np.array_equal(filtered(lib, r, K, Np), filtered(lib, single, K, Np))
        assert np.array_equal(initial(lib, r, K, Np), initial(lib, single, K, Np))
    assert len(steps) > 1  # members really had different periods


def test_batch_against_oracle(lib):
    s, probs, recipes, (xyz, tet, tags) = members(lib, 2, 2, 0, 3, seed=5)
    info = lib.cmcg_space_info(s)
    K, Np = info["K"], info["Np"]
    p0 = dg.make_problem(xyz, tet, tags, 2, np.ones(K), np.ones(K))
    iters = []
    refs = []
    for omega, centre, pol, eps in recipes:
        j = inputs.gaussian_current(p0.geo.x, centre, 0.25, pol)
        op = dg.make_problem(xyz, tet, tags, 2, eps, np.ones(K), omega=omega, j=j)
        refs.append((op, ocmcg.solve(op, tol=1e-8, max_iter=300)))
        iters.append(refs[-1][1].iters)
    # a fixed common count (the largest) keeps every member iterating
    o = lib.cmcg_options_default(fixed_iters=max(iters))
    res = lib.cmcg_solve_batch(probs, o)
    for (op, _), r in zip(refs, res):
        ref = ocmcg.solve(op, fixed_iters=max(iters))
        err = rel_norm_c(op, filtered(lib, r, K, Np), ref.F)
        print(f"batch member vs oracle: {err:.2e}", flush=True)
        assert err < 1e-11


def test_batch_rejects_different_spaces(lib):
    s1, p1, _, _ = members(lib, 1, 1, 0, 1, seed=1)
    s2, p2, _, _ = members(lib, 1, 1, 0, 1, seed=2)
    with pytest.raises(lib.CmcgError) as e:
        lib.cmcg_solve_batch([p1[0], p2[0]])
    assert e.value.code == lib.CMCG_ERR_ARG


def test_batch_rejects_more_members_than_the_grid_holds(lib):
    s, p, _, _ = members(lib, 1, 1, 0, 1, seed=3)
    with pytest.raises(lib.CmcgError) as e:
        lib.cmcg_solve_batch([p[0]] * 65536)
    assert e.value.code == lib.CMCG_ERR_ARG
