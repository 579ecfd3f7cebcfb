"""Edge cases of the GPU path: every ragged chunk size (1..10 elements in
the last 10-element chunk), a single-tetrahedron mesh, the zero-source
problem (whose periodic solution is zero), argument and state errors."""
import numpy as np
import pytest

from oracle import cmcg as ocmcg
from oracle import dg
from paper_2106_02858_amd import inputs
from tests._pairs import lib_problem, rel_norm_c

pytestmark = pytest.mark.gpu


def dev(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def first_elements(n_elem):
    """The first n_elem tetrahedra of the 2^3 x 6 cube mesh, retagged."""
    xyz, tet, tags = inputs.cube_mesh(2)
    tet = tet[:n_elem]
    used, inv = np.unique(tet.ravel(), return_inverse=True)
    tet = inv.reshape(-1, 4)
    xyz = xyz[used]
    # faces without a partner inside the subset become impedance faces
    keys = {}
    for e in range(n_elem):
        for f in range(4):
            keys.setdefault(tuple(sorted(np.delete(tet[e], f))), []).append((e, f))
    tags = np.zeros((n_elem, 4), dtype=np.int8)
    for owners in keys.values():
        if len(owners) == 1:
            tags[owners[0]] = inputs.TAG_IMPEDANCE
    return xyz, tet, tags


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("q", [1, 2, 3])
def test_every_ragged_chunk_size(lib, q, precision):
    tol = 1e-12 if precision == 0 else 1e-5
    for n_elem in list(range(1, 11)) + [11, 19, 21]:
        xyz, tet, tags = first_elements(n_elem)
        rng = np.random.default_rng(n_elem)
        K = tet.shape[0]
        eps = rng.choice([1.0, 2.0, 4.0], K)
        op = dg.make_problem(xyz, tet, tags, q, eps, np.ones(K), rng.uniform(0, 0.5, K), omega=3.0,
                             j=rng.standard_normal((K, (q + 1) * (q + 2) * (q + 3) // 6, 3)))
        s, lp = lib_problem(lib, op, precision, xyz, tet, tags)
        U = rng.standard_normal((K, 6, op.Np))
        out = dev(np.zeros_like(U))
        lib.cmcg_debug_rhs(lp, dev(U), out, t=0.3, with_source=True)
        ref = dg.phi(op, 0.3, U, with_source=True)
        err = np.max(np.abs(out.cpu().numpy() - ref)) / np.max(np.abs(ref))
        assert err < tol, (n_elem, err)


def test_single_tetrahedron_cmcg(lib):
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64)
    tet = np.array([[0, 1, 2, 3]])
    tags = np.full((1, 4), inputs.TAG_IMPEDANCE, dtype=np.int8)
    j = inputs.gaussian_current(dg.make_problem(xyz, tet, tags, 2, np.ones(1), np.ones(1)).geo.x,
                                (0.25, 0.25, 0.25), 0.5, 2)
    op = dg.make_problem(xyz, tet, tags, 2, np.ones(1), np.ones(1), omega=2 * np.pi, j=j)
    ref = ocmcg.solve(op, tol=1e-10, max_iter=200)
    s, lp = lib_problem(lib, op, 0, xyz, tet, tags)
    r = lib.cmcg_solve(lp, lib.cmcg_options_default(fixed_iters=ref.iters))
    import torch
    fr = torch.zeros((1, 6, op.Np), dtype=torch.float64, device="cuda")
    fi = torch.zeros_like(fr)
    lib.cmcg_result_filtered_device(r, fr, fi)
    got = fr.cpu().numpy() + 1j * fi.cpu().numpy()
    ref_f = ocmcg.solve(op, fixed_iters=ref.iters).F
    assert rel_norm_c(op, got, ref_f) < 1e-11


@pytest.mark.parametrize("precision", [0, 1])
def test_zero_source_gives_zero_field(lib, precision):
    xyz, tet, tags = inputs.cube_mesh(2)
    m = lib.cmcg_mesh_create(xyz, tet, tags)
    s = lib.cmcg_space_create(m, 2, precision)
    K = tet.shape[0]
    p = lib.cmcg_problem_create(s, np.ones(K), np.ones(K), None, 2 * np.pi, None)
    r = lib.cmcg_solve(p, lib.cmcg_options_default(tol=1e-8))
    st = lib.cmcg_result_stats(r)
    assert st["iters"] == 0 and st["status"] == lib.CMCG_OK and st["rel_res"] == 0.0
    import torch
    fr = torch.ones((K, 6, 10), dtype=torch.float64, device="cuda")
    fi = torch.ones_like(fr)
    lib.cmcg_result_filtered_device(r, fr, fi)
    assert float(fr.abs().max()) == 0.0 and float(fi.abs().max()) == 0.0


def test_argument_errors(lib):
    xyz, tet, tags = inputs.cube_mesh(1)
    m = lib.cmcg_mesh_create(xyz, tet, tags)
    for q, prec in ((0, 0), (4, 0), (2, 7)):
        with pytest.raises(lib.CmcgError) as e:
            lib.cmcg_space_create(m, q, prec)
        assert e.value.code == lib.CMCG_ERR_ARG
    s = lib.cmcg_space_create(m, 1, 0)
    K = tet.shape[0]
    for eps, mu, omega in ((np.ones(K), np.ones(K), 0.0), (np.ones(K), np.ones(K), -1.0),
                           (np.zeros(K), np.ones(K), 1.0), (np.ones(K), -np.ones(K), 1.0)):
        with pytest.raises(lib.CmcgError) as e:
            lib.cmcg_problem_create(s, eps, mu, None, omega, None)
        assert e.value.code == lib.CMCG_ERR_ARG
    p = lib.cmcg_problem_create(s, np.ones(K), np.ones(K), None, 1.0, None)
    for kw in (dict(steps=2), dict(scheme=3), dict(flux=5)):
        with pytest.raises(lib.CmcgError) as e:
            lib.cmcg_solve(p, lib.cmcg_options_default(**kw))
        assert e.value.code == lib.CMCG_ERR_ARG, kw
    with pytest.raises(lib.CmcgError) as e:
        lib.cmcg_tune_stage(2, 1, 99)
    assert e.value.code == lib.CMCG_ERR_ARG


def test_engine_state_errors(lib):
    xyz, tet, tags = inputs.cube_mesh(1)
    m = lib.cmcg_mesh_create(xyz, tet, tags)
    s = lib.cmcg_space_create(m, 1, 1)
    K = tet.shape[0]
    j = inputs.gaussian_current(lib.cmcg_space_nodes(s), (0.5, 0.5, 0.5), 0.3, 2)
    p = lib.cmcg_problem_create(s, np.ones(K), np.ones(K), None, 2 * np.pi, j)
    e = lib.cmcg_engine_create(1 << 30, 2)
    with pytest.raises(lib.CmcgError) as err:
        lib.cmcg_engine_cancel(e, 0)            # free slot
    assert err.value.code == lib.CMCG_ERR_STATE
    with pytest.raises(lib.CmcgError) as err:
        lib.cmcg_engine_poll(e, 5)              # no such slot
    assert err.value.code == lib.CMCG_ERR_ARG
    slot = lib.cmcg_engine_admit(e, p)
    with pytest.raises(lib.CmcgError) as err:
        lib.cmcg_engine_collect(e, slot, p)     # still running
    assert err.value.code == lib.CMCG_ERR_STATE
    while lib.cmcg_engine_poll(e, slot) == 1:
        lib.cmcg_engine_step(e)
    r = lib.cmcg_engine_collect(e, slot, p)
    assert lib.cmcg_result_stats(r)["status"] in (lib.CMCG_OK, lib.CMCG_NOT_CONVERGED)
    with pytest.raises(lib.CmcgError) as err:
        lib.cmcg_engine_create(1 << 20, 0)
    assert err.value.code == lib.CMCG_ERR_ARG


def _small_problem(lib, precision=1, q=1, omega=2 * np.pi):
    xyz, tet, tags = inputs.cube_mesh(2)
    m = lib.cmcg_mesh_create(xyz, tet, tags)
    s = lib.cmcg_space_create(m, q, precision)
    K = tet.shape[0]
    j = inputs.gaussian_current(lib.cmcg_space_nodes(s), (0.5, 0.5, 0.5), 0.3, 2)
    return lib.cmcg_problem_create(s, np.ones(K), np.ones(K), None, omega, j), s


# Three steps over a period of 1000 time units: each step is thousands of
# times the stability limit, so the FP32 fields overflow within the first
# CG iteration.
UNSTABLE = dict(steps=3, max_iter=50)
SLOW = 2 * np.pi * 1e-3


def test_unstable_step_is_reported(lib):
    """A time step far above the stability limit (forced from the host: three
    steps per period) grows without bound: the solve reports the instability
    (non-finite values, or the CG breakdown they cause) instead of a result."""
    p, _ = _small_problem(lib, precision=1, omega=SLOW)
    with pytest.raises(lib.CmcgError) as e:
        lib.cmcg_solve(p, lib.cmcg_options_default(**UNSTABLE))
    assert e.value.code in (lib.CMCG_ERR_UNSTABLE, lib.CMCG_ERR_BREAKDOWN)


def test_non_finite_current_is_rejected(lib):
    xyz, tet, tags = inputs.cube_mesh(1)
    m = lib.cmcg_mesh_create(xyz, tet, tags)
    s = lib.cmcg_space_create(m, 1, 0)
    K = tet.shape[0]
    j = np.zeros((K, 4, 3))
    j[2, 1, 0] = np.inf
    with pytest.raises(lib.CmcgError) as e:
        lib.cmcg_problem_create(s, np.ones(K), np.ones(K), None, 1.0, j)
    assert e.value.code == lib.CMCG_ERR_ARG


def test_engine_failed_slot_does_not_disturb_others(lib):
    bad, _ = _small_problem(lib, precision=1, omega=SLOW)
    good, _ = _small_problem(lib, precision=1)
    e = lib.cmcg_engine_create(1 << 30, 4)
    sb = lib.cmcg_engine_admit(e, bad, lib.cmcg_options_default(**UNSTABLE))
    sg = lib.cmcg_engine_admit(e, good, lib.cmcg_options_default(tol=1e-6))
    while lib.cmcg_engine_poll(e, sb) == 1 or lib.cmcg_engine_poll(e, sg) == 1:
        lib.cmcg_engine_step(e)
    assert lib.cmcg_engine_poll(e, sb) == 3
    with pytest.raises(lib.CmcgError) as err:
        lib.cmcg_engine_collect(e, sb, bad)
    assert err.value.code in (lib.CMCG_ERR_UNSTABLE, lib.CMCG_ERR_BREAKDOWN)
    r = lib.cmcg_engine_collect(e, sg, good)
    alone = lib.cmcg_solve(good, lib.cmcg_options_default(tol=1e-6))
    assert lib.cmcg_result_stats(r)["iters"] == lib.cmcg_result_stats(alone)["iters"]
    assert lib.cmcg_engine_info(e)["used"] == 0


def test_solve_on_a_caller_stream(lib):
    import torch
    p, s = _small_problem(lib, precision=0, q=2)
    o = lib.cmcg_options_default(fixed_iters=5)
    st = torch.cuda.Stream()
    r1 = lib.cmcg_solve(p, o, stream=st)
    r0 = lib.cmcg_solve(p, o)
    info = lib.cmcg_space_info(s)
    out = [torch.zeros((info["K"], 6, info["Np"]), dtype=torch.float64, device="cuda") for _ in range(4)]
    lib.cmcg_result_filtered_device(r1, out[0], out[1], st)
    st.synchronize()
    lib.cmcg_result_filtered_device(r0, out[2], out[3])
    torch.cuda.synchronize()
    assert float(out[2].abs().max()) > 0
    assert torch.equal(out[0], out[2]) and torch.equal(out[1], out[3])


def _shuffled_mesh(n, seed):
    """cube_mesh(n) with a random element order, random vertex numbering,
    an orientation-preserving (even) permutation of every tetrahedron's
    vertices and a random mix of PEC and impedance boundary faces: element
    blocks then hold unrelated elements, so nearly every neighbour trace comes
    from another block."""
    xyz, tet, tags = inputs.cube_mesh(n)
    rng = np.random.default_rng(seed)
    K, nv = tet.shape[0], xyz.shape[0]
    tags = tags.copy()
    tags[(tags > 0) & (rng.random(tags.shape) < 0.4)] = inputs.TAG_PEC
    order = rng.permutation(K)
    tet, tags = tet[order], tags[order]
    vnew = rng.permutation(nv)
    xyz2 = np.empty_like(xyz)
    xyz2[vnew] = xyz
    tet = vnew[tet]
    even = [p for p in __import__("itertools").permutations(range(4))
            if sum(p[i] > p[j] for i in range(4) for j in range(i + 1, 4)) % 2 == 0]
    pick = rng.integers(0, len(even), K)
    sig = np.array(even)[pick]                      # new local vertex i = old local vertex sig[i]
    tet = np.take_along_axis(tet, sig, axis=1)
    tags = np.take_along_axis(tags, sig, axis=1)    # face i is opposite vertex i
    return xyz2, np.ascontiguousarray(tet), np.ascontiguousarray(tags)


@pytest.mark.parametrize("q,precision,v", [(1, 0, 0), (1, 1, 1), (2, 1, 3), (3, 1, 3), (3, 0, 1)])
def test_rhs_on_shuffled_mesh(lib, q, precision, v):
    print(f"shuffled mesh rhs q={q} prec={precision} variant={v}", flush=True)
    old = lib.cmcg_tune_get_stage(q, precision)
    lib.cmcg_tune_stage(q, precision, v)
    try:
        xyz, tet, tags = _shuffled_mesh(3, seed=50 + q)
        K = tet.shape[0]
        rng = np.random.default_rng(60 + q)
        eps = rng.choice([1.0, 2.0, 4.0], K)
        p0 = dg.make_problem(xyz, tet, tags, q, eps, np.ones(K))
        j = inputs.gaussian_current(p0.geo.x, (0.4, 0.5, 0.6), 0.3, 2)
        op = dg.make_problem(xyz, tet, tags, q, eps, np.ones(K), sigma=rng.uniform(0, 0.5, K), j=j)
        s, lp = lib_problem(lib, op, precision, xyz, tet, tags)
        import torch
        U = rng.standard_normal((K, 6, op.Np))
        out = torch.zeros((K, 6, op.Np), dtype=torch.float64, device="cuda")
        lib.cmcg_debug_rhs(lp, torch.tensor(U, device="cuda"), out, t=0.21, with_source=True)
        ref = dg.phi(op, 0.21, U, with_source=True)
        err = np.max(np.abs(out.cpu().numpy() - ref)) / np.max(np.abs(ref))
        print(f"  rel err {err:.2e}")
        assert err < (1e-12 if precision == 0 else 1e-5)
    finally:
        lib.cmcg_tune_stage(q, precision, old)


def test_cmcg_on_shuffled_mesh(lib):
    xyz, tet, tags = _shuffled_mesh(2, seed=71)
    K = tet.shape[0]
    p0 = dg.make_problem(xyz, tet, tags, 1, np.ones(K), np.ones(K))
    j = inputs.gaussian_current(p0.geo.x, (0.5, 0.5, 0.5), 0.3, 1)
    op = dg.make_problem(xyz, tet, tags, 1, np.ones(K), np.ones(K), j=j)
    s, lp = lib_problem(lib, op, 0, xyz, tet, tags)
    ref = ocmcg.solve(op, fixed_iters=4)
    r = lib.cmcg_solve(lp, lib.cmcg_options_default(fixed_iters=4))
    import torch
    fr = torch.zeros((K, 6, op.Np), dtype=torch.float64, device="cuda")
    fi = torch.zeros_like(fr)
    lib.cmcg_result_filtered_device(r, fr, fi)
    assert rel_norm_c(op, fr.cpu().numpy() + 1j * fi.cpu().numpy(), ref.F) < 1e-11


def test_concurrent_solves_from_two_threads(lib):
    """Two host threads solve different problems (different orders and
    precisions) at the same time, each on its own stream; each result equals
    the same solve run alone."""
    import threading
    import torch
    specs = [(1, 2), (0, 3), (1, 1)]
    probs = [_small_problem(lib, precision=p, q=q) for p, q in specs]
    o = lib.cmcg_options_default(fixed_iters=4)

    def fields(r, s):
        info = lib.cmcg_space_info(s)
        f = [torch.zeros((info["K"], 6, info["Np"]), dtype=torch.float64, device="cuda") for _ in range(2)]
        lib.cmcg_result_filtered_device(r, *f)
        torch.cuda.synchronize()
        return [x.cpu() for x in f]

    alone = [fields(lib.cmcg_solve(p, o), s) for p, s in probs]
    results, errors = [None] * len(probs), []

    def work(i):
        try:
            torch.cuda.set_device(0)
            st = torch.cuda.Stream()
            for _ in range(2):
                results[i] = lib.cmcg_solve(probs[i][0], o, stream=st)
            st.synchronize()
        except Exception as ex:  # reported below
            errors.append(ex)

    threads = [threading.Thread(target=work, args=(i,)) for i in range(len(probs))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not errors and all(not t.is_alive() for t in threads)
    for (p, s), r, a in zip(probs, results, alone):
        b = fields(r, s)
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_locality_reordered_mesh_gives_the_same_fields(lib):
    """Solving on the mesh renumbered by cmcg_mesh_locality_order (every
    per-element input permuted alike) gives the same fields, permuted."""
    import torch
    xyz, tet, tags = _shuffled_mesh(2, seed=81)
    K = tet.shape[0]
    order = lib.cmcg_mesh_locality_order(xyz, tet)
    rng = np.random.default_rng(82)
    eps = rng.choice([1.0, 2.0, 4.0], K)
    out = []
    for perm in (np.arange(K), order):
        m = lib.cmcg_mesh_create(xyz, np.ascontiguousarray(tet[perm]), np.ascontiguousarray(tags[perm]))
        s = lib.cmcg_space_create(m, 2, 0)
        j = inputs.gaussian_current(lib.cmcg_space_nodes(s), (0.4, 0.5, 0.5), 0.3, 0)
        p = lib.cmcg_problem_create(s, eps[perm], np.ones(K), None, 2 * np.pi, j)
        r = lib.cmcg_solve(p, lib.cmcg_options_default(fixed_iters=4))
        f = [torch.zeros((K, 6, 10), dtype=torch.float64, device="cuda") for _ in range(2)]
        lib.cmcg_result_filtered_device(r, *f)
        out.append(f[0].cpu().numpy() + 1j * f[1].cpu().numpy())
    a, b = out[0][order], out[1]
    assert np.max(np.abs(a - b)) <= 1e-11 * np.max(np.abs(a))
