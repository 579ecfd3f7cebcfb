"""GPU parity: the HIP library (through the C-ABI) against the FP64 oracle on
the same seeded inputs.

Tolerances: FP64 path -- single right-hand side 1e-12, one period 1e-12,
CMCG at a fixed iteration count 1e-11 (relative, eps-mu norm); FP32 fields
-- 1e-5 for one right-hand side / period (FP32 rounding of O(100)-term sums).
Meshes span several 10-element workgroups with a ragged last one.
"""
import numpy as np
import pytest

from oracle import cmcg as ocmcg
from oracle import dg, timestep
from paper_2106_02858_amd import inputs
from tests._pairs import lib_problem, pair, rel_norm, rel_norm_c, workload_pair

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}


def dev(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("q", [1, 2, 3])
def test_nodes_match_oracle(lib, q):
    op, s, lp = pair(lib, n=2, q=q)
    assert np.max(np.abs(lib.cmcg_space_nodes(s) - op.geo.x)) < 1e-15


@pytest.fixture
def variant(lib, request):
    """Run a test under one stage-kernel variant, restoring the default."""
    q, prec, v = request.param
    old = lib.cmcg_tune_get_stage(q, prec)
    lib.cmcg_tune_stage(q, prec, v)
    yield request.param
    lib.cmcg_tune_stage(q, prec, old)


# 0, 1 run everywhere; the matrix-core variants 2-5, 8 and 9 (4, 5: two waves per block;
# 5, 9: all faces' gathers at once; 8, 9: four waves per block) exist at q >= 2 in both field
# precisions (FP64 on v_mfma_f64_16x16x4f64), 6 and 7 (column split) at q = 3
VARIANTS = [(q, p, v) for q in (1, 2, 3) for p in (0, 1) for v in (0, 1)] + \
    [(q, p, v) for q in (2, 3) for p in (0, 1) for v in (2, 3, 4, 5, 8, 9)] + \
    [(3, p, v) for p in (0, 1) for v in (6, 7)]


@pytest.mark.parametrize("variant", VARIANTS, indirect=True, ids=lambda t: f"q{t[0]}-p{t[1]}-v{t[2]}")
def test_rhs_parity(lib, variant):
    q, precision, v = variant
    print(f"rhs q={q} prec={precision} variant={v}", flush=True)
    op, s, lp = pair(lib, n=2, q=q, precision=precision, seed=q, g=True)
    U = np.random.default_rng(1).standard_normal((op.K, 6, op.Np))
    out = dev(np.zeros_like(U))
    for t, src in ((0.0, False), (0.123, True)):
        lib.cmcg_debug_rhs(lp, dev(U), out, t=t, with_source=src)
        ref = dg.phi(op, t, U, with_source=src)
        err = np.max(np.abs(host(out) - ref)) / np.max(np.abs(ref))
        assert err < TOL[precision], (t, src, err)


LOCAL_SOURCE_ELEMENTS = (3, 4, 17, 45)  # 48 elements: blocks 0 and 4 mixed, 2 and 3 without source


@pytest.mark.parametrize("variant", VARIANTS, indirect=True, ids=lambda t: f"q{t[0]}-p{t[1]}-v{t[2]}")
def test_rhs_localised_source(lib, variant):
    """A current confined to four elements: element blocks without any source
    value skip the source arrays and blocks mix both kinds.  The right-hand
    side still equals the oracle's, and its source part is exactly zero in
    every element without current (and in every magnetic row)."""
    q, precision, v = variant
    print(f"localised source q={q} prec={precision} variant={v}", flush=True)
    xyz, tet, tags = inputs.cube_mesh(2)
    K = tet.shape[0]
    rng = np.random.default_rng(40 + q)
    Np = dg.make_problem(xyz, tet, tags, q, np.ones(K), np.ones(K)).geo.Np
    j = np.zeros((K, Np, 3), complex)
    for e in LOCAL_SOURCE_ELEMENTS:
        j[e] = rng.standard_normal((Np, 3)) + 1j * rng.standard_normal((Np, 3))
    eps = rng.choice([1.0, 2.0, 4.0], K)
    op = dg.make_problem(xyz, tet, tags, q, eps, np.ones(K), j=j)
    s, lp = lib_problem(lib, op, precision, xyz, tet, tags)
    U = rng.standard_normal((K, 6, Np))
    a, b = dev(np.zeros_like(U)), dev(np.zeros_like(U))
    t = 0.37
    lib.cmcg_debug_rhs(lp, dev(U), a, t=t, with_source=True)
    lib.cmcg_debug_rhs(lp, dev(U), b, t=t, with_source=False)
    ref = dg.phi(op, t, U, with_source=True)
    assert np.max(np.abs(host(a) - ref)) / np.max(np.abs(ref)) < TOL[precision]
    src, ref_src = host(a) - host(b), dg.source(op, t)
    off = np.ones(K, bool)
    off[list(LOCAL_SOURCE_ELEMENTS)] = False
    assert np.all(src[off] == 0) and np.all(src[:, 3:] == 0)
    # the difference of two right-hand sides carries their rounding (|B U| >> |J|)
    assert np.max(np.abs(src - ref_src)) / np.max(np.abs(ref_src)) < (1e-11 if precision == 0 else 1e-4)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("q", [1, 2, 3])
def test_rhs_centred_flux(lib, q, precision):
    op, s, lp = pair(lib, n=3 if q < 3 else 2, q=q, precision=precision, seed=7, alpha=0.0)
    U = np.random.default_rng(2).standard_normal((op.K, 6, op.Np))
    out = dev(np.zeros_like(U))
    o = lib.cmcg_options_default(flux=lib.CMCG_FLUX_CENTRED)
    lib.cmcg_debug_rhs(lp, dev(U), out, t=0.0, with_source=False, opts=o)
    ref = dg.apply_B(op, U)
    assert np.max(np.abs(host(out) - ref)) / np.max(np.abs(ref)) < TOL[precision]


@pytest.mark.parametrize("direction", [1, -1])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("q", [1, 2, 3])
def test_step_parity(lib, q, precision, direction):
    """One Runge-Kutta step (Section 5.3: RK2 for P1, RK4 otherwise) through
    cmcg_debug_step against the oracle's rk2_step / rk4_step, element by
    element: forward with the source at the stage times of step m, and the
    adjoint step S R S, on a mesh with PEC and impedance walls, boundary
    data, conductivity and a ragged last element block."""
    print(f"step q={q} prec={precision} dir={direction}", flush=True)
    op, s, lp = pair(lib, n=2, q=q, precision=precision, seed=20 + q, g=True)
    opts = lib.cmcg_options_default()
    M, dt = lib.cmcg_problem_steps(lp, opts)
    assert M == timestep.n_steps(op)
    m = M // 3
    U = np.random.default_rng(30 + q).standard_normal((op.K, 6, op.Np))
    out = dev(np.zeros_like(U))
    lib.cmcg_debug_step(lp, dev(U), out, m=m, direction=direction, with_source=direction > 0, opts=opts)
    step = timestep.rk2_step if q == 1 else timestep.rk4_step
    if direction > 0:
        ref = step(op, m * dt, U, dt, True)[0]
    else:
        ref = dg.flip_H(step(op, m * dt, dg.flip_H(U), dt, False)[0])
    err = np.max(np.abs(host(out) - ref)) / np.max(np.abs(ref))
    assert err < TOL[precision], err
    assert rel_norm(op, host(out), ref) < TOL[precision]


def test_step_arguments(lib):
    op, s, lp = pair(lib, n=1, q=1)
    U = dev(np.zeros((op.K, 6, op.Np)))
    M, _ = lib.cmcg_problem_steps(lp)
    for kw in (dict(m=-1), dict(m=M), dict(direction=0), dict(direction=-1, with_source=True)):
        with pytest.raises(lib.CmcgError) as err:
            lib.cmcg_debug_step(lp, U, U, **kw)
        assert err.value.code == lib.CMCG_ERR_ARG


@pytest.mark.parametrize("precision", [0, 1])
def test_device_problem_with_boundary_data_equals_host_problem(lib, precision):
    """cmcg_problem_create_device with j and g in device memory builds the
    same problem as the host-pointer form: equal right-hand sides bit for bit
    (and both equal the oracle's, boundary-data term included)."""
    import torch
    op, s, lp = pair(lib, n=2, q=2, precision=precision, seed=9, g=True)
    jd = [dev(np.real(op.j)), dev(np.imag(op.j))]
    gd = [dev(np.real(op.g)), dev(np.imag(op.g))]
    ld = lib.cmcg_problem_create_device(s, op.eps, op.mu, op.sigma, op.omega, jd[0], jd[1],
                                        g_re_dev=gd[0], g_im_dev=gd[1])
    U = dev(np.random.default_rng(3).standard_normal((op.K, 6, op.Np)))
    a, b = torch.empty_like(U), torch.empty_like(U)
    lib.cmcg_debug_rhs(lp, U, a, t=0.21, with_source=True)
    lib.cmcg_debug_rhs(ld, U, b, t=0.21, with_source=True)
    assert torch.equal(a, b)
    ref = dg.phi(op, 0.21, host(U), with_source=True)
    assert np.max(np.abs(host(b) - ref)) / np.max(np.abs(ref)) < TOL[precision]


@pytest.mark.parametrize("variant", VARIANTS, indirect=True, ids=lambda t: f"q{t[0]}-p{t[1]}-v{t[2]}")
def test_period_parity(lib, variant):
    q, precision, v = variant
    print(f"period q={q} prec={precision} variant={v}", flush=True)
    op, s, lp = pair(lib, n=2 if q < 3 else 1, q=q, precision=precision, seed=10 + q, sigma=False, g=(q == 2))
    M = timestep.n_steps(op)
    sch = timestep.default_scheme(q)
    M_lib, dt = lib.cmcg_problem_steps(lp)
    assert M_lib == M
    U0 = np.random.default_rng(3).standard_normal((op.K, 6, op.Np))
    ut = dev(np.zeros_like(U0))
    fr, fi = dev(np.zeros_like(U0)), dev(np.zeros_like(U0))
    for use_graph in (0, 1):
        o = lib.cmcg_options_default(use_graph=use_graph)
        # forward with source and filter
        lib.cmcg_debug_period(lp, dev(U0), ut, 1, True, fr, fi, opts=o)
        refU, refF = timestep.forward(op, U0, M, sch, True, filt=True)
        assert rel_norm(op, host(ut), refU) < TOL[precision]
        assert rel_norm_c(op, host(fr) + 1j * host(fi), refF) < TOL[precision]
        # backward (adjoint) without source
        lib.cmcg_debug_period(lp, dev(U0), ut, -1, False, opts=o)
        refB = timestep.backward(op, U0, M, sch)
        assert rel_norm(op, host(ut), refB) < TOL[precision]


@pytest.mark.parametrize("q", [1, 2, 3])
def test_dot_parity_and_determinism(lib, q):
    op, s, lp = pair(lib, n=3, q=q, seed=4)
    rng = np.random.default_rng(5)
    U = rng.standard_normal((op.K, 6, op.Np))
    V = rng.standard_normal((op.K, 6, op.Np))
    a = lib.cmcg_debug_dot(lp, dev(U), dev(V))
    b = lib.cmcg_debug_dot(lp, dev(U), dev(V))
    ref = dg.inner(op, U, V)
    assert a == b
    assert abs(a - ref) <= 1e-13 * dg.norm(op, U) * dg.norm(op, V)


@pytest.mark.parametrize("q", [1, 2, 3])
def test_adjoint_identity_on_gpu(lib, q):
    op, s, lp = pair(lib, n=2, q=q, seed=20 + q, sigma=True)
    rng = np.random.default_rng(q)
    x, y = rng.standard_normal((2, op.K, 6, op.Np))
    px, psy = dev(np.zeros_like(x)), dev(np.zeros_like(x))
    lib.cmcg_debug_period(lp, dev(x), px, 1, False)
    lib.cmcg_debug_period(lp, dev(y), psy, -1, False)
    lhs = lib.cmcg_debug_dot(lp, px, dev(y))
    rhs = lib.cmcg_debug_dot(lp, dev(x), psy)
    assert abs(lhs - rhs) <= 1e-13 * dg.norm(op, x) * dg.norm(op, y)


def _filtered(lib, r, op):
    fr, fi = dev(np.zeros((op.K, 6, op.Np))), dev(np.zeros((op.K, 6, op.Np)))
    lib.cmcg_result_filtered_device(r, fr, fi)
    return host(fr) + 1j * host(fi)


@pytest.mark.parametrize("q,n", [(1, 2), (2, 2), (3, 1)])
def test_cmcg_fixed_iterations_fp64(lib, q, n):
    """Impedance walls (well conditioned): 1e-11 at the oracle's count."""
    print(f"cmcg q={q} n={n}", flush=True)
    op, s, lp = pair(lib, n=n, q=q, seed=1, sigma=False, g=(q == 2), tags=2)
    ref = ocmcg.solve(op, tol=1e-8, max_iter=300)
    r = lib.cmcg_solve(lp, lib.cmcg_options_default(fixed_iters=ref.iters))
    st = lib.cmcg_result_stats(r)
    assert st["iters"] == ref.iters and st["steps"] == ref.M
    assert rel_norm_c(op, _filtered(lib, r, op), ref.F) < 1e-11
    hist = lib.cmcg_result_history(r)
    assert np.allclose(hist, ref.history, rtol=1e-6, atol=1e-12)


def _oracle_self_spread(op, iters):
    """How far the oracle's own filtered field moves under rounding-level
    changes at a fixed CG count (the CG iterates of an ill-conditioned problem
    amplify rounding): its inner products summed exactly in reverse order
    (fsum), and three runs whose period outputs carry a random relative
    perturbation of 2^-50 per entry -- less than the rounding that two
    implementations' different operation orders accumulate over a period of
    O(100) right-hand sides.  Returns the reference result and the largest
    deviation."""
    import math
    import oracle.dg as odg
    ref = ocmcg.solve(op, fixed_iters=iters)
    devs = []
    orig = odg.inner

    def inner_fsum(p_, U, V):
        U = U.reshape(p_.K, 6, p_.Np)
        MV = np.einsum("ij,ecj->eci", p_.ref["M"], V.reshape(p_.K, 6, p_.Np))
        return math.fsum((odg.mass_weights(p_)[:, :, None] * MV * U).ravel()[::-1])

    odg.inner = inner_fsum
    try:
        devs.append(rel_norm_c(op, ocmcg.solve(op, fixed_iters=iters).F, ref.F))
    finally:
        odg.inner = orig
    orig_fwd = timestep.forward
    for seed in range(3):
        rng = np.random.default_rng(seed)

        def fwd(p, U0, M, scheme, with_source, filt=False, _o=orig_fwd, _r=rng):
            r = _o(p, U0, M, scheme, with_source, filt)
            return r if filt else r * (1 + 2.0 ** -50 * _r.standard_normal(r.shape))

        timestep.forward = fwd
        try:
            devs.append(rel_norm_c(op, ocmcg.solve(op, fixed_iters=iters).F, ref.F))
        finally:
            timestep.forward = orig_fwd
    return ref, max(devs)


@pytest.mark.parametrize("q,n", [(1, 2), (2, 2)])
def test_cmcg_fixed_iterations_mixed_walls(lib, q, n):
    """Mixed PEC / impedance walls need 60-70 iterations; the GPU result must
    stay within a few times the oracle's own rounding spread."""
    op, s, lp = pair(lib, n=n, q=q, seed=1, sigma=False, g=(q == 2))
    it = ocmcg.solve(op, tol=1e-8, max_iter=300).iters
    ref, spread = _oracle_self_spread(op, it)
    r = lib.cmcg_solve(lp, lib.cmcg_options_default(fixed_iters=it))
    err = rel_norm_c(op, _filtered(lib, r, op), ref.F)
    print(f"mixed q={q}: iters {it} gpu err {err:.2e} oracle spread {spread:.2e}", flush=True)
    assert err < max(1e-11, 10 * spread)


@pytest.mark.parametrize("q,n", [(1, 2), (2, 2)])
def test_cmcg_mixed_walls_against_discrete_periodic(lib, q, n):
    """Mixed PEC / impedance walls, a rounding-independent pin: the FP64 GPU
    CMCG run to a tight tolerance reaches the exactly periodic orbit of the
    fully discrete scheme, solved directly by the oracle ((z I - R) U^ = S,
    filtered by the closed forms of the trapezoid / Hermite rules).  Unlike
    a fixed-count comparison, this does not depend on the summation order of
    either side's inner products."""
    from oracle import fs
    op, s, lp = pair(lib, n=n, q=q, seed=1, sigma=False, g=(q == 2))
    r = lib.cmcg_solve(lp, lib.cmcg_options_default(tol=1e-12, max_iter=600))
    st = lib.cmcg_result_stats(r)
    _, F = fs.discrete_periodic(op, st["steps"], timestep.default_scheme(q))
    err = rel_norm_c(op, _filtered(lib, r, op), F)
    print(f"mixed q={q}: {st['iters']} iterations to {st['rel_res']:.1e}, vs exact orbit {err:.2e}", flush=True)
    assert st["rel_res"] <= 1e-12
    assert err <= 1e-9


def test_cmcg_plain_fp64_configuration(lib):
    """The 1296-tet P1 configuration (n = 6): FP64 library CMCG at the
    oracle's iteration count matches the oracle's filtered field."""
    from paper_2106_02858_amd import inputs
    w = inputs.plain_fp64()
    op, s, lp = workload_pair(lib, w, 0)
    ref = ocmcg.solve(op, tol=1e-8, max_iter=500)
    r = lib.cmcg_solve(lp, lib.cmcg_options_default(fixed_iters=ref.iters))
    fr, fi = dev(np.zeros((op.K, 6, op.Np))), dev(np.zeros((op.K, 6, op.Np)))
    lib.cmcg_result_filtered_device(r, fr, fi)
    err = rel_norm_c(op, host(fr) + 1j * host(fi), ref.F)
    print(f"plain fp64: iters {ref.iters} M {ref.M} err {err:.3e}", flush=True)
    assert err < 1e-11
    # and with the stopping rule, the library stops at (nearly) the same count
    r2 = lib.cmcg_solve(lp, lib.cmcg_options_default(tol=1e-8))
    st = lib.cmcg_result_stats(r2)
    assert abs(st["iters"] - ref.iters) <= 1 and st["rel_res"] <= 1e-8


@pytest.mark.parametrize("q,n", [(1, 3), (2, 2), (3, 2)])
def test_cmcg_fp32_against_oracle(lib, q, n):
    op, s, lp = pair(lib, n=n, q=q, precision=1, seed=2, sigma=False, tags=2)
    ref = ocmcg.solve(op, tol=1e-10, max_iter=300)
    r = lib.cmcg_solve(lp, lib.cmcg_options_default(tol=1e-6))
    st = lib.cmcg_result_stats(r)
    fr, fi = dev(np.zeros((op.K, 6, op.Np))), dev(np.zeros((op.K, 6, op.Np)))
    lib.cmcg_result_filtered_device(r, fr, fi)
    err = rel_norm_c(op, host(fr) + 1j * host(fi), ref.F)
    print(f"fp32 q={q}: iters {st['iters']} err {err:.3e}", flush=True)
    assert st["rel_res"] <= 1e-6
    assert err < 1e-5


@pytest.mark.parametrize("q,n", [(1, 2), (2, 2)])
def test_cmcg_fixed_iterations_conductive_with_boundary_data(lib, q, n):
    """Conductivity sigma > 0 on ~30% of the elements and impedance data g on
    the walls (the problem statement's full right-hand side): CMCG iterates at
    a fixed count, 1e-11 bounded by the oracle's own rounding spread."""
    op, s, lp = pair(lib, n=n, q=q, seed=6, sigma=True, g=True, tags=2)
    iters = 12
    ref, spread = _oracle_self_spread(op, iters)
    r = lib.cmcg_solve(lp, lib.cmcg_options_default(fixed_iters=iters))
    err = rel_norm_c(op, _filtered(lib, r, op), ref.F)
    print(f"conductive cmcg q={q}: {err:.2e} (oracle spread {spread:.2e})", flush=True)
    assert err < max(1e-11, 10 * spread)


@pytest.mark.parametrize("q", [2, 3])
def test_two_wave_blocks_equal_one_wave_blocks(lib, q):
    """Variants 4 (two waves per 10-element block, half the output tiles each)
    and 8 (four waves) do the same arithmetic as variant 3: right-hand side and
    a period agree bit for bit, also with a partial last block."""
    import torch
    old = lib.cmcg_tune_get_stage(q, 1)
    try:
        xyz, tet, tags = inputs.cube_mesh(2)
        tet, tags = tet[:-3], np.full((tet.shape[0] - 3, 4), 2, dtype=np.int8)  # 45 elements: ragged
        K = tet.shape[0]
        m = lib.cmcg_mesh_create(xyz, tet, tags)
        s = lib.cmcg_space_create(m, q, 1)
        Np = lib.cmcg_space_info(s)["Np"]
        j = inputs.gaussian_current(lib.cmcg_space_nodes(s), (0.5, 0.4, 0.5), 0.3, 1)
        p = lib.cmcg_problem_create(s, np.random.default_rng(3).choice([1.0, 2.0, 4.0], K), np.ones(K),
                                    np.full(K, 0.2), 2 * np.pi, j)
        U = dev(np.random.default_rng(4).standard_normal((K, 6, Np)))
        outs = []
        for v in (3, 4, 8):
            lib.cmcg_tune_stage(q, 1, v)
            r, UT = torch.empty_like(U), torch.empty_like(U)
            lib.cmcg_debug_rhs(p, U, r, t=0.3, with_source=True)
            lib.cmcg_debug_period(p, U, UT, 1, True, opts=lib.cmcg_options_default(steps=12))
            torch.cuda.synchronize()
            outs.append((r.cpu(), UT.cpu()))
        for o in outs[1:]:
            assert torch.equal(outs[0][0], o[0]) and torch.equal(outs[0][1], o[1])
    finally:
        lib.cmcg_tune_stage(q, 1, old)


def test_graphed_period_follows_a_stage_variant_change(lib):
    """A period replayed from a captured graph runs the stage variant chosen
    when it is replayed: graphs are kept per variant, so after a change of
    variant the graphed period equals the eager one of the new variant bit for
    bit (and differs from the old variant's, whose arithmetic differs)."""
    import torch
    q = 3
    old = lib.cmcg_tune_get_stage(q, 1)
    try:
        xyz, tet, tags = inputs.cube_mesh(2)
        K = tet.shape[0]
        m = lib.cmcg_mesh_create(xyz, tet, tags)
        s = lib.cmcg_space_create(m, q, 1)
        Np = lib.cmcg_space_info(s)["Np"]
        j = inputs.gaussian_current(lib.cmcg_space_nodes(s), (0.5, 0.4, 0.5), 0.3, 1)
        p = lib.cmcg_problem_create(s, np.ones(K), np.ones(K), None, 2 * np.pi, j)
        U = dev(np.random.default_rng(5).standard_normal((K, 6, Np)))
        out = {}
        for v, graph in ((0, 1), (4, 1), (4, 0)):
            lib.cmcg_tune_stage(q, 1, v)
            UT = torch.empty_like(U)
            lib.cmcg_debug_period(p, U, UT, 1, True, opts=lib.cmcg_options_default(steps=10, use_graph=graph))
            torch.cuda.synchronize()
            out[(v, graph)] = UT.cpu()
        assert torch.equal(out[(4, 1)], out[(4, 0)])
        assert not torch.equal(out[(4, 1)], out[(0, 1)])
    finally:
        lib.cmcg_tune_stage(q, 1, old)


def test_graphed_period_follows_a_step_count_change(lib):
    """With the size-based default stage form (no variant chosen), periods of
    one problem at two step counts are captured as two graphs: the second
    graphed period equals its eager counterpart bit for bit (its graph key
    once lost the step count for the default form)."""
    import torch
    q = 3
    old = lib.cmcg_tune_get_stage(q, 1)
    try:
        lib.cmcg_tune_stage(q, 1, -1)
        xyz, tet, tags = inputs.cube_mesh(2)
        K = tet.shape[0]
        m = lib.cmcg_mesh_create(xyz, tet, tags)
        s = lib.cmcg_space_create(m, q, 1)
        Np = lib.cmcg_space_info(s)["Np"]
        j = inputs.gaussian_current(lib.cmcg_space_nodes(s), (0.5, 0.4, 0.5), 0.3, 1)
        p = lib.cmcg_problem_create(s, np.ones(K), np.ones(K), None, 2 * np.pi, j)
        U = dev(np.random.default_rng(6).standard_normal((K, 6, Np)))
        out = {}
        for steps, graph in ((60, 1), (64, 1), (64, 0)):
            UT = torch.empty_like(U)
            lib.cmcg_debug_period(p, U, UT, 1, True, opts=lib.cmcg_options_default(steps=steps, use_graph=graph))
            torch.cuda.synchronize()
            out[(steps, graph)] = UT.cpu()
        assert torch.equal(out[(64, 1)], out[(64, 0)])
        assert not torch.equal(out[(64, 1)], out[(60, 1)])
    finally:
        lib.cmcg_tune_stage(q, 1, old)


@pytest.mark.parametrize("precision", [0, 1])
def test_solves_are_reproducible_bit_for_bit(lib, precision):
    """The same problem solved twice from graphs and once eagerly: identical
    iteration counts, residual histories and filtered fields, bit for bit (no
    atomics; the inner products reduce in a fixed order)."""
    op, s, lp = pair(lib, n=2, q=3, precision=precision, seed=71)
    runs = []
    for use_graph in (1, 1, 0):
        r = lib.cmcg_solve(lp, lib.cmcg_options_default(tol=1e-6, max_iter=300, use_graph=use_graph))
        fr, fi = dev(np.zeros((op.K, 6, op.Np))), dev(np.zeros((op.K, 6, op.Np)))
        lib.cmcg_result_filtered_device(r, fr, fi)
        runs.append((lib.cmcg_result_stats(r)["iters"], np.asarray(lib.cmcg_result_history(r)),
                     host(fr), host(fi)))
    for it, hist, fr, fi in runs[1:]:
        assert it == runs[0][0] and np.array_equal(hist, runs[0][1])
        assert np.array_equal(fr, runs[0][2]) and np.array_equal(fi, runs[0][3])
