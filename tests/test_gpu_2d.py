"""GPU parity of the 2-D transverse-magnetic path (triangles, fields e, h1,
h2) against the 2-D oracle, through the C-ABI.

Tolerances as for the 3-D path: FP64 right-hand side and period 1e-12, CMCG
at a fixed iteration count 1e-11; FP32 fields 1e-5.  The meshes hold 64 and
100 triangles: several 21-triangle workgroups and a ragged last one.
"""
import math

import numpy as np
import pytest

from oracle import cmcg as ocmcg
from oracle import dg2d, exact2d, fs, fw as ofw, timestep
from paper_2106_02858_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {0: 1e-12, 1: 1e-5}
P, I = inputs.TAG_PEC, inputs.TAG_IMPEDANCE


def dev(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def pair2d(lib, n=4, q=2, precision=0, seed=0, walls=(P, I, P, I), sigma=True, g=True, omega=3 * math.pi,
           source=True):
    """Seeded heterogeneous 2-D problem for the oracle and the library."""
    xy, tri, tags = inputs.cartesian_triangles(n, n, side_tags=walls)
    K = tri.shape[0]
    rng = np.random.default_rng(seed)
    eps = rng.choice([1.0, 2.0, 4.0], K)
    mu = rng.choice([1.0, 1.5], K)
    sg = rng.uniform(0.0, 0.5, K) if sigma else None
    p0 = dg2d.make_problem(xy, tri, tags, q, eps, mu)
    Np, Nfp = p0.Np, p0.geo.Nfp
    j = (rng.standard_normal((K, Np)) + 1j * rng.standard_normal((K, Np))) if source else None
    gg = None
    if g and source:
        gg = np.zeros((K, 3, Nfp), complex)
        wall = p0.geo.tag == inputs.TAG_IMPEDANCE
        gg[wall] = rng.standard_normal((wall.sum(), Nfp)) + 1j * rng.standard_normal((wall.sum(), Nfp))
    op = dg2d.make_problem(xy, tri, tags, q, eps, mu, sg, omega=omega, j=j, g=gg)
    m = lib.cmcg_mesh2d_create(xy, tri, tags)
    s = lib.cmcg_space_create(m, q, precision)
    lp = lib.cmcg_problem_create(s, eps, mu, sg, omega, j, gg)
    return op, s, lp


def rel_norm(op, a, b):
    return dg2d.norm(op, a - b) / dg2d.norm(op, b)


def rel_norm_c(op, a, b):
    d = a - b
    num = np.sqrt(abs(dg2d.inner(op, d.real, d.real)) + abs(dg2d.inner(op, d.imag, d.imag)))
    den = np.sqrt(abs(dg2d.inner(op, b.real, b.real)) + abs(dg2d.inner(op, b.imag, b.imag)))
    return num / den


def filtered(lib, r, op):
    fr, fi = dev(np.zeros((op.K, 3, op.Np))), dev(np.zeros((op.K, 3, op.Np)))
    lib.cmcg_result_filtered_device(r, fr, fi)
    return host(fr) + 1j * host(fi)


@pytest.mark.parametrize("q", [1, 2, 3])
def test_space_nodes_and_layout(lib, q):
    op, s, lp = pair2d(lib, q=q)
    info = lib.cmcg_space_info(s)
    assert info["dim"] == 2 and info["Np"] == op.Np and info["Nfp"] == q + 1
    assert info["ndof"] == op.K * 3 * op.Np
    assert np.max(np.abs(lib.cmcg_space_nodes(s) - op.geo.x)) < 1e-15


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("q", [1, 2, 3])
def test_rhs_parity(lib, q, precision):
    print(f"2-D rhs q={q} prec={precision}", flush=True)
    op, s, lp = pair2d(lib, q=q, precision=precision, seed=q)
    U = np.random.default_rng(1).standard_normal((op.K, 3, op.Np))
    out = dev(np.zeros_like(U))
    for t, src in ((0.0, False), (0.123, True)):
        lib.cmcg_debug_rhs(lp, dev(U), out, t=t, with_source=src)
        ref = dg2d.phi(op, t, U, with_source=src)
        err = np.max(np.abs(host(out) - ref)) / np.max(np.abs(ref))
        assert err < TOL[precision], (t, src, err)


def strip_mesh(K):
    """K triangles (p_t, p_t+1, p_t+2) over the zigzag p_k = (k // 2, k % 2):
    any triangle count, orientations alternating, every unmatched edge a wall
    (PEC on even triangles, impedance on odd ones)."""
    k = np.arange(K + 2)
    xy = np.stack([k // 2, k % 2], axis=1).astype(np.float64)
    tri = np.stack([k[:K], k[1:K + 1], k[2:K + 2]], axis=1).astype(np.int64)
    owners = {}
    for e in range(K):
        for f in range(3):
            owners.setdefault(tuple(sorted(np.delete(tri[e], f))), []).append((e, f))
    tags = np.zeros((K, 3), dtype=np.int8)
    for own in owners.values():
        if len(own) == 1:
            e, f = own[0]
            tags[e, f] = P if e % 2 == 0 else I
    return xy, tri, tags


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("q", [1, 3])
def test_rhs_every_ragged_wave(lib, q, precision):
    """Every remainder of K modulo the 21 triangles one 64-lane wave holds (and
    one past two full waves), on strips with mixed orientation and both wall
    kinds: right-hand side with current and wall data against the oracle."""
    for K in list(range(1, 22)) + [41, 42, 43]:
        xy, tri, tags = strip_mesh(K)
        rng = np.random.default_rng(100 + K)
        eps, mu = rng.choice([1.0, 2.0, 4.0], K), rng.choice([1.0, 1.5], K)
        sg = rng.uniform(0.0, 0.5, K)
        p0 = dg2d.make_problem(xy, tri, tags, q, eps, mu)
        Np, Nfp = p0.Np, p0.geo.Nfp
        j = rng.standard_normal((K, Np)) + 1j * rng.standard_normal((K, Np))
        gg = np.zeros((K, 3, Nfp), complex)
        wall = p0.geo.tag == I
        gg[wall] = rng.standard_normal((wall.sum(), Nfp)) + 1j * rng.standard_normal((wall.sum(), Nfp))
        op = dg2d.make_problem(xy, tri, tags, q, eps, mu, sg, omega=2.5, j=j, g=gg)
        s = lib.cmcg_space_create(lib.cmcg_mesh2d_create(xy, tri, tags), q, precision)
        lp = lib.cmcg_problem_create(s, eps, mu, sg, 2.5, j, gg)
        U = rng.standard_normal((K, 3, Np))
        out = dev(np.zeros_like(U))
        lib.cmcg_debug_rhs(lp, dev(U), out, t=0.4, with_source=True)
        ref = dg2d.phi(op, 0.4, U, with_source=True)
        err = np.max(np.abs(host(out) - ref)) / np.max(np.abs(ref))
        assert err < TOL[precision], (K, err)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("walls", [(P,) * 4, (I,) * 4])
def test_zero_source_gives_zero_field(lib, walls, precision):
    """No current and no wall data: the periodic solution is zero; CMCG stops
    before its first iteration and the filtered fields are exact zeros."""
    xy, tri, tags = inputs.cartesian_triangles(3, 3, side_tags=walls)
    K = tri.shape[0]
    s = lib.cmcg_space_create(lib.cmcg_mesh2d_create(xy, tri, tags), 2, precision)
    p = lib.cmcg_problem_create(s, np.ones(K), np.ones(K), None, 2 * np.pi, None)
    r = lib.cmcg_solve(p, lib.cmcg_options_default(tol=1e-8))
    st = lib.cmcg_result_stats(r)
    assert st["iters"] == 0 and st["status"] == lib.CMCG_OK and st["rel_res"] == 0.0
    import torch
    fr = torch.ones((K, 3, 6), dtype=torch.float64, device="cuda")
    fi = torch.ones_like(fr)
    lib.cmcg_result_filtered_device(r, fr, fi)
    assert float(fr.abs().max()) == 0.0 and float(fi.abs().max()) == 0.0


@pytest.mark.parametrize("walls", [(P,) * 4, (I,) * 4])
@pytest.mark.parametrize("q", [1, 3])
def test_rhs_centred_flux_and_walls(lib, q, walls):
    op, s, lp = pair2d(lib, n=5, q=q, seed=7, walls=walls)
    op.alpha = 0.0
    U = np.random.default_rng(2).standard_normal((op.K, 3, op.Np))
    out = dev(np.zeros_like(U))
    lib.cmcg_debug_rhs(lp, dev(U), out, t=0.0, with_source=False,
                       opts=lib.cmcg_options_default(flux=lib.CMCG_FLUX_CENTRED))
    ref = dg2d.apply_B(op, U)
    assert np.max(np.abs(host(out) - ref)) / np.max(np.abs(ref)) < 1e-12


@pytest.mark.parametrize("q", [1, 2, 3])
def test_dot_parity_and_determinism(lib, q):
    op, s, lp = pair2d(lib, n=5, q=q, seed=4)
    rng = np.random.default_rng(5)
    U = rng.standard_normal((op.K, 3, op.Np))
    V = rng.standard_normal((op.K, 3, op.Np))
    a = lib.cmcg_debug_dot(lp, dev(U), dev(V))
    b = lib.cmcg_debug_dot(lp, dev(U), dev(V))
    assert a == b
    assert abs(a - dg2d.inner(op, U, V)) <= 1e-13 * dg2d.norm(op, U) * dg2d.norm(op, V)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("q", [1, 2, 3])
def test_period_parity(lib, q, precision):
    print(f"2-D period q={q} prec={precision}", flush=True)
    op, s, lp = pair2d(lib, n=4 if q < 3 else 3, q=q, precision=precision, seed=10 + q)
    M = timestep.n_steps(op)
    sch = timestep.default_scheme(q)
    assert lib.cmcg_problem_steps(lp)[0] == M
    U0 = np.random.default_rng(3).standard_normal((op.K, 3, op.Np))
    ut = dev(np.zeros_like(U0))
    fr, fi = dev(np.zeros_like(U0)), dev(np.zeros_like(U0))
    for use_graph in (0, 1):
        o = lib.cmcg_options_default(use_graph=use_graph)
        lib.cmcg_debug_period(lp, dev(U0), ut, 1, True, fr, fi, opts=o)
        refU, refF = timestep.forward(op, U0, M, sch, True, filt=True)
        assert rel_norm(op, host(ut), refU) < TOL[precision]
        assert rel_norm_c(op, host(fr) + 1j * host(fi), refF) < TOL[precision]
        lib.cmcg_debug_period(lp, dev(U0), ut, -1, False, opts=o)
        assert rel_norm(op, host(ut), timestep.backward(op, U0, M, sch)) < TOL[precision]


@pytest.mark.parametrize("q", [1, 2, 3])
def test_cmcg_fixed_iterations_fp64(lib, q):
    print(f"2-D cmcg q={q}", flush=True)
    op, s, lp = pair2d(lib, n=4 if q < 3 else 3, q=q, seed=20 + q, walls=(I,) * 4, sigma=False)
    ref = ocmcg.solve(op, tol=1e-8, max_iter=300)
    r = lib.cmcg_solve(lp, lib.cmcg_options_default(fixed_iters=ref.iters))
    st = lib.cmcg_result_stats(r)
    assert st["iters"] == ref.iters and st["steps"] == ref.M
    assert rel_norm_c(op, filtered(lib, r, op), ref.F) < 1e-11
    assert np.allclose(lib.cmcg_result_history(r), ref.history, rtol=1e-6, atol=1e-12)


@pytest.mark.parametrize("precision", [0, 1])
def test_cmcg_converges_to_the_discrete_periodic_orbit(lib, precision):
    op, s, lp = pair2d(lib, n=4, q=2, precision=precision, seed=31, walls=(P, P, I, I))
    M = timestep.n_steps(op)
    _, F = fs.discrete_periodic(op, M, timestep.default_scheme(op.geo.q))
    tol = 1e-9 if precision == 0 else 1e-6
    r = lib.cmcg_solve(lp, lib.cmcg_options_default(tol=tol, max_iter=600))
    assert lib.cmcg_result_stats(r)["status"] == lib.CMCG_OK
    assert rel_norm_c(op, filtered(lib, r, op), F) < (1e-7 if precision == 0 else 1e-4)


@pytest.mark.parametrize("precision", [0, 1])
def test_solves_are_reproducible_bit_for_bit(lib, precision):
    """The same problem solved twice from graphs and once eagerly: identical
    iteration counts, residual histories and filtered fields, bit for bit (no
    atomics; the inner products reduce in a fixed order)."""
    op, s, lp = pair2d(lib, n=5, q=3, precision=precision, seed=61, walls=(P, I, P, I))
    runs = []
    for use_graph in (1, 1, 0):
        r = lib.cmcg_solve(lp, lib.cmcg_options_default(tol=1e-6, max_iter=300, use_graph=use_graph))
        runs.append((lib.cmcg_result_stats(r)["iters"], np.asarray(lib.cmcg_result_history(r)),
                     filtered(lib, r, op)))
    for it, hist, F in runs[1:]:
        assert it == runs[0][0]
        assert np.array_equal(hist, runs[0][1]) and np.array_equal(F, runs[0][2])


def test_fw_fixed_periods(lib):
    op, s, lp = pair2d(lib, n=4, q=1, seed=41, walls=(I,) * 4)
    ref = ofw.solve(op, periods=12)
    r = lib.cmcg_fw_solve(lp, lib.cmcg_options_default(fixed_iters=12))
    assert rel_norm_c(op, filtered(lib, r, op), ref.F) < 1e-12


def test_result_fields_layout(lib):
    op, s, lp = pair2d(lib, n=3, q=2, seed=5, walls=(I,) * 4)
    r = lib.cmcg_solve(lp, lib.cmcg_options_default(fixed_iters=3))
    F = filtered(lib, r, op)
    e, h = lib.cmcg_result_fields(r, op.K, op.Np, dim=2)
    assert np.array_equal(e, F[:, 0]) and np.array_equal(h, np.transpose(F[:, 1:3], (0, 2, 1)))


def test_unsupported_2d_calls_are_rejected(lib):
    op, s, lp = pair2d(lib, n=2, q=1)
    with pytest.raises(lib.CmcgError):   # one 2-D stage kernel per precision: nothing to tune
        lib.cmcg_autotune_stage(lp)


@pytest.mark.parametrize("delta", [0.125, 0.015625])
def test_paper_cavity_p1_32x32(lib, delta):
    """The cavity experiment at its printed size (P1, 32 x 32 Cartesian mesh,
    4096 triangles, j = 1, omega = 3 sqrt(2) pi + sqrt(2) pi delta): CMCG on
    the GPU converges to the exactly periodic discrete orbit.  Its error
    against the exact solution adds the RK2 time-discretisation error (M = 146
    steps per period at c_1 = 0.24) to that of the frequency-domain upwind
    system: 0.0074 against 0.0052 at delta = 1/8."""
    w = inputs.cavity2d(32, 1, 3 * math.sqrt(2) * math.pi, delta)
    p0 = dg2d.make_problem(w.xy, w.tri, w.tags, 1, w.eps, w.mu, omega=w.omega)
    j = inputs.current_2d(w, p0.geo.x)
    op = dg2d.make_problem(w.xy, w.tri, w.tags, 1, w.eps, w.mu, omega=w.omega, j=j)
    m = lib.cmcg_mesh2d_create(w.xy, w.tri, w.tags)
    s = lib.cmcg_space_create(m, 1, lib.CMCG_FP64)
    lp = lib.cmcg_problem_create(s, w.eps, w.mu, None, w.omega, j)
    r = lib.cmcg_solve(lp, lib.cmcg_options_default(tol=1e-10, max_iter=4000))
    st = lib.cmcg_result_stats(r)
    print(f"cavity 32x32 P1 delta={delta}: {st['iters']} iterations, M = {st['steps']}", flush=True)
    assert st["status"] == lib.CMCG_OK and st["steps"] == timestep.n_steps(op)
    F = filtered(lib, r, op)
    _, Fd = fs.discrete_periodic(op, st["steps"], 2)
    assert rel_norm_c(op, F, Fd) < 1e-8
    err, ref = exact2d.energy_error(op.geo, w.xy, w.tri, w.eps, w.mu, F, lambda x: exact2d.cavity(w.omega, x),
                                    nq=6)
    U_fs = fs.frequency_solve(op)
    err_fs, _ = exact2d.energy_error(op.geo, w.xy, w.tri, w.eps, w.mu, U_fs,
                                     lambda x: exact2d.cavity(w.omega, x), nq=6)
    print(f"  error vs exact: CMCG {err / ref:.5f}, frequency-domain upwind system {err_fs / ref:.5f}", flush=True)
    assert err_fs < err < 2.5 * err_fs


def test_serving_engine_mixes_2d_and_3d_requests(lib):
    """A 2-D and a 3-D request share one engine (overlapping on their own
    streams); each served result equals the same problem solved alone."""
    from tests._pairs import pair
    op2, s2, lp2 = pair2d(lib, n=6, q=2, seed=51, walls=(I,) * 4)
    op3, s3, lp3 = pair(lib, n=2, q=2, seed=52, tags=inputs.TAG_IMPEDANCE)
    o = lib.cmcg_options_default(tol=1e-8, max_iter=500)
    e = lib.cmcg_engine_create(1 << 32, 4)
    slots = {lib.cmcg_engine_admit(e, lp2, o): (lp2, op2, 3), lib.cmcg_engine_admit(e, lp3, o): (lp3, op3, 6)}
    assert None not in slots
    while any(lib.cmcg_engine_poll(e, s) == 1 for s in slots):
        lib.cmcg_engine_step(e)
    for slot, (lp, op, nc) in slots.items():
        served = lib.cmcg_engine_collect(e, slot, lp)
        alone = lib.cmcg_solve(lp, o)
        import torch
        bufs = [torch.zeros((op.K, nc, op.Np), dtype=torch.float64, device="cuda") for _ in range(4)]
        lib.cmcg_result_filtered_device(served, bufs[0], bufs[1])
        lib.cmcg_result_filtered_device(alone, bufs[2], bufs[3])
        assert torch.equal(bufs[0], bufs[2]) and torch.equal(bufs[1], bufs[3])
        assert lib.cmcg_result_stats(served)["iters"] == lib.cmcg_result_stats(alone)["iters"]


@pytest.fixture(scope="module")
def trap_disk_reference():
    """Oracle right-hand side and one period of the benchmarked 2-D
    configuration, computed once for both precisions."""
    w = inputs.trap2d(75, 3, "disk")
    p0 = dg2d.make_problem(w.xy, w.tri, w.tags, 3, w.eps, w.mu, omega=w.omega)
    j = inputs.current_2d(w, p0.geo.x)
    op = dg2d.make_problem(w.xy, w.tri, w.tags, 3, w.eps, w.mu, omega=w.omega, j=j)
    U = np.random.default_rng(9).standard_normal((op.K, 3, op.Np))
    t = 0.41 * 2 * math.pi / w.omega
    M = timestep.n_steps(op)
    print(f"oracle for the full-size trap disk (K={op.K}, {M} RK4 steps)", flush=True)
    refU, refF = timestep.forward(op, 1e-2 * U, M, 4, True, filt=True)
    return w, op, U, t, dg2d.phi(op, t, U), M, refU, refF


@pytest.mark.parametrize("precision", [0, 1])
def test_full_size_trap_disk(lib, precision, trap_disk_reference):
    """The benchmarked 2-D configuration at full size (22500 triangles, P3,
    Gaussian current, impedance walls): one right-hand side at every element,
    and one whole period with source and filter, against the oracle."""
    w, op, U, t, ref, M, refU, refF = trap_disk_reference
    print(f"full-size trap disk K={w.K} precision={precision}", flush=True)
    m = lib.cmcg_mesh2d_create(w.xy, w.tri, w.tags)
    s = lib.cmcg_space_create(m, 3, precision)
    nodes = lib.cmcg_space_nodes(s)
    assert np.max(np.abs(nodes - op.geo.x)) < 1e-15
    lp = lib.cmcg_problem_create(s, w.eps, w.mu, None, w.omega, inputs.current_2d(w, nodes))
    out = dev(np.zeros_like(U))
    lib.cmcg_debug_rhs(lp, dev(U), out, t=t, with_source=True)
    err = np.max(np.abs(host(out) - ref)) / np.max(np.abs(ref))
    print(f"  rhs max rel err {err:.2e}", flush=True)
    assert err < TOL[precision]
    assert lib.cmcg_problem_steps(lp)[0] == M
    ut = dev(np.zeros_like(U))
    fr, fi = dev(np.zeros_like(U)), dev(np.zeros_like(U))
    lib.cmcg_debug_period(lp, dev(1e-2 * U), ut, 1, True, fr, fi)
    e1, e2 = rel_norm(op, host(ut), refU), rel_norm_c(op, host(fr) + 1j * host(fi), refF)
    print(f"  period ({M} RK4 steps): state {e1:.2e}, filtered {e2:.2e}", flush=True)
    assert e1 < TOL[precision] and e2 < TOL[precision]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("q", [1, 3])
def test_batched_members_equal_single_solves(lib, q, precision):
    """2-D batched launches (grid.y = member): members with different
    frequencies (so different step counts), materials, currents and wall data; every
    member equals its single solve bit for bit, and the FP64 members match the
    oracle at a fixed iteration count."""
    print(f"2-D batch q={q} prec={precision}", flush=True)
    xy, tri, tags = inputs.cartesian_triangles(4, 4, side_tags=(I, I, P, I))
    K = tri.shape[0]
    m = lib.cmcg_mesh2d_create(xy, tri, tags)
    s = lib.cmcg_space_create(m, q, precision)
    rng = np.random.default_rng(60 + q)
    ops, lps = [], []
    for b in range(5):
        eps = rng.choice([1.0, 2.0], K) if b % 2 else np.ones(K)
        om = (2.0 + 0.5 * b) * math.pi
        p0 = dg2d.make_problem(xy, tri, tags, q, eps, np.ones(K), omega=om)
        j = rng.standard_normal((K, p0.Np)) + 1j * rng.standard_normal((K, p0.Np))
        g = None
        if b == 1:
            g = np.zeros((K, 3, p0.geo.Nfp), complex)
            wall = p0.geo.tag == inputs.TAG_IMPEDANCE
            g[wall] = rng.standard_normal((wall.sum(), p0.geo.Nfp))
        ops.append(dg2d.make_problem(xy, tri, tags, q, eps, np.ones(K), omega=om, j=j, g=g))
        lps.append(lib.cmcg_problem_create(s, eps, np.ones(K), None, om, j, g))
    o = lib.cmcg_options_default(fixed_iters=6)
    res = lib.cmcg_solve_batch(lps, o)
    for b, (op, lp) in enumerate(zip(ops, lps)):
        single = lib.cmcg_solve(lp, o)
        assert lib.cmcg_result_stats(res[b])["steps"] == lib.cmcg_result_stats(single)["steps"]
        assert np.array_equal(filtered(lib, res[b], op), filtered(lib, single, op)), b
        if precision == 0:
            ref = ocmcg.solve(op, fixed_iters=6)
            assert rel_norm_c(op, filtered(lib, res[b], op), ref.F) < 1e-11


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("walls", [(P,) * 4, (I,) * 4])
def test_single_cell_mesh(lib, walls, precision):
    """One Cartesian cell (4 triangles, one partly filled workgroup): right-hand
    side and a period with source and filter against the oracle."""
    op, s, lp = pair2d(lib, n=1, q=2, precision=precision, seed=70, walls=walls)
    assert op.K == 4
    U = np.random.default_rng(71).standard_normal((op.K, 3, op.Np))
    out = dev(np.zeros_like(U))
    lib.cmcg_debug_rhs(lp, dev(U), out, t=0.2, with_source=True)
    ref = dg2d.phi(op, 0.2, U)
    assert np.max(np.abs(host(out) - ref)) / np.max(np.abs(ref)) < TOL[precision]
    M = timestep.n_steps(op)
    ut = dev(np.zeros_like(U))
    fr, fi = dev(np.zeros_like(U)), dev(np.zeros_like(U))
    lib.cmcg_debug_period(lp, dev(U), ut, 1, True, fr, fi)
    refU, refF = timestep.forward(op, U, M, 4, True, filt=True)
    assert rel_norm(op, host(ut), refU) < TOL[precision]
    assert rel_norm_c(op, host(fr) + 1j * host(fi), refF) < TOL[precision]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("q", [1, 2])
def test_several_harmonics(lib, q, precision):
    """A three-harmonic current (k = 1, 2, 3 times omega0) on a 2-D problem:
    CMCG at a fixed iteration count over the base period, each harmonic
    filtered at its own frequency, against the oracle."""
    from oracle import multifreq
    xy, tri, tags = inputs.cartesian_triangles(4, 4, side_tags=(P, I, I, I))
    K = tri.shape[0]
    eps = np.random.default_rng(13).choice([1.0, 2.0], K)
    omega0 = 1.5 * np.pi
    base = dg2d.make_problem(xy, tri, tags, q, eps, np.ones(K), omega=omega0)
    ks = [1, 2, 3]
    js = [np.exp(-np.sum((base.geo.x - c) ** 2, axis=-1) / 0.1) * (1 + 0.5j * h)
          for h, c in enumerate(((0.4, 0.5), (0.6, 0.4), (0.5, 0.6)))]
    mp = multifreq.make(base, ks, js)
    m = lib.cmcg_mesh2d_create(xy, tri, tags)
    s = lib.cmcg_space_create(m, q, precision)
    lp = lib.cmcg_problem_create_harmonics(s, eps, np.ones(K), None, omega0, ks, np.stack(js))
    M0 = 6 * ((lib.cmcg_problem_steps(lp, lib.cmcg_options_default())[0] + 5) // 6)
    ref = multifreq.solve(mp, M=M0, fixed_iters=8)
    r = lib.cmcg_solve(lp, lib.cmcg_options_default(fixed_iters=8, steps=M0))
    assert lib.cmcg_result_harmonics(r) == 3
    import torch
    for h in range(3):
        fr = torch.zeros((K, 3, base.Np), dtype=torch.float64, device="cuda")
        fi = torch.zeros_like(fr)
        lib.cmcg_result_filtered_harmonic_device(r, h, fr, fi)
        err = rel_norm_c(base, fr.cpu().numpy() + 1j * fi.cpu().numpy(), ref.Fs[h])
        print(f"  2-D harmonic k={ks[h]} q={q} prec={precision}: {err:.2e}", flush=True)
        assert err < (1e-11 if precision == 0 else 1e-5)


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_lean_form_equals_single_early_form(lib, precision):
    """A batch above the early-load threshold (30 members x 77 workgroups) runs
    the lean stage form while each single solve of the same 1600-triangle
    problem runs the early-load form: the two forms do the same arithmetic in
    the same order, so the members still equal their single solves bit for
    bit."""
    xy, tri, tags = inputs.cartesian_triangles(20, 20, side_tags=(I, I, P, I))
    K = tri.shape[0]
    m = lib.cmcg_mesh2d_create(xy, tri, tags)
    s = lib.cmcg_space_create(m, 3, precision)
    nodes = lib.cmcg_space_nodes(s)
    rng = np.random.default_rng(80)
    lps = []
    for b in range(30):
        c = rng.uniform(0.2, 0.8, 2)
        j = np.exp(-np.sum((nodes - c) ** 2, axis=-1) / 0.02)
        lps.append(lib.cmcg_problem_create(s, np.ones(K), np.ones(K), None, 4 * math.pi, j))
    o = lib.cmcg_options_default(fixed_iters=3)
    res = lib.cmcg_solve_batch(lps, o)
    op = dg2d.make_problem(xy, tri, tags, 3, np.ones(K), np.ones(K))
    for b in (0, 13, 29):
        single = lib.cmcg_solve(lps[b], o)
        assert np.array_equal(filtered(lib, res[b], op), filtered(lib, single, op)), b
