"""Pins of the local-time-stepping oracle (oracle/lts.py: Runge-Kutta-based
LTS with Taylor-frozen coarse unknowns; the paper's concluding remarks name
local time stepping as the remedy for locally refined meshes).

* equivalence to global stepping: with no fine element the homogeneous
  coarse step is the global RK step R(H B) (RK2 and RK4); with every element
  fine it is m global steps of H / m, source included; with m = 1 the RK2
  form is the global midpoint step for any fine set;
* order of accuracy on a locally refined (graded) mesh: the error of one
  period against the exact flow (sparse matrix exponential) and of a forced
  period against a far finer global RK4 reference falls at least at the base
  scheme's order (2 for RK2, 4 for RK4) when the coarse step is halved;
* the adjoint step is the eps,mu-adjoint of the homogeneous step;
* energy does not grow over periods with upwind fluxes and impedance walls;
* CMCG with local time stepping (exact adjoint periods) reaches a periodic
  orbit of the LTS scheme and its filtered field converges to the
  frequency-domain solution at the scheme's order.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import cmcg, dg, fs, lts, timestep
from paper_2106_02858_amd import inputs

# slab of thin cells in x (0.05 wide against 0.45): those elements' CFL steps
# are 4.5 times shorter than the others'
GRADED = ([0, .45, .5, .55, 1.], [0, .5, 1.], [0, .5, 1.])


def graded_problem(q, source=True, eps_seed=None, omega=2 * np.pi):
    xyz, tet, tags = inputs.graded_cube_mesh(*GRADED)
    K = tet.shape[0]
    eps = np.ones(K) if eps_seed is None else np.random.default_rng(eps_seed).choice([1.0, 2.0], K)
    p0 = dg.make_problem(xyz, tet, tags, q, eps, np.ones(K), omega=omega)
    j = inputs.gaussian_current(p0.geo.x, [.5, .5, .5], .3, 2) if source else None
    return dg.make_problem(xyz, tet, tags, q, eps, np.ones(K), omega=omega, j=j)


def step_fn(scheme):
    return timestep.rk2_step if scheme == 2 else timestep.rk4_step


@pytest.mark.parametrize("q", [1, 2])
def test_no_fine_element_is_the_global_step(q):
    p = graded_problem(q)
    sch = timestep.default_scheme(q)
    y = np.random.default_rng(1).standard_normal((p.K, 6, p.Np))
    H = 0.01
    z = lts.coarse_step(p, y, 0.3, H, 4, np.zeros(p.K, bool), sch, False)
    ref = step_fn(sch)(p, 0.3, y, H, False)[0]
    assert np.max(np.abs(z - ref)) <= 1e-14 * np.max(np.abs(ref))


@pytest.mark.parametrize("q", [1, 2])
def test_every_element_fine_is_global_substepping(q):
    p = graded_problem(q)
    sch = timestep.default_scheme(q)
    y = np.random.default_rng(2).standard_normal((p.K, 6, p.Np))
    H, m = 0.012, 3
    z = lts.coarse_step(p, y, 0.3, H, m, np.ones(p.K, bool), sch, True)
    ref = y
    for l in range(m):
        ref = step_fn(sch)(p, 0.3 + l * H / m, ref, H / m, True)[0]
    assert np.array_equal(z, ref)


def test_rk2_single_substep_is_the_midpoint_step():
    p = graded_problem(1)
    y = np.random.default_rng(3).standard_normal((p.K, 6, p.Np))
    fine = np.random.default_rng(4).random(p.K) < 0.5
    z = lts.coarse_step(p, y, 0.0, 0.01, 1, fine, 2, False)
    ref = timestep.rk2_step(p, 0.0, y, 0.01, False)[0]
    assert np.max(np.abs(z - ref)) <= 1e-14 * np.max(np.abs(ref))


def test_fine_elements_are_the_thin_slab():
    p = graded_problem(1)
    M, fine = lts.lts_steps(p, 4)
    xc = p.geo.x.mean(axis=1)[:, 0]
    assert np.array_equal(fine, (xc > .45) & (xc < .55))
    assert M * 4 >= timestep.n_steps(p) and M < timestep.n_steps(p)


@pytest.mark.parametrize("q,order", [(1, 2), (2, 4)])
def test_order_of_the_homogeneous_and_forced_period(q, order):
    p = graded_problem(q, eps_seed=5)
    sch = timestep.default_scheme(q)
    m = 4
    M0, fine = lts.lts_steps(p, m)
    y0 = np.random.default_rng(6).standard_normal((p.K, 6, p.Np)) * 1e-2
    T = 2 * np.pi / p.omega
    B = dg.assemble_B(p)
    exact = spla.expm_multiply(B * T, y0.ravel()).reshape(y0.shape)
    # forced reference: zero start, global RK4 with 16 steps per finest coarse step
    ref_f = timestep.forward(p, np.zeros_like(y0), 16 * 4 * M0, 4, True)
    eh, ef = [], []
    for M in (M0, 2 * M0, 4 * M0):
        eh.append(dg.norm(p, lts.forward(p, y0, M, m, fine, sch, False) - exact) / dg.norm(p, exact))
        ef.append(dg.norm(p, lts.forward(p, np.zeros_like(y0), M, m, fine, sch, True) - ref_f) / dg.norm(p, ref_f))
    for errs in (eh, ef):
        rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
        # at least the base scheme's order (RK4 on this mesh: 4.5, the
        # dissipated high modes' error falls faster than the leading term)
        assert np.all(rates > order - 0.3) and np.all(rates < order + 1), (errs, rates)


@pytest.mark.parametrize("q", [1, 2])
def test_adjoint_step(q):
    p = graded_problem(q, eps_seed=7)
    sch = timestep.default_scheme(q)
    M, fine = lts.lts_steps(p, 4)
    H = 2 * np.pi / p.omega / M
    rng = np.random.default_rng(8)
    x, w = rng.standard_normal((2, p.K, 6, p.Np))
    a = dg.inner(p, lts.coarse_step(p, x, 0.0, H, 4, fine, sch, False), w)
    b = dg.inner(p, x, lts.adjoint_step(p, w, H, 4, fine, sch))
    assert abs(a - b) <= 1e-13 * np.sqrt(dg.inner(p, x, x) * dg.inner(p, w, w))


@pytest.mark.parametrize("q", [1, 2])
def test_energy_does_not_grow(q):
    p = graded_problem(q, source=False, eps_seed=9)
    sch = timestep.default_scheme(q)
    M, fine = lts.lts_steps(p, 4)
    U = np.random.default_rng(10).standard_normal((p.K, 6, p.Np))
    e = [dg.energy(p, U)]
    for _ in range(3):
        U = lts.forward(p, U, M, 4, fine, sch, False)
        e.append(dg.energy(p, U))
    assert np.all(np.diff(e) <= 0), e


def test_cmcg_with_local_time_stepping():
    """CMCG on the LTS propagator: the iterate becomes periodic under the LTS
    period (so the backward periods are its exact adjoint: CG would stall
    otherwise), J decreases, and the filtered field converges to the FS
    solution at second order in the coarse step (P1, RK2)."""
    p = graded_problem(1)
    m = 4
    M0, fine = lts.lts_steps(p, m)
    r = cmcg.solve(p, tol=1e-10, max_iter=200, lts=m)
    assert r.rel_res <= 1e-10
    assert np.all(np.diff(r.J) <= 0)
    ops = cmcg.Operators(p, lts=m)
    misfit = r.U0 - ops.P_psi(r.U0)
    assert dg.norm(p, misfit) <= 1e-9 * dg.norm(p, r.U0)
    Ufs = fs.frequency_solve(p)

    def err(F):
        d = F - Ufs
        return np.sqrt(abs(dg.inner(p, d, d)) / abs(dg.inner(p, Ufs, Ufs)))

    e1 = err(r.F)
    r2 = cmcg.solve(p, tol=1e-10, max_iter=200, lts=m, M=2 * M0)
    e2 = err(r2.F)
    assert 3.0 < e1 / e2 < 5.0, (e1, e2)
