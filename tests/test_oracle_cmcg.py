"""Pins of the oracle's CMCG (Algorithms 1-3) and its relation to the
frequency-domain solution (Sections 5, 6).

* filtered CMCG equals the exactly periodic orbit of the fully discrete
  scheme, obtained by an independent sparse direct solve of (z I - R) U^ = S;
* J decreases monotonically and its CG recurrence matches J evaluated
  directly (convergence theory of Section 5.1);
* the gradient of Algorithm 2 matches a central difference of J (J is
  quadratic, so the difference is exact up to rounding);
* convergence from a random initial guess to the same filtered field;
* time-discretisation error against the FS solution decays as dt^2 (RK2 +
  trapezoid) and dt^4 (RK4 + Hermite);
* the FS solution converges to a manufactured PEC-cavity solution under
  mesh refinement.
"""
import numpy as np
import pytest

from oracle import cmcg, dg, fs, timestep
from tests._problems import hetero_problem


# sigma = 0 as in all experiments of Section 6; scattered conductive elements
# spread the small singular values of (I - P) and slow CG down a lot.
CASES = [(1, 2, 1, "mixed"), (2, 2, 1, 2), (3, 1, 1, "mixed")]


@pytest.mark.parametrize("q,n,seed,tags", CASES)
def test_cmcg_matches_discrete_periodic(q, n, seed, tags):
    p = hetero_problem(n=n, q=q, seed=seed, g=(q == 2), tags=tags, sigma=False)
    r = cmcg.solve(p, tol=1e-11, max_iter=200)
    assert r.rel_res <= 1e-11
    M, sch = r.M, timestep.default_scheme(q)
    _, F = fs.discrete_periodic(p, M, sch)
    assert dg.norm(p, r.F - F) <= 1e-9 * dg.norm(p, F)
    # the periodic initial condition has (numerically) zero misfit
    misfit = r.U0 - timestep.forward(p, r.U0, M, sch, True)
    assert dg.norm(p, misfit) <= 1e-8 * dg.norm(p, r.U0)


def test_J_monotone_and_recurrence():
    p = hetero_problem(n=2, q=1, seed=4)
    ops = cmcg.Operators(p)
    G, Gstar = cmcg.initialise(ops)
    r = cmcg.solve(p, tol=1e-6, max_iter=50)
    assert np.all(np.diff(r.J) <= 0)
    # recompute J at the iterate reached after 3 iterations
    r3 = cmcg.solve(p, fixed_iters=3, filt=False)
    assert abs(cmcg.functional(ops, r3.U0, G) - r3.J[3]) <= 1e-10 * r3.J[0]


def test_gradient_finite_difference():
    p = hetero_problem(n=2, q=2, seed=6)
    ops = cmcg.Operators(p)
    G, Gstar = cmcg.initialise(ops)
    rng = np.random.default_rng(2)
    U = rng.standard_normal((p.K, 6, p.Np)) * 1e-2
    V = rng.standard_normal((p.K, 6, p.Np)) * 1e-2
    g = cmcg.gradient(ops, U, Gstar)
    h = 0.5
    fd = (cmcg.functional(ops, U + h * V, G) - cmcg.functional(ops, U - h * V, G)) / (2 * h)
    assert abs(fd - ops.ip(g, V)) <= 1e-10 * abs(fd)


def test_random_initial_guess_same_filtered_field():
    p = hetero_problem(n=2, q=1, seed=8, sigma=False)
    r0 = cmcg.solve(p, tol=1e-11, max_iter=300)
    u0 = np.random.default_rng(1).standard_normal((p.K, 6, p.Np))
    r1 = cmcg.solve(p, tol=1e-12, max_iter=300, u0=u0)
    assert dg.norm(p, r0.F - r1.F) <= 1e-8 * dg.norm(p, r0.F)


@pytest.mark.parametrize("q,order", [(1, 2), (2, 4)])
def test_time_discretisation_order_against_fs(q, order):
    p = hetero_problem(n=1, q=q, seed=3)
    B = dg.assemble_B(p)
    Ufs = fs.frequency_solve(p, B)
    M0 = 2 * timestep.n_steps(p)
    errs = []
    for M in (M0, 2 * M0, 4 * M0):
        _, F = fs.discrete_periodic(p, M, timestep.default_scheme(q), B)
        errs.append(dg.norm(p, F - Ufs) / dg.norm(p, Ufs))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(rates - order) < 0.3), (errs, rates)


def cavity_exact(x, omega):
    """PEC cavity field e = (sin pi y sin pi z, 2 sin pi x sin pi z,
    3 sin pi x sin pi y), h = curl e / (i omega), j = i(omega - 2 pi^2/omega) e
    for eps = mu = 1 in the convention of eq. (1.1)."""
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    s, c, pi = np.sin, np.cos, np.pi
    e = np.stack([s(pi * Y) * s(pi * Z), 2 * s(pi * X) * s(pi * Z), 3 * s(pi * X) * s(pi * Y)], -1)
    curl = np.stack([3 * pi * s(pi * X) * c(pi * Y) - 2 * pi * s(pi * X) * c(pi * Z),
                     pi * s(pi * Y) * c(pi * Z) - 3 * pi * c(pi * X) * s(pi * Y),
                     2 * pi * c(pi * X) * s(pi * Z) - pi * c(pi * Y) * s(pi * Z)], -1)
    h = curl / (1j * omega)
    j = 1j * (omega - 2 * pi ** 2 / omega) * e
    return e, h, j


def test_fs_mesh_convergence_pec_cavity():
    from paper_2106_02858_amd import inputs
    omega = 2 * np.pi
    errs = []
    for n in (1, 2, 4):
        xyz, tet, tags = inputs.cube_mesh(n, inputs.TAG_PEC)
        K = tet.shape[0]
        p0 = dg.make_problem(xyz, tet, tags, 1, np.ones(K), np.ones(K), omega=omega)
        e, h, j = cavity_exact(p0.geo.x, omega)
        p = dg.make_problem(xyz, tet, tags, 1, np.ones(K), np.ones(K), omega=omega, j=j)
        U = fs.frequency_solve(p)
        ex = np.concatenate([np.transpose(e, (0, 2, 1)), np.transpose(h, (0, 2, 1))], axis=1)
        errs.append(dg.norm(p, U - ex) / dg.norm(p, ex))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert errs[-1] < 0.15
    assert rates[-1] > 1.3, (errs, rates)
