"""Pins of the run-up variant of the CMCG oracle (Section 6 names a few
limiting-amplitude periods before CMCG as an accelerator): the run-up state
is the exactly periodic orbit's initial state plus the homogeneous
propagator applied to the initial difference; the cost functional at that
state is the homogeneous propagator applied to Algorithm 1's G; and CMCG
from it reaches the exactly periodic discrete solution."""
import numpy as np
import pytest

from oracle import cmcg as ocmcg
from oracle import fs, timestep
from tests._problems import hetero_problem


@pytest.mark.parametrize("q", [1, 2])
def test_runup_state_is_orbit_plus_transient(q):
    p = hetero_problem(n=1, q=q, seed=3, tags=2, sigma=False)
    M = timestep.n_steps(p)
    scheme = timestep.default_scheme(q)
    Ustar = fs.discrete_periodic(p, M, scheme)[0].real
    for l in (1, 4):
        r = ocmcg.solve(p, M=M, scheme=scheme, fixed_iters=0, filt=False, runup=l)
        trans = -Ustar
        for _ in range(l):
            trans = timestep.forward(p, trans, M, scheme, with_source=False)
        assert np.max(np.abs(r.U0 - (Ustar + trans))) < 1e-11 * np.max(np.abs(Ustar))


def test_runup_functional_is_propagated_G():
    """J(U_l) = 1/2 ||P_psi U_l - U_l||^2 = 1/2 ||P^l G|| ^2 with G = P_psi 0,
    smaller than J(0) = 1/2 ||G||^2 when the walls dissipate."""
    p = hetero_problem(n=1, q=1, seed=4, tags=2, sigma=False)
    ops = ocmcg.Operators(p)
    G, _ = ocmcg.initialise(ops)
    U = np.zeros((p.K, 6, p.Np))
    PlG = G.copy()
    prev = 0.5 * ops.ip(G, G)
    for _ in range(3):
        U = ops.P_psi(U)
        PlG = ops.P(PlG)
        J = ocmcg.functional(ops, U, G)
        ref = 0.5 * ops.ip(PlG, PlG)
        assert abs(J - ref) <= 1e-12 * ref
        assert J < prev
        prev = J


@pytest.mark.parametrize("runup", [0, 3])
def test_cmcg_after_runup_reaches_periodic_solution(runup):
    p = hetero_problem(n=1, q=1, seed=6, tags=2, sigma=False)
    M = timestep.n_steps(p)
    _, Fdp = fs.discrete_periodic(p, M, 2)
    r = ocmcg.solve(p, tol=1e-10, M=M, scheme=2, runup=runup)
    assert r.rel_res <= 1e-10
    d = r.F - Fdp
    assert np.sqrt(np.vdot(d, d).real / np.vdot(Fdp, Fdp).real) < 1e-8
