"""Pins of the FW (limiting amplitude) oracle: the state after l periods is
the periodic orbit's initial state U* plus the homogeneous propagator applied
l times to the initial difference, and the filtered field converges to the
exactly periodic orbit's (impedance walls dissipate the transient)."""
import numpy as np
import pytest

from oracle import dg, fs, fw, timestep
from tests._problems import hetero_problem


@pytest.mark.parametrize("q", [1, 2])
def test_fw_state_is_orbit_plus_decaying_transient(q):
    p = hetero_problem(n=1, q=q, seed=3, tags=2, sigma=False)
    M = timestep.n_steps(p)
    scheme = timestep.default_scheme(q)
    Uh, Fdp = fs.discrete_periodic(p, M, scheme)
    Ustar = Uh.real
    for l in (1, 3):
        r = fw.solve(p, l + 1, M=M, scheme=scheme)   # l plain periods + the filtered one
        trans = -Ustar
        for _ in range(l):
            trans = timestep.forward(p, trans, M, scheme, with_source=False)
        assert np.max(np.abs(r.U0 - (Ustar + trans))) < 1e-11 * np.max(np.abs(Ustar))
        trans = timestep.forward(p, trans, M, scheme, with_source=False)
        scale = np.max(np.abs(Ustar))
        assert np.max(np.abs(r.U_end - (Ustar + trans))) < 1e-11 * scale
        # filter linearity: F(U0) = F(U*) + F_0(U0 - U*)
        _, Ftr = timestep.forward(p, r.U0 - Ustar, M, scheme, with_source=False, filt=True)
        assert np.max(np.abs(r.F - (Fdp + Ftr))) < 1e-10 * np.max(np.abs(Fdp))


def test_fw_converges_to_periodic_orbit():
    p = hetero_problem(n=1, q=1, seed=5, tags=2, sigma=False)
    M = timestep.n_steps(p)
    _, Fdp = fs.discrete_periodic(p, M, 2)
    errs = []
    for L in (2, 8, 32):
        r = fw.solve(p, L, M=M, scheme=2)
        errs.append(fw.rel_change(p, r.F, Fdp))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-3 * errs[0]


def test_fw_stops_on_tolerance():
    p = hetero_problem(n=1, q=1, seed=5, tags=2, sigma=False)
    r = fw.solve(p, 200, tol=1e-6)
    assert r.periods < 200 and r.history[-1] <= 1e-6 and r.history[0] == 1.0  # first: from zero
    assert all(h > 1e-6 for h in r.history[:-1])
    assert r.periods == len(r.history) + 1


def _problem_2d(q, seed):
    """Small 2-D TM problem with impedance walls (dissipative), seeded current."""
    from oracle import dg2d
    from paper_2106_02858_amd import inputs
    xy, tri, tags = inputs.cartesian_triangles(2, 2, side_tags=(2, 2, 2, 2))
    K = tri.shape[0]
    rng = np.random.default_rng(seed)
    eps = rng.choice([1.0, 2.0], K)
    p0 = dg2d.make_problem(xy, tri, tags, q, eps, np.ones(K), omega=2 * np.pi)
    j = rng.standard_normal((K, p0.Np)) + 1j * rng.standard_normal((K, p0.Np))
    return dg2d.make_problem(xy, tri, tags, q, eps, np.ones(K), omega=2 * np.pi, j=j)


@pytest.mark.parametrize("q", [1, 3])
def test_fw_state_is_orbit_plus_decaying_transient_2d(q):
    """The same identity for the 2-D TM operator."""
    p = _problem_2d(q, 11)
    M = timestep.n_steps(p)
    scheme = timestep.default_scheme(q)
    Uh, Fdp = fs.discrete_periodic(p, M, scheme)
    Ustar = Uh.real
    r = fw.solve(p, 3, M=M, scheme=scheme)   # two plain periods + the filtered one
    trans = -Ustar
    for _ in range(2):
        trans = timestep.forward(p, trans, M, scheme, with_source=False)
    assert np.max(np.abs(r.U0 - (Ustar + trans))) < 1e-11 * np.max(np.abs(Ustar))
    _, Ftr = timestep.forward(p, r.U0 - Ustar, M, scheme, with_source=False, filt=True)
    assert np.max(np.abs(r.F - (Fdp + Ftr))) < 1e-10 * np.max(np.abs(Fdp))
    errs = [fw.rel_change(p, fw.solve(p, L, M=M, scheme=scheme).F, Fdp) for L in (2, 8, 32)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-3 * errs[0]
