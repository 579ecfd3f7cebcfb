"""Pins of the several-frequencies-in-one-solve oracle: each filtered
harmonic of the converged CMCG solution equals the exactly periodic discrete
orbit of that harmonic alone (fs.discrete_periodic over its own period with
the same time step), and a single harmonic k = 1 reproduces the ordinary
CMCG oracle."""
import numpy as np
import pytest

from oracle import cmcg as ocmcg
from oracle import dg, fs, multifreq, timestep
from paper_2106_02858_amd import inputs
from tests._pairs import rel_norm_c


def base_problem(q, omega0):
    xyz, tet, tags = inputs.cube_mesh(1)
    K = tet.shape[0]
    rng = np.random.default_rng(8)
    return dg.make_problem(xyz, tet, tags, q, rng.choice([1.0, 2.0], K), np.ones(K), omega=omega0)


@pytest.mark.parametrize("q", [1, 2])
def test_harmonics_equal_single_harmonic_orbits(q):
    omega0 = np.pi
    base = base_problem(q, omega0)
    ks = [1, 2, 3]
    js = [inputs.gaussian_current(base.geo.x, c, 0.4, pol) for c, pol in
          (((0.4, 0.5, 0.5), 2), ((0.6, 0.4, 0.5), 0), ((0.5, 0.5, 0.6), 1))]
    mp = multifreq.make(base, ks, js)
    scheme = timestep.default_scheme(q)
    M0 = 6 * ((timestep.n_steps(dg.Problem(base.geo, base.ref, base.eps, base.mu, base.sigma, 3 * omega0,
                                          None, None)) * 3 + 5) // 6)  # divisible by every k, dt within CFL
    res = multifreq.solve(mp, tol=1e-12, max_iter=400, M=M0, scheme=scheme)
    assert res.rel_res <= 1e-12
    for k, ph, F in zip(ks, mp.harm, res.Fs):
        _, Fdp = fs.discrete_periodic(ph, M0 // k, scheme)
        err = rel_norm_c(ph, F, Fdp)
        print(f"q={q} k={k}: {err:.2e}")
        assert err < 1e-9


def test_single_harmonic_is_plain_cmcg():
    base = base_problem(2, 2 * np.pi)
    j = inputs.gaussian_current(base.geo.x, (0.5, 0.5, 0.5), 0.3, 2)
    mp = multifreq.make(base, [1], [j])
    p = dg.Problem(base.geo, base.ref, base.eps, base.mu, base.sigma, base.omega, j, None)
    a = multifreq.solve(mp, fixed_iters=7)
    b = ocmcg.solve(p, fixed_iters=7)
    assert rel_norm_c(p, a.Fs[0], b.F) < 1e-13
    assert np.allclose(a.history, b.history, rtol=1e-12)


@pytest.mark.parametrize("q", [1, 3])
def test_harmonics_equal_single_harmonic_orbits_2d(q):
    """The same pin on a 2-D TM problem (triangles, fields e, h1, h2)."""
    from oracle import dg2d
    xy, tri, tags = inputs.cartesian_triangles(2, 2, side_tags=(1, 2, 2, 2))
    K = tri.shape[0]
    omega0 = np.pi
    base = dg2d.make_problem(xy, tri, tags, q, np.random.default_rng(9).choice([1.0, 2.0], K), np.ones(K),
                             omega=omega0)
    ks = [1, 2, 3]
    js = [np.exp(-np.sum((base.geo.x - c) ** 2, axis=-1) / 0.2) * (1 + 0.5j * h)
          for h, c in enumerate(((0.4, 0.5), (0.6, 0.4), (0.5, 0.6)))]
    mp = multifreq.make(base, ks, js)
    scheme = timestep.default_scheme(q)
    p3 = dg2d.Problem2D(base.geo, base.ref, base.eps, base.mu, base.sigma, 3 * omega0, None, None)
    M0 = 6 * ((timestep.n_steps(p3) * 3 + 5) // 6)
    res = multifreq.solve(mp, tol=1e-12, max_iter=400, M=M0, scheme=scheme)
    assert res.rel_res <= 1e-12
    for k, ph, F in zip(ks, mp.harm, res.Fs):
        _, Fdp = fs.discrete_periodic(ph, M0 // k, scheme)
        d = F - Fdp
        err = np.sqrt((dg2d.norm(ph, d.real) ** 2 + dg2d.norm(ph, d.imag) ** 2) /
                      (dg2d.norm(ph, Fdp.real) ** 2 + dg2d.norm(ph, Fdp.imag) ** 2))
        print(f"2-D q={q} k={k}: {err:.2e}")
        assert err < 1e-9
