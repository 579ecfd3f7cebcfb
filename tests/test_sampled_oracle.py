"""The sampled-element oracle used by the full-size GPU parity tests equals
the full-mesh oracle at the sampled elements (small meshes, CPU)."""
import numpy as np
import pytest

from oracle import dg
from paper_2106_02858_amd import inputs
from tests._sampled import face_neighbours, sample_elements, sampled_oracle_rhs


@pytest.mark.parametrize("q,n", [(1, 4), (2, 3), (3, 2)])
def test_sampled_rhs_equals_full_rhs(q, n):
    w = inputs.large_single(n=n, q=q)
    p0 = dg.make_problem(w.xyz, w.tet, w.tags, w.q, w.eps, w.mu, w.sigma, omega=w.omega)
    nodes = p0.geo.x
    j = inputs.gaussian_current(nodes, w.centre, w.width, w.pol)
    op = dg.make_problem(w.xyz, w.tet, w.tags, w.q, w.eps, w.mu, w.sigma, omega=w.omega, j=j)
    U = np.random.default_rng(3).standard_normal((w.K, 6, op.Np))
    t = 0.21
    samples = sample_elements(w, np.random.default_rng(4))
    full = dg.phi(op, t, U, with_source=True)[samples]
    got = sampled_oracle_rhs(w, nodes, U, samples, t)
    assert np.max(np.abs(got - full)) <= 1e-13 * np.max(np.abs(full))


def test_face_neighbours_symmetric():
    w = inputs.large_single(n=3, q=1)
    nb = face_neighbours(w.tet, np.arange(w.K))
    for e in range(w.K):
        for f in range(4):
            if nb[e, f] >= 0:
                assert e in nb[nb[e, f]]
            else:
                assert w.tags[e, f] != 0
