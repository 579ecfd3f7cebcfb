"""Small seeded oracle problems shared by the tests."""
import numpy as np

from paper_2106_02858_amd import inputs
from oracle import dg


def mixed_tags(n, seed=0, pec_frac=0.5):
    """Cube mesh whose boundary faces are PEC or impedance at random."""
    xyz, tet, tags = inputs.cube_mesh(n, inputs.TAG_IMPEDANCE)
    rng = np.random.default_rng(seed)
    b = tags > 0
    t = np.where(rng.random(tags.shape) < pec_frac, inputs.TAG_PEC, inputs.TAG_IMPEDANCE)
    tags = np.where(b, t, 0).astype(np.int8)
    return xyz, tet, tags


def hetero_problem(n=2, q=2, seed=0, alpha=1.0, sigma=True, tags="mixed", omega=2 * np.pi,
                   source=True, g=False):
    rng = np.random.default_rng(seed)
    if tags == "mixed":
        xyz, tet, tg = mixed_tags(n, seed)
    else:
        xyz, tet, tg = inputs.cube_mesh(n, tags)
    K = tet.shape[0]
    eps = rng.choice([1.0, 2.0, 4.0], K)
    mu = rng.choice([1.0, 1.5], K)
    sig = rng.uniform(0, 0.5, K) * (rng.random(K) < 0.3) if sigma else None
    p0 = dg.make_problem(xyz, tet, tg, q, eps, mu, sig, omega=omega, alpha=alpha)
    j = None
    if source:
        j = (inputs.gaussian_current(p0.geo.x, [0.4, 0.5, 0.6], 0.3, 2)
             + 1j * inputs.gaussian_current(p0.geo.x, [0.6, 0.4, 0.5], 0.3, 0))
    gg = None
    if g:
        gg = rng.standard_normal((K, 4, p0.geo.Nfp, 3)) + 1j * rng.standard_normal((K, 4, p0.geo.Nfp, 3))
    return dg.make_problem(xyz, tet, tg, q, eps, mu, sig, omega=omega, j=j, g=gg, alpha=alpha)
