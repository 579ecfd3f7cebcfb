"""Build the same seeded problem for the oracle and for the HIP library."""
import numpy as np

from paper_2106_02858_amd import inputs
from oracle import dg
from tests._problems import hetero_problem


def lib_problem(cm, op, precision, xyz=None, tet=None, tags=None):
    """Library problem with exactly the oracle problem's input arrays."""
    geo = op.geo
    m = cm.cmcg_mesh_create(xyz, tet, tags)
    s = cm.cmcg_space_create(m, geo.q, precision)
    lp = cm.cmcg_problem_create(s, op.eps, op.mu, op.sigma, op.omega, op.j, op.g)
    return s, lp


def pair(cm, n=2, q=2, precision=0, seed=0, tags="mixed", sigma=True, g=False, alpha=1.0, omega=2 * np.pi,
         source=True):
    op = hetero_problem(n=n, q=q, seed=seed, tags=tags, sigma=sigma, g=g, alpha=alpha, omega=omega,
                        source=source)
    # mesh arrays: regenerate exactly as hetero_problem does
    from tests._problems import mixed_tags
    if tags == "mixed":
        xyz, tet, tg = mixed_tags(n, seed)
    else:
        xyz, tet, tg = inputs.cube_mesh(n, tags)
    s, lp = lib_problem(cm, op, precision, xyz, tet, tg)
    return op, s, lp


def workload_pair(cm, w, precision, j_pol_width=None):
    """Oracle + library problems for an inputs.Workload (Gaussian source)."""
    p0 = dg.make_problem(w.xyz, w.tet, w.tags, w.q, w.eps, w.mu, w.sigma, omega=w.omega)
    j = inputs.gaussian_current(p0.geo.x, w.centre, w.width, w.pol)
    op = dg.make_problem(w.xyz, w.tet, w.tags, w.q, w.eps, w.mu, w.sigma, omega=w.omega, j=j)
    s, lp = lib_problem(cm, op, precision, w.xyz, w.tet, w.tags)
    return op, s, lp


def rel_norm(op, a, b):
    return dg.norm(op, a - b) / dg.norm(op, b)


def rel_norm_c(op, a, b):
    d = a - b
    num = np.sqrt(abs(dg.inner(op, d.real, d.real)) + abs(dg.inner(op, d.imag, d.imag)))
    den = np.sqrt(abs(dg.inner(op, b.real, b.real)) + abs(dg.inner(op, b.imag, b.imag)))
    return num / den
