"""Pins of the 2-D transverse-magnetic oracle (Section 5.2.1, two-dimensional
setting; Section 5.2.2, DG scheme; Section 5.3, CFL rule; Section 6, numerical
examples).

* reference triangle: exact integrals and derivatives of polynomials;
* geometry of the Cartesian meshes of Section 6 (four triangles per cell);
* energy: the centred flux conserves, the upwind flux dissipates;
* the paper's CFL constants c_1 = 0.24 (RK2, P1) and c_3 = 0.12 (RK4, P3)
  lie just below the stability limits of the upwind operator, and above
  those of an operator with twice its penalty;
* exact solutions against independent closed forms;
* the FS error levels printed in Section 6 (tests/golden/fs_errors_2d.txt);
* CMCG on a 2-D problem converges to the exactly periodic discrete orbit.
"""
import math
from pathlib import Path

import numpy as np
import pytest

from oracle import cmcg, dg2d, exact2d, fs, refelem2d, timestep
from paper_2106_02858_amd import inputs

GOLDEN = Path(__file__).parent / "golden" / "fs_errors_2d.txt"


def _golden():
    rows = []
    for line in GOLDEN.read_text().splitlines():
        if not line.strip() or line.startswith("#"):
            continue
        f = line.split()
        rows.append(dict(exp=f[0], q=int(f[1]), n=int(f[2]), w=float(f[3]), delta=float(f[4]),
                         printed=float(f[5])))
    return rows


def _problem(w, alpha=1.0, project=True):
    p0 = dg2d.make_problem(w.xy, w.tri, w.tags, w.q, w.eps, w.mu, None, w.omega)
    j = inputs.current_2d(w, p0.geo.x)
    g = None
    if w.source == "planewave":
        g = inputs.planewave_boundary_data(w, p0.geo.x[:, p0.ref["fmask"]], project=project)
    if w.source == "wallwave":
        g = inputs.waveguide_boundary_data(w, p0.geo.x[:, p0.ref["fmask"]], project=project)
    return dg2d.make_problem(w.xy, w.tri, w.tags, w.q, w.eps, w.mu, None, w.omega, j=j, g=g, alpha=alpha)


# ------------------------------------------------------------- reference triangle

@pytest.mark.parametrize("q", [1, 2, 3])
def test_reference_triangle_is_exact(q):
    r = refelem2d.matrices(q)
    xi = refelem2d.nodes(q)
    Np = refelem2d.np_count(q)
    # unit-area element: the integral of 1 is 1; of xi1 is 1/3; of xi1 xi2 is 1/12
    one = np.ones(Np)
    assert abs(one @ r["M"] @ one - 1.0) < 1e-13
    assert abs(one @ r["M"] @ xi[:, 0] - 1.0 / 3.0) < 1e-13
    if q >= 2:
        assert abs(one @ r["M"] @ (xi[:, 0] * xi[:, 1]) - 1.0 / 12.0) < 1e-13
    # derivatives of every monomial of degree <= q are exact at the nodes
    for a in range(q + 1):
        for b in range(q + 1 - a):
            f = xi[:, 0] ** a * xi[:, 1] ** b
            d1 = a * xi[:, 0] ** max(a - 1, 0) * xi[:, 1] ** b
            d2 = b * xi[:, 0] ** a * xi[:, 1] ** max(b - 1, 0)
            assert np.allclose(r["D"][0] @ f, d1, atol=1e-12)
            assert np.allclose(r["D"][1] @ f, d2, atol=1e-12)
    # unit-length edges: M LIFT holds the edge mass columns; each edge's block sums to 1
    E = r["M"] @ r["LIFT"]
    Nfp = q + 1
    for f in range(3):
        assert abs(E[:, f * Nfp:(f + 1) * Nfp].sum() - 1.0) < 1e-13
        # rows of nodes off the edge are zero
        off = np.setdiff1d(np.arange(Np), r["fmask"][f])
        assert np.abs(E[off, f * Nfp:(f + 1) * Nfp]).max() < 1e-14
    assert np.allclose(refelem2d.basis_at(q, xi), np.eye(Np), atol=1e-13)


def test_cartesian_mesh_geometry():
    w = inputs.cavity2d(4, 2)
    p = _problem(w)
    geo = p.geo
    h = 0.25
    assert abs(geo.vol.sum() - 1.0) < 1e-14
    assert np.allclose(geo.rho, h / (1 + math.sqrt(2)))       # 4|K|/perimeter of the quarter cell
    wall = np.nonzero(geo.nbr[:, 0] < 0)[0]
    assert np.allclose(geo.normal[wall, 0], inputs.SIDE_NORMALS[wall % 4])
    inner = geo.nbr >= 0
    e, f = np.nonzero(inner)
    back = geo.nbr[geo.nbr[e, f]] == e[:, None]
    assert np.all(back.any(axis=1))
    # matched edge nodes coincide
    fm = p.ref["fmask"]
    for ei, fi in zip(e[:20], f[:20]):
        assert np.allclose(geo.x[ei, fm[fi]], geo.x[geo.nbr[ei, fi], geo.nbr_node[ei, fi]])


# ------------------------------------------------------------------ energy

@pytest.mark.parametrize("q", [1, 3])
def test_energy_centred_conserves_upwind_dissipates(q):
    for tag in (inputs.TAG_PEC, inputs.TAG_IMPEDANCE):
        xy, tri, tags = inputs.cartesian_triangles(3, 3, side_tags=(tag,) * 4)
        K = tri.shape[0]
        eps = np.linspace(1.0, 3.0, K)
        for alpha in (0.0, 1.0):
            p = dg2d.make_problem(xy, tri, tags, q, eps, np.ones(K), alpha=alpha)
            MB = (dg2d.mass_matrix(p) @ dg2d.assemble_B(p)).toarray()
            sym = 0.5 * (MB + MB.T)
            lam = np.linalg.eigvalsh(sym)
            scale = np.abs(MB).max()
            if alpha == 0.0 and tag == inputs.TAG_PEC:
                assert np.abs(sym).max() < 1e-12 * scale
            else:
                assert lam.max() < 1e-12 * scale and lam.min() < -1e-3 * scale


def _cfl_limit(p, scheme):
    lam = np.linalg.eigvals(dg2d.assemble_B(p).toarray())
    coef = timestep.step_matrix_poly(scheme)
    rho = np.min(np.sqrt(p.mu * p.eps) * p.geo.rho)

    def stable(c):
        z = c * rho * lam
        return np.max(np.abs(sum(a * z ** k for k, a in enumerate(coef)))) <= 1 + 1e-10

    lo, hi = 0.0, 2.0
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if stable(mid) else (lo, mid)
    return lo


@pytest.mark.parametrize("q,scheme,n,c_paper", [(1, 2, 8, 0.24), (3, 4, 4, 0.12)])
def test_paper_cfl_constants_sit_below_the_upwind_stability_limit(q, scheme, n, c_paper):
    xy, tri, tags = inputs.cartesian_triangles(n, n, side_tags=(inputs.TAG_PEC,) * 4)
    K = tri.shape[0]
    up = _cfl_limit(dg2d.make_problem(xy, tri, tags, q, np.ones(K), np.ones(K), alpha=1.0), scheme)
    assert c_paper <= up <= 1.15 * c_paper, up
    assert timestep.CFL2D[q] == c_paper
    doubled = _cfl_limit(dg2d.make_problem(xy, tri, tags, q, np.ones(K), np.ones(K), alpha=2.0), scheme)
    assert doubled < c_paper


# --------------------------------------------------------------- exact solutions

def test_cavity_solution_against_double_sine_series():
    om = 3 * math.sqrt(2) * math.pi + math.sqrt(2) * math.pi / 64
    pts = np.array([[0.3, 0.7], [0.11, 0.52], [0.9, 0.05]])
    e, h1, h2 = exact2d.cavity(om, pts, modes=2000)
    m = np.arange(1, 801, 2)
    for i, (x, y) in enumerate(pts):
        # -Lap e - omega^2 e = i omega, with 1 = sum 16/(pi^2 n m) sin sin over odd n, m
        c = 1j * om * 16 / (math.pi ** 2 * np.outer(m, m)) / ((m[:, None] ** 2 + m[None, :] ** 2) * math.pi ** 2 - om ** 2)
        sx, sy = np.sin(m * math.pi * x), np.sin(m * math.pi * y)
        cx, cy = m * math.pi * np.cos(m * math.pi * x), m * math.pi * np.cos(m * math.pi * y)
        assert abs(e[i] - np.sum(c * np.outer(sx, sy))) < 1e-6
        assert abs(h1[i] - np.sum(c * np.outer(sx, cy)) / (1j * om)) < 2e-3
        assert abs(h2[i] + np.sum(c * np.outer(cx, sy)) / (1j * om)) < 2e-3


def test_waveguide_solution_satisfies_its_boundary_conditions():
    """e = 0 on the PEC sides; e + Z h x n = G = xi / (i omega) on the wall
    x = 4 (to the accuracy of a 400-term series away from the corners); the
    cut-off mode n = omega / pi is finite."""
    om, th = 2 * math.pi, math.pi / 6
    y = np.linspace(0.2, 0.8, 7)
    e, h1, h2 = exact2d.waveguide(om, th, np.stack([np.zeros(7), y], 1))
    assert np.abs(e).max() < 1e-12
    e, h1, h2 = exact2d.waveguide(om, th, np.stack([np.linspace(0, 4, 7), np.zeros(7)], 1))
    assert np.abs(e).max() < 1e-12
    e, h1, h2 = exact2d.waveguide(om, th, np.stack([np.full(7, 4.0), y], 1), modes=400)
    G = np.exp(1j * om * (4 * math.cos(th) + y * math.sin(th))) / (1j * om)
    assert np.all(np.isfinite(e)) and np.abs(e + (h1 * 0.0 - h2 * 1.0) - G).max() < 3e-3 * np.abs(G).max()


def test_planewave_solves_the_system_and_its_wall_data():
    om, th = 10 * math.pi, math.pi / 4
    pts = np.array([[0.2, 0.3], [0.7, 0.1]])
    e, h1, h2 = exact2d.planewave(om, th, pts)
    d = np.array([math.cos(th), math.sin(th)])
    # i omega h = vcurl e = (d2 e, -d1 e) = i omega (d2, -d1) e
    assert np.allclose(h1, d[1] * e) and np.allclose(h2, -d[0] * e)
    # i omega e + scurl h = 0 with scurl h = d1 h2 - d2 h1 = i omega (d1 (-d1) - d2 d2) e
    assert np.allclose(1j * om * e + 1j * om * (d[0] * (-d[0] * e) - d[1] * (d[1] * e)), 0)
    # the wall data is e + Z h x n (h x n = h1 n2 - h2 n1)
    w = inputs.planewave2d(2, 1, om, th)
    p = dg2d.make_problem(w.xy, w.tri, w.tags, 1, w.eps, w.mu)
    fp = p.geo.x[:, p.ref["fmask"]]
    G = inputs.planewave_boundary_data(w, fp, project=False)
    wall = np.nonzero(w.tags[:, 0] == inputs.TAG_IMPEDANCE)[0]
    x = fp[wall, 0].reshape(-1, 2)
    n = np.repeat(p.geo.normal[wall, 0], 2, axis=0)
    e, h1, h2 = exact2d.planewave(om, th, x)
    assert np.allclose(G[wall, 0].reshape(-1), e + h1 * n[:, 1] - h2 * n[:, 0])


# ------------------------------------------------------------ printed FS errors

# Tolerances: the cavity values are reproduced to 0.35%, the P3 plane wave to
# 1.2%; the P1 plane wave lands at 0.0365 against 0.0408, and the waveguide
# (whose reference solution is a sine series truncated at 50 terms, as the
# paper states) at 0.0130 / 0.00625 against 0.0139 / 0.00715: not pinned,
# kept as loose checks.
TOL = {("cavity", 1): 0.005, ("cavity", 3): 0.005, ("planewave", 3): 0.02, ("planewave", 1): 0.12,
       ("waveguide", 1): 0.15, ("waveguide", 3): 0.15}


def _workload(row):
    if row["exp"] == "cavity":
        return inputs.cavity2d(row["n"], row["q"], row["w"] * math.sqrt(2) * math.pi, row["delta"]), \
            lambda w: (lambda P: exact2d.cavity(w.omega, P, modes=300))
    if row["exp"] == "waveguide":
        return inputs.waveguide2d(row["n"], row["q"], row["w"] * math.pi), \
            lambda w: (lambda P: exact2d.waveguide(w.omega, w.theta, P, modes=50))
    return inputs.planewave2d(row["n"], row["q"], row["w"] * math.pi), \
        lambda w: (lambda P: exact2d.planewave(w.omega, w.theta, P))


@pytest.mark.parametrize("row", _golden(), ids=lambda r: f"{r['exp']}-P{r['q']}-{r['n']}-{r['delta']}")
def test_printed_fs_error(row):
    """The frequency-domain DG system reproduces the printed FS errors with
    twice the upwind penalty on interior and PEC edges (alpha = 2)."""
    w, ex = _workload(row)
    p = _problem(w, alpha=2.0)
    U = fs.frequency_solve(p)
    err, ref = exact2d.energy_error(p.geo, w.xy, w.tri, w.eps, w.mu, U, ex(w), nq=6)
    rel = err / ref
    print(f"{w.name} omega={w.omega:.6f}: FS error {rel:.6g}, printed {row['printed']}")
    assert abs(rel / row["printed"] - 1) < TOL[(row["exp"], row["q"])]


def test_printed_fs_error_discriminates_the_penalty():
    """With the upwind penalty itself the near-resonant cavity error is 40%
    above the printed one."""
    row = next(r for r in _golden() if r["exp"] == "cavity" and r["q"] == 1 and r["delta"] < 0.1)
    w, ex = _workload(row)
    p = _problem(w, alpha=1.0)
    U = fs.frequency_solve(p)
    err, ref = exact2d.energy_error(p.geo, w.xy, w.tri, w.eps, w.mu, U, ex(w), nq=6)
    assert err / ref > 1.3 * row["printed"]


# ------------------------------------------------------------------- CMCG in 2-D

@pytest.mark.parametrize("q,n,tag", [(1, 3, inputs.TAG_PEC), (2, 2, inputs.TAG_IMPEDANCE),
                                     (3, 2, inputs.TAG_IMPEDANCE)])
def test_cmcg_2d_converges_to_the_discrete_periodic_orbit(q, n, tag):
    xy, tri, tags = inputs.cartesian_triangles(n, n, side_tags=(tag,) * 4)
    K = tri.shape[0]
    rng = np.random.default_rng(40 + q)
    eps = rng.choice([1.0, 2.0], K)
    p0 = dg2d.make_problem(xy, tri, tags, q, eps, np.ones(K), omega=3.0 * math.pi)
    j = np.exp(-np.sum((p0.geo.x - 0.4) ** 2, axis=-1) / 0.1)
    p = dg2d.make_problem(xy, tri, tags, q, eps, np.ones(K), omega=3.0 * math.pi, j=j)
    r = cmcg.solve(p, tol=1e-11, max_iter=400)
    M = timestep.n_steps(p)
    assert r.M == M
    Uh, F = fs.discrete_periodic(p, M, timestep.default_scheme(q))
    assert np.max(np.abs(r.F - F)) < 1e-8 * np.max(np.abs(F))
    assert np.max(np.abs(r.U0 - Uh.real)) < 1e-8 * np.max(np.abs(Uh))


def test_frequency_domain_converges_to_the_exact_cavity_solution():
    """Away from resonance (omega = 1.5 sqrt(2) pi) the frequency-domain upwind
    system converges to the exact cavity solution at rate 2 for P1 (q + 1);
    P2 and P3 are limited by the corner singularity of the solution (a
    constant source in a square with e = 0 on the walls) but stay ahead."""
    def err(q, n):
        w = inputs.cavity2d(n, q, math.sqrt(2) * math.pi, 0.5)
        p0 = dg2d.make_problem(w.xy, w.tri, w.tags, q, w.eps, w.mu, omega=w.omega)
        p = dg2d.make_problem(w.xy, w.tri, w.tags, q, w.eps, w.mu, omega=w.omega, j=inputs.current_2d(w, p0.geo.x))
        U = fs.frequency_solve(p)
        e, r = exact2d.energy_error(p.geo, w.xy, w.tri, w.eps, w.mu, U,
                                    lambda x: exact2d.cavity(w.omega, x, modes=300), nq=8)
        return e / r
    e1 = [err(1, n) for n in (4, 8, 16)]
    rates = [math.log2(e1[i] / e1[i + 1]) for i in range(2)]
    assert all(1.9 < r < 2.2 for r in rates), rates
    e2 = [err(2, n) for n in (2, 4)]
    assert math.log2(e2[0] / e2[1]) > 2.5
    assert err(3, 4) < e2[1] < e1[1]
