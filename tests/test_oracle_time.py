"""Pins of the oracle's time stepping, propagators and filters.

* one period of RK2 / RK4 against the matrix exponential of T B (dense), with
  error ratios 4 and 16 under step halving;
* adjoint identity (P x, y)_M = (x, P* y)_M (lemma on dual propagators);
* the affine split P_psi U = P U + P_psi 0;
* stability: spectral radius of R(dt B) <= 1 at the CFL constants in use,
  and energy decay over many periods with zero source;
* Hermite weights against an independent power series; the Hermite filter is
  exact on cubic-in-time data; the trapezoid filter returns U^ exactly for
  U_m = Re(U^ z^m).
"""
import numpy as np
import pytest
import scipy.linalg as sl

from oracle import dg, filters, timestep
from tests._problems import hetero_problem


@pytest.mark.parametrize("q,scheme,ratio", [(1, 2, 4.0), (2, 4, 16.0)])
def test_period_against_expm(q, scheme, ratio):
    p = hetero_problem(n=1, q=q, seed=2, source=False)
    B = dg.assemble_B(p).toarray()
    T = 2 * np.pi / p.omega
    x = np.random.default_rng(0).standard_normal(p.ndof)
    exact = sl.expm(T * B) @ x
    M0 = 3 * timestep.n_steps(p)
    errs = []
    for M in (M0, 2 * M0, 4 * M0):
        y = timestep.forward(p, x.reshape(p.K, 6, p.Np), M, scheme, False).ravel()
        errs.append(np.linalg.norm(y - exact))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert abs(r1 / ratio - 1) < 0.15 and abs(r2 / ratio - 1) < 0.15, (errs, r1, r2)


@pytest.mark.parametrize("q", [1, 2, 3])
def test_adjoint_identity(q):
    p = hetero_problem(n=2 if q < 3 else 1, q=q, seed=20 + q, source=False)
    M = timestep.n_steps(p)
    sch = timestep.default_scheme(q)
    rng = np.random.default_rng(q)
    x = rng.standard_normal((p.K, 6, p.Np))
    y = rng.standard_normal((p.K, 6, p.Np))
    lhs = dg.inner(p, timestep.forward(p, x, M, sch, False), y)
    rhs = dg.inner(p, x, timestep.backward(p, y, M, sch))
    assert abs(lhs - rhs) <= 1e-13 * dg.norm(p, x) * dg.norm(p, y)


def test_affine_split():
    p = hetero_problem(n=2, q=2, seed=4, g=True)
    M = timestep.n_steps(p)
    x = np.random.default_rng(3).standard_normal((p.K, 6, p.Np))
    a = timestep.forward(p, x, M, 4, True)
    b = timestep.forward(p, x, M, 4, False) + timestep.forward(p, np.zeros_like(x), M, 4, True)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


@pytest.mark.parametrize("q,n,tag", [(1, 2, 2), (1, 2, 1), (2, 2, 2), (3, 1, 2), (3, 1, 1)])
def test_cfl_spectral_radius(q, n, tag):
    from paper_2106_02858_amd import inputs
    w = inputs.plain_fp64(n=n, q=q, boundary_tag=tag)
    p = dg.make_problem(w.xyz, w.tet, w.tags, q, w.eps, w.mu, omega=w.omega)
    lam = sl.eigvals(dg.assemble_B(p).toarray())
    dt = 2 * np.pi / p.omega / timestep.n_steps(p)
    c = np.array(timestep.step_matrix_poly(timestep.default_scheme(q)))
    amp = np.max(np.abs(np.polyval(c[::-1], dt * lam)))
    assert amp <= 1 + 1e-12
    assert np.max(lam.real) <= 1e-12 * np.max(np.abs(lam))


def test_energy_decay_zero_source():
    p = hetero_problem(n=2, q=1, seed=9, source=False)
    M = timestep.n_steps(p)
    U = np.random.default_rng(5).standard_normal((p.K, 6, p.Np))
    e = [dg.energy(p, U)]
    for _ in range(20):
        U = timestep.forward(p, U, M, 2, False)
        e.append(dg.energy(p, U))
    assert np.all(np.diff(e) <= 0)


def test_central_pec_rk4_energy_per_step():
    """Centred flux + PEC: B is M-skew, so |R(dt lam)| <= 1 for RK4 below
    2 sqrt 2 and the energy cannot grow."""
    from paper_2106_02858_amd import inputs
    p = hetero_problem(n=2, q=1, seed=6, alpha=0.0, sigma=False, tags=inputs.TAG_PEC, source=False)
    M = timestep.n_steps(p)
    dt = 2 * np.pi / p.omega / M
    U = np.random.default_rng(8).standard_normal((p.K, 6, p.Np))
    e0 = dg.energy(p, U)
    for m in range(3 * M):
        U, _ = timestep.rk4_step(p, m * dt, U, dt, False)
        e1 = dg.energy(p, U)
        assert e1 <= e0 * (1 + 1e-13)
        e0 = e1


def _xi_series(omega, dt, nterms=40):
    """int_0^dt h_ij(s) e^{-i w s} ds from the power series of the exponential:
    int_0^dt s^k e^{-i w s} ds = sum_n (-i w)^n dt^(n+k+1) / (n! (n+k+1))."""
    from math import factorial

    def mom(k):
        return sum((-1j * omega) ** n * dt ** (n + k + 1) / (factorial(n) * (n + k + 1)) for n in range(nterms))

    m = [mom(k) for k in range(4)]
    # h00 = 1 - 3 s^2/dt^2 + 2 s^3/dt^3 ...
    h00 = m[0] - 3 * m[2] / dt ** 2 + 2 * m[3] / dt ** 3
    h01 = 3 * m[2] / dt ** 2 - 2 * m[3] / dt ** 3
    h10 = m[1] - 2 * m[2] / dt + m[3] / dt ** 2
    h11 = m[3] / dt ** 2 - m[2] / dt
    return h00, h01, h10, h11


@pytest.mark.parametrize("theta", [1e-3, 0.03, 0.3, 1.0])
def test_hermite_weights_series(theta):
    omega, dt = 4 * np.pi, theta / (4 * np.pi)
    a = filters.hermite_xi(omega, dt)
    b = _xi_series(omega, dt)
    for x, y in zip(a, b):
        assert abs(x - y) <= 1e-15 * dt


def test_hermite_filter_exact_on_cubics():
    omega = 3.0
    T = 2 * np.pi / omega
    c = np.array([0.7, -1.3, 2.1, 0.4])  # P(t) = sum c_k t^k
    M = 7
    t = np.arange(M + 1) * T / M
    Us = [np.array([np.polyval(c[::-1], tt)]) for tt in t]
    dc = np.array([c[1], 2 * c[2], 3 * c[3]])
    Ps = [np.array([np.polyval(dc[::-1], tt)]) for tt in t]
    # exact (2/T) int_0^T t^k e^{-i w t} dt, with e^{-i w T} = 1:
    # I_0 = 0, I_k = T^k / (-i w) + k/(i w) I_{k-1}
    I = [0.0]
    for k in range(1, 4):
        I.append(T ** k / (-1j * omega) + k / (1j * omega) * I[-1])
    exact = (2 / T) * sum(ck * Ik for ck, Ik in zip(c, I))
    got = filters.hermite(Us, Ps, omega, M)[0]
    assert abs(got - exact) < 1e-13


@pytest.mark.parametrize("M", [3, 5, 64])
def test_trapezoid_exact_on_discrete_harmonic(M):
    omega = 2.5
    dt = 2 * np.pi / omega / M
    z = np.exp(1j * omega * dt)
    rng = np.random.default_rng(M)
    Uh = rng.standard_normal(11) + 1j * rng.standard_normal(11)
    Us = [np.real(Uh * z ** m) for m in range(M + 1)]
    got = filters.trapezoid(Us, omega, M)
    assert np.max(np.abs(got - Uh)) < 1e-14 * M
    # a static field is filtered to zero
    const = [np.ones(3)] * (M + 1)
    assert np.max(np.abs(filters.trapezoid(const, omega, M))) < 1e-14 * M
