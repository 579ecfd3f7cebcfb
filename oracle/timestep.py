"""Explicit Runge-Kutta time stepping and one-period propagators
(Section 5.3 RK2 / RK4 algorithms, CFL rule; Section 4.1.2 propagators).

* ``n_steps``: M = the smallest integer with T/M <= c_q min_K sqrt(mu_K eps_K)
  rho_K, T = 2 pi / omega, rho_K the insphere diameter.
* ``forward``: P_psi U0 (with source) or P U0 (without) over one period.
* ``backward``: P* W_T = S P S W_T, S flipping the magnetic sign (the
  remark after the backward propagator: same time stepping, H sign changed).
* optional on-the-fly filter accumulation (trapezoid with RK2, Hermite with
  RK4), computed from the current and the previous time level only.
"""
from __future__ import annotations

import numpy as np

from . import dg, dg2d
from . import filters

# CFL constants c_q for 3-D tetrahedra.  The paper's 2-D values are
# c_1 = 0.24 (RK2) and c_3 = 0.12 (RK4).  In 3-D the RK2/P1 limit measured on
# Kuhn cube meshes is 0.22-0.24, so c_1 = 0.20 is used; c_3 = 0.12 keeps its
# margin (limit >= 0.13); c_2 = 0.16 is a reading for P2 (limit ~0.20),
# which the paper does not run.
CFL = {1: 0.20, 2: 0.16, 3: 0.12}
# 2-D triangles: the paper's c_1 = 0.24 and c_3 = 0.12, rho_K the diameter of
# the inscribed circle; c_2 = 0.16 is a reading (the paper runs P1 and P3).
CFL2D = {1: 0.24, 2: 0.16, 3: 0.12}


def ops_of(p):
    """The DG module of a problem: 3-D (dg) or 2-D transverse magnetic (dg2d)."""
    return dg2d if getattr(p, "dim", 3) == 2 else dg


def default_scheme(q: int) -> int:
    """RK2 with P1, RK4 otherwise (P3 in the paper; P2 is a reading)."""
    return 2 if q == 1 else 4


def n_steps(p: dg.Problem, cfl: float | None = None) -> int:
    c = (CFL2D if getattr(p, "dim", 3) == 2 else CFL)[p.geo.q] if cfl is None else cfl
    T = 2 * np.pi / p.omega
    dtmax = c * np.min(np.sqrt(p.mu * p.eps) * p.geo.rho)
    M = int(np.ceil(T / dtmax))
    while T / M > dtmax:
        M += 1
    while M > 1 and T / (M - 1) <= dtmax:
        M -= 1
    return M


def rk2_step(p, t, U, dt, with_source):
    k1 = ops_of(p).phi(p, t, U, with_source)
    k2 = ops_of(p).phi(p, t + dt / 2, U + dt / 2 * k1, with_source)
    return U + dt * k2, k1


def rk4_step(p, t, U, dt, with_source):
    k1 = ops_of(p).phi(p, t, U, with_source)
    k2 = ops_of(p).phi(p, t + dt / 2, U + dt / 2 * k1, with_source)
    k3 = ops_of(p).phi(p, t + dt / 2, U + dt / 2 * k2, with_source)
    k4 = ops_of(p).phi(p, t + dt, U + dt * k3, with_source)
    return U + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4), k1


def forward(p: dg.Problem, U0: np.ndarray, M: int, scheme: int, with_source: bool,
            filt: bool = False):
    """Propagate U0 over one period T = 2 pi / omega in M steps.

    Returns U(T), and the filtered field (2/T) int U e^{-i omega t} dt when
    ``filt``; time levels t_m = m T / M."""
    T = 2 * np.pi / p.omega
    dt = T / M
    om = p.omega
    U = np.array(U0, dtype=np.float64, copy=True).reshape(p.K, p.ncomp, p.Np)
    step = rk2_step if scheme == 2 else rk4_step
    Us, Phis = [U], []
    for m in range(M):
        t = m * dt
        U, k1 = step(p, t, U, dt, with_source)
        if filt:
            Us.append(U)
            Phis.append(k1)  # k1 = Phi(t_m, U_m)
    if not filt:
        return U
    if scheme == 2:
        F = filters.trapezoid(Us, om, M)
    else:
        Phis.append(ops_of(p).phi(p, M * dt, U, with_source))
        F = filters.hermite(Us, Phis, om, M)
    return U, F


def backward(p: dg.Problem, WT: np.ndarray, M: int, scheme: int) -> np.ndarray:
    """P* W_T = S P S W_T (homogeneous)."""
    flip = ops_of(p).flip_H
    return flip(forward(p, flip(np.asarray(WT).reshape(p.K, p.ncomp, p.Np)), M, scheme, False))


def step_matrix_poly(scheme: int):
    """Coefficients (ascending) of the RK stability polynomial R(x)."""
    if scheme == 2:
        return [1.0, 1.0, 0.5]
    return [1.0, 1.0, 0.5, 1.0 / 6.0, 1.0 / 24.0]
