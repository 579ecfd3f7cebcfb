"""Local time stepping for locally refined meshes (the paper's concluding
remarks name it as the way to avoid the global CFL restriction of small
elements).  Test infrastructure: the plain FP64 form of the scheme the GPU
library implements; nothing here is used by the library.

Scheme (one coarse step of size H from t to t + H, m fine substeps of size
h = H / m): the Runge-Kutta-based local time stepping of Grote, Mehlin and
Mitkova (LTS-RK; SIAM J. Sci. Comput. 37 (2015)), written for the first-order
system y' = B y + F(t) of the DG discretisation (Section 5.2) with the RK2
midpoint / classical RK4 schemes of Section 5.3 as the base method:

* P is the diagonal projection onto the unknowns of the fine elements (those
  whose own CFL step is shorter than H), I - P onto the coarse ones;
* the solution's Taylor coefficients at t: y^(0) = y, y^(k+1) = B y^(k) +
  F^(k)(t) for k < p - 1 (p = 2 for RK2, 4 for RK4), with F^(k) the k-th
  time derivative of F(t) = Re(JJ e^{i omega t});
* the coarse unknowns' influence over the step is frozen into the
  polynomial w(tau) = sum_{k<p} tau^k / k! B (I - P) y^(k);
* z' = B P z + w(tau) + F(t + tau), z(0) = y, is integrated with m steps of
  the base RK scheme of size h; the step's result is z(H).

With no fine element (P = 0) the base RK method integrates the polynomial w
exactly, so the homogeneous step is sum_{k<=p} (H B)^k / k! y = R(H B) y: the
global RK step.  With every element fine (P = I) it is m global steps of
size h.  With m = 1 and RK2 it is the global midpoint step for any P.

The adjoint step (backward periods of Algorithm 2 need the exact adjoint of
the discrete propagator in the eps,mu inner product) runs the homogeneous
step's operations in reverse order with B* = S B S and P* = P.
"""
from __future__ import annotations

import math

import numpy as np

from . import timestep
from .timestep import ops_of


def element_steps(p, cfl: float | None = None) -> np.ndarray:
    """Each element's own CFL step c_q sqrt(mu_K eps_K) rho_K (Section 5.3)."""
    c = (timestep.CFL2D if getattr(p, "dim", 3) == 2 else timestep.CFL)[p.geo.q] if cfl is None else cfl
    return c * np.sqrt(p.mu * p.eps) * p.geo.rho


def lts_steps(p, m: int, cfl: float | None = None):
    """(M, fine): coarse steps per period and the fine-element mask for the
    substep ratio m.  H = T / M is the largest coarse step with H / m no longer
    than the smallest element step; an element is fine when its own step is
    shorter than H."""
    dts = element_steps(p, cfl)
    T = 2 * np.pi / p.omega
    hmax = float(np.min(dts))
    M = int(np.ceil(T / (m * hmax)))
    while T / (M * m) > hmax:
        M += 1
    while M > 1 and T / ((M - 1) * m) <= hmax:
        M -= 1
    H = T / M
    return M, dts < H


def _source_derivative(p, t: float, k: int) -> np.ndarray:
    """k-th time derivative of F(t) = Re(JJ e^{i w t}): Re((i w)^k JJ e^{i w t})
    = w^k F(t + k pi / (2 w))."""
    return p.omega ** k * ops_of(p).source(p, t + k * np.pi / (2 * p.omega))


def _mask(p, fine: np.ndarray) -> np.ndarray:
    return fine.astype(np.float64)[:, None, None]


def coarse_step(p, y: np.ndarray, t: float, H: float, m: int, fine: np.ndarray, scheme: int,
                with_source: bool, with_derivative: bool = False):
    """One LTS coarse step from t; returns y(t + H) (and, with
    with_derivative, y'(t) = B y + F(t), the derivative the Hermite filter
    uses at the step's start)."""
    B = lambda x: ops_of(p).apply_B(p, x)
    F = lambda tt: ops_of(p).source(p, tt)
    order = 2 if scheme == 2 else 4
    P = _mask(p, fine)
    ders = [y]
    for k in range(1, order):
        d = B(ders[-1])
        if with_source:
            d = d + _source_derivative(p, t, k - 1)
        ders.append(d)
    w = [B((1.0 - P) * d) for d in ders]

    def rhs(tau, z):
        r = B(P * z)
        for k, wk in enumerate(w):
            r = r + tau ** k / math.factorial(k) * wk
        if with_source:
            r = r + F(t + tau)
        return r

    h = H / m
    z = np.array(y, copy=True)
    for l in range(m):
        tau = l * h
        if scheme == 2:
            k1 = rhs(tau, z)
            k2 = rhs(tau + h / 2, z + h / 2 * k1)
            z = z + h * k2
        else:
            k1 = rhs(tau, z)
            k2 = rhs(tau + h / 2, z + h / 2 * k1)
            k3 = rhs(tau + h / 2, z + h / 2 * k2)
            k4 = rhs(tau + h, z + h * k3)
            z = z + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    if with_derivative:
        return z, ders[1] if order > 1 else None
    return z


def adjoint_step(p, zbar: np.ndarray, H: float, m: int, fine: np.ndarray, scheme: int) -> np.ndarray:
    """The eps,mu-adjoint of the homogeneous coarse step: its operations in
    reverse order, each transposed (B* = S B S, P* = P)."""
    flip = ops_of(p).flip_H
    Bs = lambda x: flip(ops_of(p).apply_B(p, flip(x)))
    order = 2 if scheme == 2 else 4
    P = _mask(p, fine)
    h = H / m
    zbar = np.array(zbar, copy=True)
    wbar = [np.zeros_like(zbar) for _ in range(order)]

    def rhs_bar(tau, kbar):
        """Adjoint of r = B P z + sum_k tau^k/k! w_k: returns zbar part,
        accumulates wbar."""
        for k in range(order):
            wbar[k] += tau ** k / math.factorial(k) * kbar
        return P * Bs(kbar)

    for l in reversed(range(m)):
        tau = l * h
        if scheme == 2:
            # z1 = z + h k2, k2 = r(tau + h/2, zm), zm = z + h/2 k1, k1 = r(tau, z)
            k2b = h * zbar
            zmb = rhs_bar(tau + h / 2, k2b)
            zbar = zbar + zmb
            k1b = h / 2 * zmb
            zbar = zbar + rhs_bar(tau, k1b)
        else:
            # z1 = z + h/6 (k1 + 2 k2 + 2 k3 + k4); k4 = r(tau + h, z + h k3);
            # k3 = r(tau + h/2, z + h/2 k2); k2 = r(tau + h/2, z + h/2 k1); k1 = r(tau, z)
            k1b = h / 6 * zbar
            k2b = h / 3 * zbar
            k3b = h / 3 * zbar
            k4b = h / 6 * zbar
            a4 = rhs_bar(tau + h, k4b)       # adjoint of the argument z + h k3
            zbar = zbar + a4
            k3b = k3b + h * a4
            a3 = rhs_bar(tau + h / 2, k3b)   # argument z + h/2 k2
            zbar = zbar + a3
            k2b = k2b + h / 2 * a3
            a2 = rhs_bar(tau + h / 2, k2b)   # argument z + h/2 k1
            zbar = zbar + a2
            k1b = k1b + h / 2 * a2
            zbar = zbar + rhs_bar(tau, k1b)  # argument z
    # w_k = B (I - P) y^(k);  y^(k+1) = B y^(k);  y^(0) = y
    ybar = zbar
    dbar = [None] * order
    for k in range(order):
        dbar[k] = (1.0 - P) * Bs(wbar[k])
    for k in reversed(range(1, order)):
        dbar[k - 1] = dbar[k - 1] + Bs(dbar[k])
    return ybar + dbar[0]


def forward(p, U0: np.ndarray, M: int, m: int, fine: np.ndarray, scheme: int, with_source: bool,
            filt: bool = False):
    """One period T = 2 pi / omega of M coarse LTS steps (the library's
    P_psi / P with local time stepping); with filt also the filtered field of
    Section 5.4 from the coarse time levels (trapezoid with RK2, cubic Hermite
    with the derivatives y'(t_m) = B U_m + F(t_m) with RK4)."""
    from . import filters
    T = 2 * np.pi / p.omega
    H = T / M
    U = np.array(U0, dtype=np.float64, copy=True).reshape(p.K, p.ncomp, p.Np)
    Us, Phis = [U], []
    for n in range(M):
        U, d = coarse_step(p, U, n * H, H, m, fine, scheme, with_source, with_derivative=True)
        if filt:
            Us.append(U)
            Phis.append(d)
    if not filt:
        return U
    if scheme == 2:
        return U, filters.trapezoid(Us, p.omega, M)
    Phis.append(ops_of(p).phi(p, M * H, U, with_source))
    return U, filters.hermite(Us, Phis, p.omega, M)


def backward(p, WT: np.ndarray, M: int, m: int, fine: np.ndarray, scheme: int) -> np.ndarray:
    """The adjoint of the homogeneous LTS period, P* (Algorithm 2's backward
    period): M adjoint coarse steps."""
    T = 2 * np.pi / p.omega
    H = T / M
    W = np.array(WT, dtype=np.float64, copy=True).reshape(p.K, p.ncomp, p.Np)
    for _ in range(M):
        W = adjoint_step(p, W, H, m, fine, scheme)
    return W
