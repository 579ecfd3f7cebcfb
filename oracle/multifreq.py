"""Several frequencies in one solve: a source made of harmonics of a base
frequency omega0, J(t) = sum_h Re(j_h e^{i k_h omega0 t}) with distinct
integers k_h >= 1, is periodic with T = 2 pi / omega0, so one CMCG solve over
that period (Algorithms 1-3) gives the periodic solution, and the filter at
each frequency k_h omega0, F_h = (2/T) int_0^T U(t) e^{-i k_h omega0 t} dt,
extracts that harmonic (the concluding remarks of the paper mention this
use; the method is the same CG with a different right-hand side).

Test infrastructure only (see oracle/__init__.py).  Pinned in
tests/test_oracle_multifreq.py: every filtered harmonic equals the exactly
periodic discrete orbit of that harmonic alone at the same time step.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import cmcg, dg, timestep
from .timestep import ops_of
from .filters import hermite_xi


@dataclass
class MultiProblem:
    base: dg.Problem          # mesh and media, omega = omega0, no source (3-D or 2-D TM)
    ks: list                  # harmonic numbers k_h
    harm: list                # problem per harmonic: omega = k_h omega0, its j_h

    @property
    def omega0(self):
        return self.base.omega


def make(base: dg.Problem, ks, js) -> MultiProblem:
    harm = [type(base)(base.geo, base.ref, base.eps, base.mu, base.sigma, k * base.omega, np.asarray(j), None,
                       base.alpha) for k, j in zip(ks, js)]
    return MultiProblem(base, list(ks), harm)


def phi(mp: MultiProblem, t: float, U: np.ndarray, with_source: bool) -> np.ndarray:
    r = ops_of(mp.base).apply_B(mp.base, U)
    if with_source:
        for ph in mp.harm:
            r = r + ops_of(ph).source(ph, t)
    return r


def forward(mp: MultiProblem, U0, M: int, scheme: int, with_source: bool, filt: bool = False):
    """One period T = 2 pi / omega0 in M steps; with ``filt`` also the
    filtered field of every harmonic (trapezoid for RK2, Hermite for RK4)."""
    T = 2 * np.pi / mp.omega0
    dt = T / M
    U = np.array(U0, dtype=np.float64, copy=True).reshape(mp.base.K, mp.base.ncomp, mp.base.Np)
    Us, Phis = [U], []
    for m in range(M):
        t = m * dt
        k1 = phi(mp, t, U, with_source)
        if scheme == 2:
            k2 = phi(mp, t + dt / 2, U + dt / 2 * k1, with_source)
            U = U + dt * k2
        else:
            k2 = phi(mp, t + dt / 2, U + dt / 2 * k1, with_source)
            k3 = phi(mp, t + dt / 2, U + dt / 2 * k2, with_source)
            k4 = phi(mp, t + dt, U + dt * k3, with_source)
            U = U + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        if filt:
            Us.append(U)
            Phis.append(k1)
    if not filt:
        return U
    Fs = []
    for k in mp.ks:
        w = k * mp.omega0
        acc = 0.0
        if scheme == 2:
            for m in range(1, M + 1):
                acc = acc + (2 / T) * (dt / 2) * (Us[m - 1] * np.exp(-1j * w * (m - 1) * dt)
                                                  + Us[m] * np.exp(-1j * w * m * dt))
        else:
            if len(Phis) == M:
                Phis.append(phi(mp, M * dt, U, with_source))
            x00, x01, x10, x11 = hermite_xi(w, dt)
            for m in range(1, M + 1):
                acc = acc + (2 / T) * np.exp(-1j * w * (m - 1) * dt) * (
                    x00 * Us[m - 1] + x01 * Us[m] + x10 * Phis[m - 1] + x11 * Phis[m])
        Fs.append(acc)
    return U, Fs


@dataclass
class MultiResult:
    U0: np.ndarray
    Fs: list
    iters: int
    rel_res: float
    M: int
    history: list


def solve(mp: MultiProblem, tol: float = 1e-8, max_iter: int = 1000, M: int | None = None,
          scheme: int | None = None, fixed_iters: int | None = None) -> MultiResult:
    """Algorithms 1-3 over the base period; the source enters through
    G = P_psi 0 (Algorithm 1) and the final filtered period only."""
    ops = cmcg.Operators(mp.base, M, scheme)
    M, scheme = ops.M, ops.scheme
    G = forward(mp, np.zeros((mp.base.K, mp.base.ncomp, mp.base.Np)), M, scheme, True)
    Gstar = G - ops.P_star(G)
    U = np.zeros_like(G)
    R = -Gstar
    D = R.copy()
    rr = rr0 = ops.ip(R, R)
    hist, it = [1.0], 0
    limit = max_iter if fixed_iters is None else fixed_iters
    while it < limit:
        if fixed_iters is None and np.sqrt(rr) <= tol * np.sqrt(rr0):
            break
        A = cmcg.hessian_apply(ops, D)
        alpha = rr / ops.ip(D, A)
        U = U - alpha * D
        R = R - alpha * A
        rr_new = ops.ip(R, R)
        D = R + (rr_new / rr) * D
        rr = rr_new
        it += 1
        hist.append(float(np.sqrt(rr / rr0)))
    _, Fs = forward(mp, U, M, scheme, True, filt=True)
    return MultiResult(U, Fs, it, float(np.sqrt(rr / rr0)), M, hist)
