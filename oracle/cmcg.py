"""Controllability conjugate gradient (Section 2.2, Algorithms 1-3; gradient
and Hessian of the energy functional, Section 5.1).

J(U0) = 1/2 ||(I - P) U0 - G||^2_{eps,mu},  G = P_psi 0,
J'(U0) = (I - P*)(I - P) U0 - G*,  G* = (I - P*) G.

Readings of the printed algorithms (the theorem on the structure of J fixes
them): the gradient is W_0 - W_T - G* with W_T = P U0 - U0, W_0 = P* W_T;
with R the gradient the iterate moves against D, U0 <- U0 - alpha D; the new
direction uses the new residual, D <- R_new + beta D.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import dg, timestep


@dataclass
class Result:
    U0: np.ndarray               # periodic initial condition [K,6,Np]
    F: np.ndarray                # filtered complex field F_psi U0 [K,6,Np]
    iters: int
    rel_res: float
    M: int
    history: list = field(default_factory=list)   # ||R_l||/||R_0||
    J: list = field(default_factory=list)         # J by the CG recurrence


class Operators:
    """P, P*, P_psi for one problem and time discretisation.  lts = m > 1
    uses local time stepping (oracle.lts) with m substeps on the fine
    elements; M then counts coarse steps."""

    def __init__(self, p: dg.Problem, M: int | None = None, scheme: int | None = None,
                 cfl: float | None = None, lts: int = 1):
        self.p = p
        self.scheme = timestep.default_scheme(p.geo.q) if scheme is None else scheme
        self.lts = lts
        if lts > 1:
            from . import lts as olts
            M_lts, self.fine = olts.lts_steps(p, lts, cfl)
            self.M = M_lts if M is None else M
        else:
            self.M = timestep.n_steps(p, cfl) if M is None else M
        self.periods = 0

    def _fwd(self, U, src, filt=False):
        if self.lts > 1:
            from . import lts as olts
            return olts.forward(self.p, U, self.M, self.lts, self.fine, self.scheme, src, filt=filt)
        return timestep.forward(self.p, U, self.M, self.scheme, src, filt=filt)

    def P(self, U):
        self.periods += 1
        return self._fwd(U, False)

    def P_psi(self, U):
        self.periods += 1
        return self._fwd(U, True)

    def P_star(self, W):
        self.periods += 1
        if self.lts > 1:
            from . import lts as olts
            return olts.backward(self.p, W, self.M, self.lts, self.fine, self.scheme)
        return timestep.backward(self.p, W, self.M, self.scheme)

    def filtered(self, U):
        self.periods += 1
        return self._fwd(U, True, filt=True)[1]

    def ip(self, U, V):
        return float(timestep.ops_of(self.p).inner(self.p, U, V))


def initialise(ops: Operators):
    """Algorithm 1: G = P_psi 0, G_T = P* G, G* = G - G_T."""
    p = ops.p
    G = ops.P_psi(np.zeros((p.K, p.ncomp, p.Np)))
    GT = ops.P_star(G)
    return G, G - GT


def gradient(ops: Operators, U0, Gstar):
    """Algorithm 2: J'(U0) = W_0 - W_T - G*."""
    UT = ops.P(U0)
    WT = UT - U0
    W0 = ops.P_star(WT)
    return W0 - WT - Gstar


def hessian_apply(ops: Operators, D):
    """A = J'(D) + G* = (I - P*)(I - P) D."""
    UT = ops.P(D)
    WT = UT - D
    W0 = ops.P_star(WT)
    return W0 - WT


def functional(ops: Operators, U0, G):
    """J(U0) = 1/2 ||U0 - P U0 - G||^2 (costs one period)."""
    r = U0 - ops.P(U0) - G
    return 0.5 * ops.ip(r, r)


def solve(p: dg.Problem, tol: float = 1e-8, max_iter: int = 1000, u0=None, M=None,
          scheme=None, fixed_iters: int | None = None, cfl=None, filt: bool = True, runup: int = 0,
          lts: int = 1) -> Result:
    """Algorithm 3.  Stops when ||R_l|| <= tol ||R_0|| or after ``fixed_iters``
    iterations when that is given (used for parity at a fixed count).

    ``runup`` > 0: the run-up phase Section 6 mentions as an accelerator --
    that many limiting-amplitude periods U <- P_psi U from the initial guess
    (zero or u0) before the first residual; CG then starts from their state.
    ``lts`` = m > 1: local time stepping with m fine substeps (oracle.lts);
    the backward periods are the exact adjoint of the LTS forward period."""
    ops = Operators(p, M, scheme, cfl, lts)
    G, Gstar = initialise(ops)
    U = np.zeros((p.K, p.ncomp, p.Np)) if u0 is None else np.array(u0, dtype=np.float64).reshape(p.K, p.ncomp, p.Np)
    for _ in range(runup):
        U = ops.P_psi(U)
    if u0 is None and runup == 0:
        R = -Gstar
    else:
        R = gradient(ops, U, Gstar)
    D = R.copy()
    rr = ops.ip(R, R)
    rr0 = rr
    hist = [1.0]
    Jrec = [0.5 * ops.ip(G, G)] if u0 is None and runup == 0 else []
    it = 0
    limit = max_iter if fixed_iters is None else fixed_iters
    while it < limit:
        if fixed_iters is None and np.sqrt(rr) <= tol * np.sqrt(rr0):
            break
        A = hessian_apply(ops, D)
        dA = ops.ip(D, A)
        if not (dA > 0):
            raise FloatingPointError("CG breakdown: (D, A) <= 0")
        alpha = rr / dA
        U = U - alpha * D
        R = R - alpha * A
        rr_new = ops.ip(R, R)
        beta = rr_new / rr
        D = R + beta * D
        if Jrec:
            Jrec.append(Jrec[-1] - 0.5 * alpha * rr)
        rr = rr_new
        it += 1
        hist.append(float(np.sqrt(rr / rr0)))
    F = ops.filtered(U) if filt else None
    return Result(U, F, it, float(np.sqrt(rr / rr0)), ops.M, hist, Jrec)
