"""Limiting-amplitude ("full wave", FW) iteration, the method the numerical
examples (Section 6) compare CMCG against: plain time stepping with the
source from a zero (or given) state, one period after another.  The iterate
after l periods is the state U_0^(l) = P_psi^l U_0^(0); its time-harmonic
approximation is the filter F_psi U_0^(l), obtained by simulating one more
period with the filter.  Cost is counted in simulated periods, as in the
paper.

Test infrastructure only (see oracle/__init__.py).  Pinned in
tests/test_oracle_fw.py against the exactly periodic discrete orbit (fs) and
the homogeneous propagator: U_0^(l) = U* + P^l (U_0^(0) - U*).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import dg, timestep


@dataclass
class FwResult:
    F: np.ndarray          # filtered field F_psi U0 of the final period (complex)
    U0: np.ndarray         # the iterate: state at the start of the final period
    U_end: np.ndarray      # state at its end
    history: list          # relative change of the state, one entry per plain period
    periods: int           # periods simulated, the filtered one included
    M: int


def rel_change(p: dg.Problem, F: np.ndarray, Fprev: np.ndarray) -> float:
    """||F - Fprev|| / ||F|| in the eps-mu norm (real or complex fields)."""
    d = F - Fprev
    num = timestep.ops_of(p).inner(p, d.real, d.real) + timestep.ops_of(p).inner(p, np.imag(d), np.imag(d))
    den = timestep.ops_of(p).inner(p, F.real, F.real) + timestep.ops_of(p).inner(p, np.imag(F), np.imag(F))
    return float(np.sqrt(num / den)) if den > 0 else 0.0


def solve(p: dg.Problem, periods: int, tol: float = 0.0, M: int | None = None, scheme: int | None = None,
          u0=None) -> FwResult:
    """At most periods - 1 plain periods with the source (stopping early once
    the state at a period start changes by at most `tol` relative to the
    previous one), then one period with the filter from the last state; the
    approximation after l plain periods is F_psi U_0^(l)."""
    if M is None:
        M = timestep.n_steps(p)
    if scheme is None:
        scheme = timestep.default_scheme(p.geo.q)
    U = np.zeros((p.K, p.ncomp, p.Np)) if u0 is None else np.array(u0, dtype=np.float64).reshape(p.K, p.ncomp, p.Np)
    hist = []
    for _ in range(periods - 1):
        Un = timestep.forward(p, U, M, scheme, with_source=True)
        hist.append(rel_change(p, Un, U))
        U = Un
        if tol > 0 and hist[-1] <= tol:
            break
    U_end, F = timestep.forward(p, U, M, scheme, with_source=True, filt=True)
    return FwResult(F, U, U_end, hist, len(hist) + 1, M)
