"""Limiting-amplitude ("full wave", FW) iteration, the method the numerical
examples (Section 6) compare CMCG against: plain time stepping with the
source from a zero (or given) state, one period after another.  The iterate
after l periods is the state U_0^(l) = P_psi^l U_0^(0); its time-harmonic
approximation is the filter F_psi U_0^(l), obtained while simulating the next
period.  Cost is counted in simulated periods, as in the paper.

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
    F: np.ndarray          # filtered field of the last simulated period (complex)
    U0: np.ndarray         # state at the start of that period
    U_end: np.ndarray      # state at its end
    history: list          # relative change of F per period (1 for the first)
    periods: int
    M: int


def rel_change(p: dg.Problem, F: np.ndarray, Fprev: np.ndarray) -> float:
    d = F - Fprev
    num = dg.inner(p, d.real, d.real) + dg.inner(p, d.imag, d.imag)
    den = dg.inner(p, F.real, F.real) + dg.inner(p, F.imag, F.imag)
    return float(np.sqrt(num / den)) if den > 0 else 0.0


def solve(p: dg.Problem, periods: int, tol: float = 0.0, M: int | None = None, scheme: int | None = None,
          u0=None) -> FwResult:
    """Simulate up to `periods` periods; stop early once the relative change
    of the filtered field between consecutive periods is at most `tol`."""
    if M is None:
        M = timestep.n_steps(p)
    if scheme is None:
        scheme = timestep.default_scheme(p.geo.q)
    U = np.zeros((p.K, 6, p.Np)) if u0 is None else np.array(u0, dtype=np.float64).reshape(p.K, 6, p.Np)
    hist, F, Fprev, start = [], None, None, U
    for l in range(periods):
        start = U
        U, F = timestep.forward(p, U, M, scheme, with_source=True, filt=True)
        hist.append(1.0 if Fprev is None else rel_change(p, F, Fprev))
        Fprev = F
        if tol > 0 and l > 0 and hist[-1] <= tol:
            break
    return FwResult(F, start, U, hist, len(hist), M)
