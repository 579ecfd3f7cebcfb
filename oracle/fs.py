"""Direct solves used as pins of the time-domain oracle.

* ``frequency_solve``: the frequency-domain DG system (i omega M + K) U = M JJ
  (the FS reference of Section 6), by sparse LU.
* ``discrete_periodic``: the exactly periodic orbit of the fully discrete
  scheme.  With z = e^{i omega dt}, R = R(dt B) the RK step polynomial and S
  the response of one complexified RK step from 0 to the forcing JJ e^{i omega
  t}, the orbit is U_m = Re(U^ z^m) with (z I - R) U^ = S.  Its U_0 is a zero
  of J, and the trapezoid filter returns U^ exactly; the Hermite filter returns
  (1/dt)[(xi00 + z xi01) U^ + (xi10 + z xi11)(B U^ + JJ)].
  (z I - R(x)) is factored over the roots of R(x) = z, so only shifted
  sparse LUs of B are needed.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import dg, timestep
from .timestep import ops_of
from .filters import hermite_xi


def frequency_solve(p: dg.Problem, B: sp.csr_matrix | None = None) -> np.ndarray:
    if B is None:
        B = ops_of(p).assemble_B(p)
    M = ops_of(p).mass_matrix(p)
    Kmat = -(M @ B)
    JJ = ops_of(p).source_vector(p)
    A = (1j * p.omega * M + Kmat).tocsc()
    U = spla.splu(A).solve(M @ JJ)
    return U.reshape(p.K, p.ncomp, p.Np)


def rk_forced_step(B, JJ, omega, dt, scheme):
    """One RK step from U=0 at t=0 of U' = B U + JJ e^{i omega t}."""
    f = lambda t: JJ * np.exp(1j * omega * t)
    if scheme == 2:
        k1 = f(0.0)
        k2 = B @ (dt / 2 * k1) + f(dt / 2)
        return dt * k2
    k1 = f(0.0)
    k2 = B @ (dt / 2 * k1) + f(dt / 2)
    k3 = B @ (dt / 2 * k2) + f(dt / 2)
    k4 = B @ (dt * k3) + f(dt)
    return dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)


def discrete_periodic(p: dg.Problem, M: int, scheme: int, B: sp.csr_matrix | None = None):
    """Returns (U_hat, filtered) for the exactly periodic discrete orbit."""
    if B is None:
        B = ops_of(p).assemble_B(p)
    B = B.tocsc().astype(np.complex128)
    n = B.shape[0]
    T = 2 * np.pi / p.omega
    dt = T / M
    z = np.exp(1j * p.omega * dt)
    JJ = ops_of(p).source_vector(p)
    S = rk_forced_step(B, JJ, p.omega, dt, scheme)
    # z - R(x) = c prod_k (x - r_k), x = dt B
    coef = timestep.step_matrix_poly(scheme)  # ascending
    poly = -np.array(coef[::-1], dtype=np.complex128)
    poly[-1] += z
    roots = np.roots(poly)
    c = poly[0]
    I = sp.identity(n, format="csc", dtype=np.complex128)
    x = S / c
    for r in roots:
        x = spla.splu((dt * B - r * I).tocsc()).solve(x)
    Uh = x
    if scheme == 2:
        F = Uh
    else:
        x00, x01, x10, x11 = hermite_xi(p.omega, dt)
        F = ((x00 + z * x01) * Uh + (x10 + z * x11) * (B @ Uh + JJ)) / dt
    return Uh.reshape(p.K, p.ncomp, p.Np), F.reshape(p.K, p.ncomp, p.Np)
