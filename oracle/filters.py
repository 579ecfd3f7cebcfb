"""Period filters F U = (2/T) int_0^T U(t) e^{-i omega t} dt (the filtering
operator of Section 4.1; quadratures of Section 5.4).

* trapezoid rule, paired with RK2 (eq. of the RK2 filter);
* cubic-Hermite quadrature, paired with RK4: on [t_{m-1}, t_m] the field is
  interpolated by the cubic Hermite polynomial of (U_{m-1}, U_m, Phi_{m-1},
  Phi_m) and the product with e^{-i omega t} is integrated exactly.

Readings (the printed formulas are garbled): T = 2 pi / omega; the 2/T
prefactor of the definition is kept in both quadratures; the Hermite weights
carry the phase e^{-i omega t_{m-1}} of each sub-interval; p00/p01 take value
one at the left/right end point, p10/p11 slope one there.
"""
from __future__ import annotations

import numpy as np


def hermite_basis(s: np.ndarray, dt: float):
    """Cubic Hermite basis on [0, dt] at offsets s: (h00, h01, h10, h11)."""
    x = s / dt
    h00 = 1 - 3 * x ** 2 + 2 * x ** 3
    h01 = 3 * x ** 2 - 2 * x ** 3
    h10 = dt * (x - 2 * x ** 2 + x ** 3)
    h11 = dt * (x ** 3 - x ** 2)
    return h00, h01, h10, h11


def hermite_xi(omega: float, dt: float, npts: int = 16):
    """xi_ij = int_0^dt h_ij(s) e^{-i omega s} ds by Gauss-Legendre quadrature
    (16 points integrate the degree-3 x smooth integrand to rounding for
    omega dt << 1; avoids the cancellation of the closed form)."""
    xg, wg = np.polynomial.legendre.leggauss(npts)
    s = 0.5 * dt * (xg + 1.0)
    w = 0.5 * dt * wg
    ph = np.exp(-1j * omega * s)
    return tuple(np.sum(w * h * ph) for h in hermite_basis(s, dt))


def trapezoid(Us, omega: float, M: int):
    """(2/T)(dt/2) sum_{m=1}^{M} (U_{m-1} e^{-i w t_{m-1}} + U_m e^{-i w t_m}),
    t_m = m T / M, given the time levels Us = [U_0, ..., U_M]."""
    T = 2 * np.pi / omega
    dt = T / M
    acc = 0.0
    for m in range(1, M + 1):
        acc = acc + (2 / T) * (dt / 2) * (Us[m - 1] * np.exp(-1j * omega * (m - 1) * dt)
                                          + Us[m] * np.exp(-1j * omega * m * dt))
    return acc


def hermite(Us, Phis, omega: float, M: int):
    """(2/T) sum_{m=1}^{M} e^{-i w t_{m-1}} (xi00 U_{m-1} + xi01 U_m
    + xi10 Phi_{m-1} + xi11 Phi_m), given U_m and Phi_m = dU/dt at t_m."""
    T = 2 * np.pi / omega
    dt = T / M
    x00, x01, x10, x11 = hermite_xi(omega, dt)
    acc = 0.0
    for m in range(1, M + 1):
        acc = acc + (2 / T) * np.exp(-1j * omega * (m - 1) * dt) * (
            x00 * Us[m - 1] + x01 * Us[m] + x10 * Phis[m - 1] + x11 * Phis[m])
    return acc
