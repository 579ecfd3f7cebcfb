"""Exact solutions of the 2-D experiments and the relative energy-norm error
of Section 6 (error = ||U - U_h||_{eps,mu} / ||U||_{eps,mu}).

Time-harmonic TM system (Section 5.2.1): i omega eps e + sigma e + scurl h = j,
i omega mu h - vcurl e = 0, so h = vcurl e / (i omega mu) = (d2 e, -d1 e) /
(i omega mu), and with eps = mu = 1, sigma = 0: -Lap e - omega^2 e = i omega j.

* ``cavity``: PEC walls of (0,1)^2 (e = 0), j = 1.  Expanding in y,
  1 = sum over odd m of 4/(m pi) sin(m pi y), each mode e_m(x) sin(m pi y)
  solves -e_m'' + kappa^2 e_m = 4 i omega / (m pi), e_m(0) = e_m(1) = 0,
  kappa^2 = m^2 pi^2 - omega^2:  e_m = (f_m / kappa^2)(1 - cosh(kappa s) /
  cosh(kappa / 2)), s = x - 1/2 (cosines when kappa^2 < 0).  The series is
  summed to ``modes`` odd m.
* ``planewave``: e = exp(i omega d.x), d = (cos theta, sin theta), and from
  the second equation h = (sin theta, -cos theta) e.
* ``energy_error``: both norms by a collapsed Gauss-Legendre rule on every
  triangle (n x n points, exact for polynomials of degree 2n - 2 in each
  collapsed variable), the discrete field evaluated from its nodal values.
"""
from __future__ import annotations

import numpy as np

from . import refelem2d


def _profile(kappa2: float, s: np.ndarray):
    """c(s) = cosh(kappa s)/cosh(kappa/2) and c'(s), for |s| <= 1/2, evaluated
    without overflow (exponentials of non-positive arguments only)."""
    if kappa2 > 0:
        k = np.sqrt(kappa2)
        a = np.abs(s)
        c = np.exp(k * (a - 0.5)) * (1 + np.exp(-2 * k * a)) / (1 + np.exp(-k))
        dc = k * np.sign(s) * np.exp(k * (a - 0.5)) * (1 - np.exp(-2 * k * a)) / (1 + np.exp(-k))
        return c, dc
    k = np.sqrt(-kappa2)
    return np.cos(k * s) / np.cos(k / 2), -k * np.sin(k * s) / np.cos(k / 2)


def cavity(omega: float, pts: np.ndarray, modes: int = 500):
    """(e, h1, h2) of the PEC cavity with j = 1 at points [P, 2]."""
    x, y = pts[:, 0], pts[:, 1]
    s = x - 0.5
    e = np.zeros(len(x), dtype=np.complex128)
    dxe = np.zeros_like(e)
    dye = np.zeros_like(e)
    for i in range(modes):
        m = 2 * i + 1
        k2 = (m * np.pi) ** 2 - omega ** 2
        fm = 4j * omega / (m * np.pi)
        c, dc = _profile(k2, s)
        em = fm / k2 * (1.0 - c)
        dem = -fm / k2 * dc
        sy, cy = np.sin(m * np.pi * y), np.cos(m * np.pi * y)
        e += em * sy
        dxe += dem * sy
        dye += em * (m * np.pi) * cy
    return e, dye / (1j * omega), -dxe / (1j * omega)


def planewave(omega: float, theta: float, pts: np.ndarray):
    """(e, h1, h2) of the plane wave exp(i omega d.x) at points [P, 2]."""
    d = np.array([np.cos(theta), np.sin(theta)])
    e = np.exp(1j * omega * (pts @ d))
    return e, np.sin(theta) * e, -np.cos(theta) * e


def _collapsed_rule(n: int):
    a, wa = np.polynomial.legendre.leggauss(n)
    a, wa = (a + 1) / 2, wa / 2
    A, B = np.meshgrid(a, a, indexing="ij")
    WA, WB = np.meshgrid(wa, wa, indexing="ij")
    xi = np.stack([A.ravel(), (B * (1 - A)).ravel()], axis=1)
    w = (WA * WB * (1 - A)).ravel()        # sums to 1/2, the reference area
    return xi, w


def energy_error(geo, xy, tri, eps, mu, U_h: np.ndarray, exact, nq: int = 8):
    """(||U - U_h||, ||U||) in the (eps, mu) energy norm; U_h [K, 3, Np]
    complex nodal values, exact(points [P,2]) -> (e, h1, h2)."""
    xi, w = _collapsed_rule(nq)
    phi = refelem2d.basis_at(geo.q, xi)                    # [P, Np]
    v = np.asarray(xy)[np.asarray(tri)]
    Jm = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]], axis=2)
    pts = v[:, 0][:, None, :] + np.einsum("kab,pb->kpa", Jm, xi)   # [K, P, 2]
    K, P = pts.shape[:2]
    ex = exact(pts.reshape(-1, 2))
    ex = np.stack(ex, axis=1).reshape(K, P, 3)
    uh = np.einsum("pn,ecn->epc", phi, U_h)                # [K, P, 3]
    wt = (2 * geo.vol)[:, None] * w[None, :]               # physical weights
    coef = np.stack([eps, mu, mu], axis=1)[:, None, :]     # [K, 1, 3]
    err = np.sum(wt[..., None] * coef * np.abs(ex - uh) ** 2)
    ref = np.sum(wt[..., None] * coef * np.abs(ex) ** 2)
    return float(np.sqrt(err)), float(np.sqrt(ref))


def waveguide(omega: float, theta: float, pts: np.ndarray, modes: int = 50, robin: bool = True):
    """(e, h1, h2) of the half-open waveguide (0,4) x (0,1): PEC at y = 0, 1 and
    x = 0, impedance wall at x = 4 with data from xi = exp(i omega d.x),
    d = (cos theta, sin theta); eps = mu = Z = 1, j = 0.

    e = sum_n e_n(x) sin(n pi y), -e_n'' + kappa_n^2 e_n = 0, kappa_n^2 =
    n^2 pi^2 - omega^2, e_n(0) = 0, so e_n = A_n sinh(kappa_n x).  At x = 4 the
    impedance condition e + Z h x n = G reads e + d_x e / (i omega) = G; with
    ``robin`` the data xi is the Robin data of d_x e + i omega e (G = xi /
    (i omega)), else G = xi.  g_n are the sine coefficients of the data on the
    wall (Gauss-Legendre, 8 points per mode and at least 200, so that the
    highest mode is resolved); the series stops at ``modes`` terms."""
    x, y = pts[:, 0], pts[:, 1]
    sg, wg = np.polynomial.legendre.leggauss(max(200, 8 * modes))
    sg, wg = (sg + 1) / 2, wg / 2
    wall = np.exp(1j * omega * (4.0 * np.cos(theta) + sg * np.sin(theta)))
    e = np.zeros(len(x), dtype=np.complex128)
    dxe = np.zeros_like(e)
    dye = np.zeros_like(e)
    for n in range(1, modes + 1):
        gn = 2.0 * np.sum(wg * wall * np.sin(n * np.pi * sg))
        k = np.sqrt(complex((n * np.pi) ** 2 - omega ** 2))
        if k.real < 0:
            k = -k
        # d_x e_n(4) + i omega e_n(4) = g_n (Robin), or e_n(4) + d_x e_n(4) / (i omega) = g_n
        if not robin:
            gn = gn * 1j * omega
        if abs(k) < 1e-12:  # cut-off mode (n pi = omega): e_n is linear in x
            en = gn * x / (1 + 4j * omega)
            den_d = gn * np.ones_like(x) / (1 + 4j * omega)
        else:  # sinh(k x) / (k cosh 4k + i omega sinh 4k), scaled by e^{-4k}
            den = k * (1 + np.exp(-8 * k)) + 1j * omega * (1 - np.exp(-8 * k))
            en = gn * (np.exp(k * (x - 4)) - np.exp(-k * (x + 4))) / den
            den_d = gn * k * (np.exp(k * (x - 4)) + np.exp(-k * (x + 4))) / den
        sy, cy = np.sin(n * np.pi * y), np.cos(n * np.pi * y)
        e += en * sy
        dxe += den_d * sy
        dye += en * (n * np.pi) * cy
    return e, dye / (1j * omega), -dxe / (1j * omega)
