"""A manufactured time-harmonic solution of eq. (1.1) in a homogeneous
medium with eps = 2, mu = 3/2 (so Z = sqrt(mu / eps) != 1 and eps != mu),
used to pin the oracle's volume source, impedance boundary data and
convergence order.

Field (closed form, shifted sines so that no trace vanishes on the walls):
    e = (a sin pi(y+s0) sin pi(z+s1), b sin pi(x+s2) sin pi(z+s3),
         c sin pi(x+s4) sin pi(y+s5)).
Each component is independent of its own coordinate, so div e = 0 and
curl curl e = -lap e = 2 pi^2 e.  With i w mu h - curl e = 0 and
i w eps e + curl h = j (sigma = 0):
    h = curl e / (i w mu),   j = i (w eps - 2 pi^2 / (w mu)) e.
On the impedance walls the data is what the dissipative Silver-Mueller
condition E x n - Z H_tau = G gives for the exact fields.
"""
import numpy as np

from oracle import dg
from oracle import mesh as omesh
from oracle import refelem
from paper_2106_02858_amd import inputs

EPS, MU, OMEGA = 2.0, 1.5, 2 * np.pi
AMP = (1.0, -2.0, 1.5)
SHIFT = (0.3, 0.7, 0.2, 0.55, 0.1, 0.45)


def exact(x):
    """(e, h, j) at points x[..., 3], complex amplitudes."""
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    pi, s, c = np.pi, np.sin, np.cos
    a, b, cc = AMP
    s0, s1, s2, s3, s4, s5 = SHIFT
    e = np.stack([a * s(pi * (Y + s0)) * s(pi * (Z + s1)),
                  b * s(pi * (X + s2)) * s(pi * (Z + s3)),
                  cc * s(pi * (X + s4)) * s(pi * (Y + s5))], -1)
    # partial derivatives entering curl e
    de3_dy = cc * s(pi * (X + s4)) * pi * c(pi * (Y + s5))
    de2_dz = b * s(pi * (X + s2)) * pi * c(pi * (Z + s3))
    de1_dz = a * s(pi * (Y + s0)) * pi * c(pi * (Z + s1))
    de3_dx = cc * pi * c(pi * (X + s4)) * s(pi * (Y + s5))
    de2_dx = b * pi * c(pi * (X + s2)) * s(pi * (Z + s3))
    de1_dy = a * pi * c(pi * (Y + s0)) * s(pi * (Z + s1))
    curl_e = np.stack([de3_dy - de2_dz, de1_dz - de3_dx, de2_dx - de1_dy], -1)
    h = curl_e / (1j * OMEGA * MU)
    j = 1j * (OMEGA * EPS - 2 * pi ** 2 / (OMEGA * MU)) * e
    return e, h, j


def impedance_data(geo):
    """G = e x n - Z h_tau at the face nodes of impedance faces, [K,4,Nfp,3]."""
    fm = refelem.face_nodes(geo.q)
    xf = np.stack([geo.x[:, fm[f], :] for f in range(4)], axis=1)
    ef, hf, _ = exact(xf)
    n = np.broadcast_to(geo.normal[:, :, None, :], ef.shape)
    h_tau = hf - np.sum(hf * n, -1, keepdims=True) * n
    G = np.cross(ef, n) - np.sqrt(MU / EPS) * h_tau
    return np.where((geo.tag == omesh.TAG_IMPEDANCE)[:, :, None, None], G, 0.0)


def problem(n, q):
    """Impedance-walled Kuhn cube mesh n^3 x 6, the manufactured j and G.
    Returns (oracle problem, exact dof vector [K,6,Np] at the nodes)."""
    xyz, tet, tags = inputs.cube_mesh(n, inputs.TAG_IMPEDANCE)
    K = tet.shape[0]
    eps, mu = np.full(K, EPS), np.full(K, MU)
    geo_only = dg.make_problem(xyz, tet, tags, q, eps, mu, omega=OMEGA)
    e, h, j = exact(geo_only.geo.x)
    p = dg.make_problem(xyz, tet, tags, q, eps, mu, omega=OMEGA, j=j, g=impedance_data(geo_only.geo))
    ex = np.concatenate([np.transpose(e, (0, 2, 1)), np.transpose(h, (0, 2, 1))], axis=1)
    return p, ex
