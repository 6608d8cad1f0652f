"""Closed-form fields the oracle is pinned to (TEST INFRASTRUCTURE ONLY).

Kuzmin disk (Sec. 3.1, from Binney & Tremaine): surface density
Sigma_K(R) = a M / (2 pi) (R^2 + a^2)^(-3/2), enclosed mass
M_K(R) = M (1 - a / sqrt(R^2 + a^2)).  Above the plane its Newtonian field is
that of a point mass M at (R, z) = (0, -a), below it that of one at (0, +a),
so Phi_N = -G M / sqrt(R^2 + (a + |z|)^2).  The disk has no curl field in
QUMOND, so the QUMOND field is exactly nu(|g_N|/a0) g_N and the potential is
the point-mass QUMOND potential evaluated at the distance from the image
point.  Exponential disk: Sigma = M / (2 pi Rd^2) exp(-R/Rd) with
M(<R) = M [1 - (1 + R/Rd) exp(-R/Rd)].
"""
from __future__ import annotations

import numpy as np

G_KPC = 4.300917270e-6
A0_KPC = 3600.0


def nu_closed(y):
    y = np.asarray(y, dtype=np.float64)
    return 0.5 + 0.5 * np.sqrt(1.0 + 4.0 / y)


def kuzmin_sigma(R, a, M):
    R = np.asarray(R, dtype=np.float64)
    return a * M / (2.0 * np.pi) * (R * R + a * a) ** -1.5


def kuzmin_enclosed(R, a, M):
    R = np.asarray(R, dtype=np.float64)
    return M * (1.0 - a / np.sqrt(R * R + a * a))


def kuzmin_image_distance(x, y, z, a):
    return np.sqrt(x * x + y * y + (a + np.abs(z)) ** 2)


def kuzmin_phi_newton(x, y, z, a, M, G=G_KPC):
    return -G * M / kuzmin_image_distance(x, y, z, a)


def kuzmin_g_newton(x, y, z, a, M, G=G_KPC):
    """Newtonian acceleration vector: toward (0,0,-a) above the plane, (0,0,+a) below."""
    x, y, z = (np.asarray(v, dtype=np.float64) for v in (x, y, z))
    zi = np.where(z >= 0.0, z + a, z - a)
    r = np.sqrt(x * x + y * y + zi * zi)
    c = -G * M / r ** 3
    return c * x, c * y, c * zi


def kuzmin_g_mond(x, y, z, a, M, G=G_KPC, a0=A0_KPC):
    gx, gy, gz = kuzmin_g_newton(x, y, z, a, M, G)
    gn = np.sqrt(gx * gx + gy * gy + gz * gz)
    v = nu_closed(gn / a0)
    return v * gx, v * gy, v * gz


def phi_point_mond_closed(r, G, M, a0):
    r = np.asarray(r, dtype=np.float64)
    GM = G * M
    return (-GM / (2.0 * r) - np.sqrt(GM) * np.sqrt(GM + 4.0 * a0 * r * r) / (2.0 * r)
            + np.sqrt(GM * a0) * np.arcsinh(2.0 * r * np.sqrt(a0 / GM)))


def kuzmin_phi_mond(x, y, z, a, M, G=G_KPC, a0=A0_KPC):
    return phi_point_mond_closed(kuzmin_image_distance(x, y, z, a), G, M, a0)


def kuzmin_vc2_newton(R, a, M, G=G_KPC):
    """Midplane v_c^2 = R |g_N,R| = G M R^2 (R^2 + a^2)^(-3/2)."""
    R = np.asarray(R, dtype=np.float64)
    return G * M * R * R * (R * R + a * a) ** -1.5


def kuzmin_vc2_mond(R, a, M, G=G_KPC, a0=A0_KPC):
    """Midplane QUMOND v_c^2 = R nu(|g_N,r|/a0) |g_N,R| with |g_N,r| = GM/(R^2+a^2)."""
    R = np.asarray(R, dtype=np.float64)
    gr = G * M / (R * R + a * a)
    return nu_closed(gr / a0) * kuzmin_vc2_newton(R, a, M, G)


def exp_enclosed(R, Rd, M):
    x = np.asarray(R, dtype=np.float64) / Rd
    return M * (1.0 - (1.0 + x) * np.exp(-x))
