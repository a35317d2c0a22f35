"""Manufactured transport solution of Sec. 8.1 (Eq. eq:mms_psi) and its source.

psi = (alpha + Omega.beta + Omega Omega : Theta) / (4 pi) on [0,1]^2 with
delta = 1.25, zeta = 0.1, omega = 0.05; the source is obtained by substituting
psi in Eq. eq:transport (sigma_s = 0 here): q_d = Omega_d . grad psi_d + sigma_t psi_d.
"""
from __future__ import annotations

import numpy as np

DELTA, ZETA, OMEGA = 1.25, 0.1, 0.05


def _s(k, c, x, y):
    a = k * np.pi / (1.0 + 2.0 * c)
    sx, sy = np.sin(a * (x + c)), np.sin(a * (y + c))
    cx, cy = np.cos(a * (x + c)), np.cos(a * (y + c))
    return sx * sy, a * cx * sy, a * sx * cy


def fields(x, y):
    """alpha, beta (2), Theta (11, 12, 22) and their x/y derivatives."""
    al = np.sin(np.pi * x) * np.sin(np.pi * y) + DELTA
    alx = np.pi * np.cos(np.pi * x) * np.sin(np.pi * y)
    aly = np.pi * np.sin(np.pi * x) * np.cos(np.pi * y)
    s2, s2x, s2y = _s(2, OMEGA, x, y)
    s3, s3x, s3y = _s(3, ZETA, x, y)
    return dict(alpha=(al, alx, aly), beta=(s2, s2x, s2y), t11=(0.5 * s3, 0.5 * s3x, 0.5 * s3y),
                t12=(s2, s2x, s2y), t22=(0.25 * s3, 0.25 * s3x, 0.25 * s3y))


def psi(x, y, ox, oy):
    """value, d/dx, d/dy of the manufactured angular flux for direction (ox, oy)."""
    F = fields(x, y)
    out = []
    for k in range(3):
        v = (F["alpha"][k] + ox * F["beta"][k] + oy * F["beta"][k] + ox * ox * F["t11"][k]
             + 2.0 * ox * oy * F["t12"][k] + oy * oy * F["t22"][k])
        out.append(v / (4.0 * np.pi))
    return tuple(out)


def moments_closed_form(x, y):
    """phi, J, P of the manufactured solution from the paper's formulas (P_xy with factor 2/15)."""
    F = fields(x, y)
    al, b = F["alpha"][0], F["beta"][0]
    t11, t12, t22 = F["t11"][0], F["t12"][0], F["t22"][0]
    phi = al + (t11 + t22) / 3.0
    J = (b / 3.0, b / 3.0)
    P = (al / 3.0 + (3 * t11 + t22) / 15.0, 2.0 * t12 / 15.0, al / 3.0 + (t11 + 3 * t22) / 15.0)
    return phi, J, P


def attach(pr, vol_xy, bnd_xy, sigma_t=1.0):
    """Set q_dir at volume quadrature points and psi_bc at boundary points of problem pr."""
    nd = pr.n_dir
    qd = np.zeros((nd,) + vol_xy.shape[:2])
    bc = np.zeros((nd,) + bnd_xy.shape[:2])
    for d in range(nd):
        ox, oy = pr.omega[d]
        f, fx, fy = psi(vol_xy[..., 0], vol_xy[..., 1], ox, oy)
        qd[d] = ox * fx + oy * fy + sigma_t * f
        bc[d] = psi(bnd_xy[..., 0], bnd_xy[..., 1], ox, oy)[0]
    pr.q_dir = qd
    pr.psi_bc = bc
    return pr
