"""Diagnostics: conserved quantities (Remark 2.1), discrete norms and the G-norm
error of section 6.1 (def:discrete_Gerr).  Test infrastructure only."""
from __future__ import annotations

import numpy as np

from . import operators as op


def mass(eta, h, g):
    """m = integral of zeta = eta - h (Remark 2.1), grid sum times the cell size."""
    return float(np.sum(eta - h) * g.cell)


def energy(eta, u, h, grad_h, g):
    """E = 1/2 integral [zeta^2 + u . G u]  (Remark 2.1 prints the flat-bottom form
    zeta^2 + eta |u|^2 + eta^3 (div u)^2 / 3; u . G u is the weak form B[u, u]
    of section 3.1, which adds the bathymetry terms of the depth-integrated
    vertical kinetic energy)."""
    Gu = op.apply_G(eta, grad_h, u, g)
    zeta = eta - h
    return float(0.5 * (np.sum(zeta ** 2) + np.sum(u * Gu)) * g.cell)


def norm2(v, g):
    """Discrete 2-norm ||v||_{2,dx} (section 6.1)."""
    return float(np.sqrt(np.sum(v * v) * g.cell))


def g_error(Gmat, u, u_star, b):
    """epsilon(u) = ||u - u*||_{G} / ||b||_2 (def:discrete_Gerr); the grid cell
    factor cancels between numerator and denominator."""
    e = (u - u_star).ravel()
    return float(np.sqrt(e @ (Gmat @ e)) / np.sqrt(np.sum(b * b)))


def rel_l2(a, ref):
    """Relative L2 difference ||a - ref||_2 / ||ref||_2 (ref nonzero)."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.sqrt(np.sum(ref * ref))
    return float(np.sqrt(np.sum((a - ref) ** 2)) / den) if den > 0 else float(np.sqrt(np.sum(a * a)))


def field_errors(eta, U, u, eta_ref, U_ref, u_ref, h):
    """Relative L2 errors used for parity: zeta = eta - h (not eta, whose unit
    mean depth would hide errors), the velocity u (all components together) and
    U (all components together)."""
    return {"zeta": rel_l2(eta - h, eta_ref - h), "u": rel_l2(u, u_ref), "U": rel_l2(U, U_ref)}
