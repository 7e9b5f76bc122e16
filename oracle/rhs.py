"""Right-hand side f(w, p) of the constraint form (Eq:DSWEcf, Eq:DAE_DSWE).

    eta_t = -div(eta u)
    U_t   = -eta grad(zeta) - div(eta u (x) u) + F(eta, u, h),   zeta = eta - h

with the forcing F of Def:bigF written as F = grad S - grad(h) T, where
(delta = div u, m = div(eta u), beta = grad h . u, P = u.grad(delta) - delta^2,
 Q = (u.grad)^2 h):

    S = eta^3/3 P + eta^2 m delta + eta^2/2 Q + eta m beta
    T = eta^2/2 P + eta m delta + eta Q + m beta

Reading of (u.grad)^2 h (Eq:defGF): the operator (u.grad) applied twice,
Q = u.grad(u.grad h) = u.grad(beta); with h time independent this is the
material derivative of the bottom normal flux, the term that pairs with
u_t.grad h in F of Eq:defGF.  Every derivative is the spectral one
(section 6.1).  Test infrastructure only.
"""
from __future__ import annotations

import numpy as np

from . import spectral as sp


def rhs(eta, u, h, grad_h, g):
    """Return (eta_t, U_t) for total depth eta, velocity u (d, ...), bathymetry h."""
    delta = sp.div(u, g)
    m = sp.div(eta[None] * u, g)
    beta = np.sum(grad_h * u, axis=0)
    grad_delta = sp.grad(delta, g)
    P = np.sum(u * grad_delta, axis=0) - delta ** 2
    Q = np.sum(u * sp.grad(beta, g), axis=0)
    S = eta ** 3 / 3.0 * P + eta ** 2 * m * delta + eta ** 2 / 2.0 * Q + eta * m * beta
    T = eta ** 2 / 2.0 * P + eta * m * delta + eta * Q + m * beta
    F = sp.grad(S, g) - grad_h * T[None]
    zeta = eta - h
    grad_zeta = sp.grad(zeta, g)
    # div(eta u (x) u), component i = sum_j d_j (eta u_i u_j)
    if g.d == 1:
        flux = sp.dx(eta * u[0] * u[0], g)[None]
    else:
        flux = np.stack([
            sp.dx(eta * u[0] * u[0], g) + sp.dy(eta * u[0] * u[1], g),
            sp.dx(eta * u[0] * u[1], g) + sp.dy(eta * u[1] * u[1], g),
        ])
    eta_t = -m
    U_t = -eta[None] * grad_zeta - flux + F
    return eta_t, U_t


def rhs_hessian_reading(eta, u, h, grad_h, g):
    """The same right-hand side with the other reading of (u.grad)^2 h,
    Q = u_i u_j d_i d_j h (Hessian form).  Kept only so a test can show which
    reading conserves the energy of Remark 2.1 over bathymetry."""
    delta = sp.div(u, g)
    m = sp.div(eta[None] * u, g)
    beta = np.sum(grad_h * u, axis=0)
    P = np.sum(u * sp.grad(delta, g), axis=0) - delta ** 2
    if g.d == 1:
        Q = u[0] * u[0] * sp.dx(grad_h[0], g)
    else:
        hxx = sp.dx(grad_h[0], g)
        hxy = sp.dy(grad_h[0], g)
        hyy = sp.dy(grad_h[1], g)
        Q = u[0] * u[0] * hxx + 2 * u[0] * u[1] * hxy + u[1] * u[1] * hyy
    S = eta ** 3 / 3.0 * P + eta ** 2 * m * delta + eta ** 2 / 2.0 * Q + eta * m * beta
    T = eta ** 2 / 2.0 * P + eta * m * delta + eta * Q + m * beta
    F = sp.grad(S, g) - grad_h * T[None]
    zeta = eta - h
    if g.d == 1:
        flux = sp.dx(eta * u[0] * u[0], g)[None]
    else:
        flux = np.stack([
            sp.dx(eta * u[0] * u[0], g) + sp.dy(eta * u[0] * u[1], g),
            sp.dx(eta * u[0] * u[1], g) + sp.dy(eta * u[1] * u[1], g),
        ])
    return -m, -eta[None] * sp.grad(zeta, g) - flux + F


def momentum_rhs(eta, u, h, grad_h, g):
    """Right-hand side of the eta-multiplied momentum equation (Eq:MomEq) without
    the G u_t term:  G u_t = -eta u.grad u - eta grad zeta + grad{eta^3/3 P + eta^2/2 Q}
                             - eta {eta/2 P + Q} grad h.
    Used only to cross-check F (Def:bigF) through the commutation
    U_t = G u_t + (d/dt G) u of section 2.2."""
    delta = sp.div(u, g)
    beta = np.sum(grad_h * u, axis=0)
    P = np.sum(u * sp.grad(delta, g), axis=0) - delta ** 2
    Q = np.sum(u * sp.grad(beta, g), axis=0)
    if g.d == 1:
        adv = (u[0] * sp.dx(u[0], g))[None]
    else:
        adv = np.stack([u[0] * sp.dx(u[0], g) + u[1] * sp.dy(u[0], g),
                        u[0] * sp.dx(u[1], g) + u[1] * sp.dy(u[1], g)])
    zeta = eta - h
    return (-eta[None] * adv - eta[None] * sp.grad(zeta, g)
            + sp.grad(eta ** 3 / 3.0 * P + eta ** 2 / 2.0 * Q, g)
            - (eta * (eta / 2.0 * P + Q))[None] * grad_h)
