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

import dataclasses

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


# ---------------------------------------------------------------------------
# De-aliased right-hand side (subsec:dswe_1d, remark on aliasing after Test 2:
# zeros are padded onto the high wavenumbers before the nonlinear terms are
# formed).  Reading: the inputs are interpolated onto a grid `factor` times as
# fine per axis by zero-padding their spectra, f(w, p) is evaluated there with
# the fine grid's spectral derivatives, and the result is truncated back to the
# modes of the original grid.  On both transfers only the modes with
# |m| < n/2 of the coarser grid are kept: its Nyquist modes, which the spectral
# derivative already treats as carrying no wavenumber (section 6.1), are set
# to zero.
# ---------------------------------------------------------------------------

def _axis_modes(n_src, n_dst):
    """(source index, destination index) of the signed modes kept on one axis."""
    n_min = min(n_src, n_dst)
    if n_min == 1:
        return np.array([0]), np.array([0])
    m = np.arange(-(n_min // 2) + 1, n_min // 2)   # |m| < n_min / 2
    return m % n_src, m % n_dst


def resample(f, g_src, g_dst):
    """Spectral interpolation (finer destination) or truncation (coarser) of a
    real periodic scalar field between two grids of the same domain, keeping
    the amplitude of every retained Fourier mode."""
    F = np.fft.fftn(f) / f.size
    if g_src.d == 1:
        si, di = _axis_modes(g_src.nx, g_dst.nx)
        G = np.zeros(g_dst.nx, dtype=complex)
        G[di] = F[si]
    else:
        sx, dxi = _axis_modes(g_src.nx, g_dst.nx)
        sy, dyi = _axis_modes(g_src.ny, g_dst.ny)
        G = np.zeros((g_dst.ny, g_dst.nx), dtype=complex)
        G[np.ix_(dyi, dxi)] = F[np.ix_(sy, sx)]
    return np.real(np.fft.ifftn(G) * G.size)


def fine_grid(g, factor=2):
    """The same domain with `factor` times as many points per axis."""
    if g.d == 1:
        return dataclasses.replace(g, nx=g.nx * factor)
    return dataclasses.replace(g, nx=g.nx * factor, ny=g.ny * factor)


def rhs_dealiased(eta, u, h, g, factor=2):
    """(eta_t, U_t) with the nonlinear terms formed on the padded grid."""
    gf = fine_grid(g, factor)
    eta_f = resample(eta, g, gf)
    u_f = np.stack([resample(c, g, gf) for c in u])
    h_f = resample(h, g, gf)
    grad_h_f = sp.grad(h_f, gf)
    e_t, U_t = rhs(eta_f, u_f, h_f, grad_h_f, gf)
    return resample(e_t, gf, g), np.stack([resample(c, gf, g) for c in U_t])
