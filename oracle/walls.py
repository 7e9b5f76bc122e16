"""Homogeneous Neumann (wall) boundaries for the constraint operator.

The paper computes with periodic boundaries but states its operator results for
walls as well: n . u = 0 on the boundary (Subsec:DAEform), the space H_div of
Subsec:linop, and the bounds of Sec:BoundonG.  Reading for a spectral method on
walls: the domain is [0, Lx] (x [0, Ly]) with a cell-centred grid
x_j = (j + 1/2) Lx / nx; scalar fields (eta, h, div u, grad h . u) are cosine
series cos(m pi x / Lx) cos(l pi y / Ly); a velocity component is a sine series
along its own axis and a cosine series along the other, so that it vanishes on
the walls it is normal to (u = sum U sin(m pi x / Lx) cos(l pi y / Ly), v the
transpose).  The spectral derivative maps cosine to sine series and back with
wavenumber m pi / L; the highest sine mode m = n takes wavenumber zero, as the
Nyquist wavenumber does on a periodic grid (section 6.1).  Transforms are the
type-II DCT / DST of scipy.fft (library primitives); coefficients are kept as
series amplitudes indexed by the mode number m = 0..n on each axis, so that the
u and v amplitudes of one mode can be combined directly.  Test infrastructure
only.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sf

from . import krylov
from . import operators as op
from . import stepping


# ---- transforms: samples <-> series amplitudes on one axis ------------------------
def _fwd_axis(f, kind, axis):
    """Amplitudes (mode m = 0..n along `axis`) of the cosine ('c') or sine ('s')
    series through the samples f."""
    n = f.shape[axis]
    f = np.moveaxis(f, axis, -1)
    out = np.zeros(f.shape[:-1] + (n + 1,))
    if kind == "c":
        X = sf.dct(f, type=2, axis=-1)           # X_m = 2 sum_j f_j cos(pi m (2j+1) / 2n)
        out[..., 0] = X[..., 0] / (2 * n)
        out[..., 1:n] = X[..., 1:] / n
    else:
        Y = sf.dst(f, type=2, axis=-1)           # Y_{m-1} = 2 sum_j f_j sin(pi m (2j+1) / 2n)
        out[..., 1:n] = Y[..., :n - 1] / n
        out[..., n] = Y[..., n - 1] / (2 * n)
    return np.moveaxis(out, -1, axis)


def _inv_axis(A, kind, axis):
    """Samples of the series with amplitudes A (modes 0..n along `axis`)."""
    n = A.shape[axis] - 1
    A = np.moveaxis(A, axis, -1)
    if kind == "c":
        X = np.concatenate([A[..., :1] * (2 * n), A[..., 1:n] * n], axis=-1)
        f = sf.idct(X, type=2, axis=-1)
    else:
        Y = np.concatenate([A[..., 1:n] * n, A[..., n:] * (2 * n)], axis=-1)
        f = sf.idst(Y, type=2, axis=-1)
    return np.moveaxis(f, -1, axis)


def to_modes(f, kinds):
    """kinds: one letter per axis in array order ((y, x) in 2D)."""
    A = f
    for ax, k in enumerate(kinds):
        A = _fwd_axis(A, k, ax)
    return A


def from_modes(A, kinds):
    f = A
    for ax, k in enumerate(kinds):
        f = _inv_axis(f, k, ax)
    return f


def wavenumbers(n, L):
    """m pi / L for m = 0..n, with the sine Nyquist mode m = n at zero."""
    k = np.arange(n + 1) * np.pi / L
    k[n] = 0.0
    return k


SCALAR = {1: "c", 2: "cc"}
VECTOR = {1: ("s",), 2: ("cs", "sc")}   # kinds in (y, x) order: u is sine in x, v sine in y


def _deriv(f, kinds, axis, L):
    """Derivative along array axis `axis` of a field with the given kinds; returns
    (derivative samples, their kinds)."""
    A = to_modes(f, kinds)
    n = f.shape[axis]
    shape = [1] * f.ndim
    shape[axis] = n + 1
    k = wavenumbers(n, L).reshape(shape)
    k_ax = kinds[axis]
    if k_ax == "c":
        dA, nk = -k * A, "s"
    else:
        dA, nk = k * A, "c"
    new = kinds[:axis] + nk + kinds[axis + 1:]
    return from_modes(dA, new), new


def grad(f, g):
    """Gradient of a scalar (cosine) field: component-major (d, ...)."""
    if g.d == 1:
        return _deriv(f, "c", 0, g.Lx)[0][None]
    fx, _ = _deriv(f, "cc", 1, g.Lx)
    fy, _ = _deriv(f, "cc", 0, g.Ly)
    return np.stack([fx, fy])


def div(u, g):
    """Divergence of a wall velocity field (sine along each component's own axis)."""
    if g.d == 1:
        return _deriv(u[0], "s", 0, g.Lx)[0]
    ux, _ = _deriv(u[0], "cs", 1, g.Lx)
    vy, _ = _deriv(u[1], "sc", 0, g.Ly)
    return ux + vy


# ---- the constraint operator and the preconditioner --------------------------------
def bathy_gradient(h, g):
    """grad h = D h with the wall derivative; a constant h is flat (grad h = 0)."""
    h = np.asarray(h, dtype=np.float64)
    if np.all(h == h.flat[0]):
        return np.zeros((g.d,) + h.shape), True
    return grad(h, g), False


def apply_G(eta, grad_h, u, g):
    """G_{eta,h} u of Def:G with the wall derivatives (the same five terms as on a
    periodic grid)."""
    delta = div(u, g)
    beta = np.sum(grad_h * u, axis=0)
    return (eta[None] * u - grad((eta ** 3 / 3.0) * delta, g) - grad((eta ** 2 / 2.0) * beta, g)
            + (eta ** 2 / 2.0)[None] * grad_h * delta[None] + eta[None] * grad_h * beta[None])


def apply_A(sigma, alpha, u, g):
    return sigma * u - alpha * grad(div(u, g), g)


def solve_A(sigma, alpha, r, g):
    """A^{-1} r mode by mode: the symbol of A = sigma I - alpha grad(div) (Def:A)
    at mode (m, l) is sigma I + alpha k k^T with k = (m pi / Lx, l pi / Ly) (the
    sine Nyquist wavenumbers at zero); split along k and across it as on a
    periodic grid."""
    if g.d == 1:
        R = to_modes(r[0], "s")
        k = wavenumbers(g.nx, g.Lx)
        return from_modes(R / (sigma + alpha * k * k), "s")[None]
    U = to_modes(r[0], "cs")
    V = to_modes(r[1], "sc")
    kx = wavenumbers(g.nx, g.Lx)[None, :]
    ky = wavenumbers(g.ny, g.Ly)[:, None]
    k2 = kx * kx + ky * ky
    proj = np.where(k2 > 0, (kx * U + ky * V) / np.where(k2 > 0, k2, 1.0), 0.0)
    pu, pv = kx * proj, ky * proj
    Zu = (U - pu) / sigma + pu / (sigma + alpha * k2)
    Zv = (V - pv) / sigma + pv / (sigma + alpha * k2)
    return np.stack([from_modes(Zu, "cs"), from_modes(Zv, "sc")])


def dense(apply, g):
    """Dense matrix of a linear map on wall velocity fields, by columns (small grids)."""
    n = g.d * g.npts
    M = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        M[:, j] = apply(e.reshape((g.d,) + g.shape)).ravel()
    return M


def pcg_solve(eta, grad_h, flat, b, g, tol=1e-12, max_iter=2000, x0=None, kind="optimal"):
    """PCG (section 3.2) on G u = b with walls, A built from sigma*, alpha* of
    Sec:BoundonG (the coefficients are pointwise quantities, the same on walls)."""
    s, a, k = op.coefficients(eta, grad_h, flat, kind=kind)
    u, it, ok, hist = krylov.pcg(lambda v: apply_G(eta, grad_h, v, g), lambda r: solve_A(s, a, r, g), b,
                                 x0=x0, tol=tol, max_iter=max_iter)
    return u, it, ok, (s, a, k)


# ---- right-hand side between walls ---------------------------------------------
def _dx(f, kinds, g):
    return _deriv(f, kinds, f.ndim - 1, g.Lx)[0]


def _dy(f, kinds, g):
    return _deriv(f, kinds, 0, g.Ly)[0]


def rhs(eta, u, h, grad_h, g):
    """(eta_t, U_t) of the constraint form (Eq:DSWEcf, Def:bigF) between walls:
    the terms of the periodic right-hand side with the wall derivatives.  Every
    derivative acts on a product whose series kind follows from the parities:
    scalars are cosine series, each velocity component a sine series along its
    own axis, so eta u u_i is sine along axis i and eta u v sine along both."""
    delta = div(u, g)
    m = div(eta[None] * u, g)
    beta = np.sum(grad_h * u, axis=0)
    P = np.sum(u * grad(delta, g), axis=0) - delta ** 2
    Q = np.sum(u * grad(beta, g), axis=0)
    S = eta ** 3 / 3.0 * P + eta ** 2 * m * delta + eta ** 2 / 2.0 * Q + eta * m * beta
    T = eta ** 2 / 2.0 * P + eta * m * delta + eta * Q + m * beta
    F = grad(S, g) - grad_h * T[None]
    if g.d == 1:
        flux = _dx(eta * u[0] * u[0], "c", g)[None]
    else:
        flux = np.stack([
            _dx(eta * u[0] * u[0], "cc", g) + _dy(eta * u[0] * u[1], "ss", g),
            _dx(eta * u[0] * u[1], "ss", g) + _dy(eta * u[1] * u[1], "cc", g),
        ])
    return -m, -eta[None] * grad(eta - h, g) - flux + F


class Problem(stepping.Problem):
    """A stepping problem between walls: the steppers of oracle.stepping with the
    wall right-hand side, G, A and A^{-1}."""

    @classmethod
    def from_h(cls, g, h, tol=1e-12, max_iter=1000, guess="extrapolate"):
        gh, fl = bathy_gradient(h, g)
        return cls(g, np.asarray(h, dtype=np.float64), gh, fl, tol, max_iter,
                   hist=stepping.GuessHistory(guess))

    def f(self, eta, u):
        return rhs(eta, u, self.h, self.grad_h, self.g)

    def G(self, eta, u):
        return apply_G(eta, self.grad_h, u, self.g)

    def A(self, sigma, alpha, u):
        return apply_A(sigma, alpha, u, self.g)

    def A_inv(self, sigma, alpha, r):
        return solve_A(sigma, alpha, r, self.g)
