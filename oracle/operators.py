"""The SGN constraint operator G_{eta,h}, the preconditioner A and its coefficients.

Test infrastructure only (see the package docstring).  Fields follow the
layout of paper_2506_16045_amd.inputs: scalars (n,) or (ny, nx), vectors
component-major (d, ...).  grad_h is the bathymetry gradient on the grid
(the oracle takes it as the spectral gradient D h, see bathy_gradient).
"""
from __future__ import annotations

import math

import numpy as np

from . import spectral as sp

# Eigenvalues of the number matrix [[1, 1/2], [1/2, 1/3]] (Appendix A, Eq:NumberMatrix)
LAMBDA_PLUS = (4.0 + math.sqrt(13.0)) / 6.0
LAMBDA_MINUS = (4.0 - math.sqrt(13.0)) / 6.0


def bathy_gradient(h, g):
    """grad h on the grid and the flat flag.

    The paper treats |grad h|_max as a one-time computation from the prescribed h
    (section 4) without fixing how grad h is discretised; reading: grad h is the
    spectral gradient D h, except that a bathymetry that is exactly constant on
    the grid is flat and gets grad h = 0 exactly (the flat coefficients
    Eq:FlatbathCoeff apply only when |grad h|_max = 0).
    Returns (grad_h (d, ...), flat: bool).
    """
    h = np.asarray(h, dtype=np.float64)
    if np.all(h == h.flat[0]):
        return np.zeros((g.d,) + h.shape), True
    return sp.grad(h, g), False


def apply_G(eta, grad_h, u, g):
    """G_{eta,h} u, term by term as in Def:G (section 2.2):

        G u = eta u - grad( eta^3/3 div u ) - grad( eta^2/2 (grad h . u) )
              + eta^2/2 grad h (div u) + eta grad h (grad h . u)

    with every derivative the spectral one (section 6.1).
    """
    delta = sp.div(u, g)                              # div u
    beta = np.sum(grad_h * u, axis=0)                 # grad h . u
    term1 = eta[None] * u
    term2 = -sp.grad((eta ** 3 / 3.0) * delta, g)
    term3 = -sp.grad((eta ** 2 / 2.0) * beta, g)
    term4 = (eta ** 2 / 2.0)[None] * grad_h * delta[None]
    term5 = eta[None] * grad_h * beta[None]
    return term1 + term2 + term3 + term4 + term5


def dense_G(eta, grad_h, g):
    """Dense matrix of G on small grids, assembled from the weak form B (section 3.1).

    Unknowns are ordered [u; v] (2D) or [u] (1D), each flattened (y, x) row-major.
    G = diag(eta) (x) I_d + H^T diag(eta) H + Ddiv^T diag(eta^3/3) Ddiv
        + Ddiv^T diag(eta^2/2) H + H^T diag(eta^2/2) Ddiv
    with Ddiv = [Dx Dy] (the discrete divergence) and H = [diag(hx) diag(hy)].
    This is the B[u, v] form written with the grid sum; it equals the strong
    form because the spectral D is real antisymmetric.
    """
    N = g.npts
    if g.d == 1:
        Ddiv = sp.dense_D(g.nx, g.Lx)
        H = np.diag(grad_h[0].ravel())
    else:
        Dx, Dy = sp.dense_Dx_Dy(g.nx, g.ny, g.Lx, g.Ly)
        Ddiv = np.hstack([Dx, Dy])
        H = np.hstack([np.diag(grad_h[0].ravel()), np.diag(grad_h[1].ravel())])
    e = eta.ravel()
    I = np.kron(np.eye(g.d), np.diag(e))
    G = (I + H.T @ np.diag(e) @ H + Ddiv.T @ np.diag(e ** 3 / 3.0) @ Ddiv
         + Ddiv.T @ np.diag(e ** 2 / 2.0) @ H + H.T @ np.diag(e ** 2 / 2.0) @ Ddiv)
    assert G.shape == (g.d * N, g.d * N)
    return G


def apply_A(sigma, alpha, u, g):
    """A u = sigma u - alpha grad(div u)  (Def:A)."""
    return sigma * u - alpha * sp.grad(sp.div(u, g), g)


def dense_A(sigma, alpha, g):
    """Dense A = sigma I + alpha Ddiv^T Ddiv (section 6.1, A = sigma I + alpha D^dagger D)."""
    if g.d == 1:
        Ddiv = sp.dense_D(g.nx, g.Lx)
    else:
        Dx, Dy = sp.dense_Dx_Dy(g.nx, g.ny, g.Lx, g.Ly)
        Ddiv = np.hstack([Dx, Dy])
    return sigma * np.eye(g.d * g.npts) + alpha * Ddiv.T @ Ddiv


def solve_A(sigma, alpha, r, g):
    """z = A^{-1} r, diagonal in Fourier space (section 6.1).

    1D: z_hat = r_hat / (sigma + alpha k^2).
    2D: the symbol of A = sigma I - alpha grad(div) (Def:A) at wavevector k is
    sigma I + alpha k k^T (each Nyquist wavenumber set to zero); k is its
    eigenvector with eigenvalue sigma + alpha |k|^2 and the direction across k
    has eigenvalue sigma, so with r_par = k (k . r_hat) / |k|^2
        z_hat = (r_hat - r_par) / sigma + r_par / (sigma + alpha |k|^2).
    (Solving the assembled 2x2 symbol instead loses the digits of sigma
    whenever alpha |k|^2 >> sigma.)
    """
    if g.d == 1:
        k = sp.wavenumbers(g.nx, g.Lx)
        rh = np.fft.fft(r[0])
        return np.real(np.fft.ifft(rh / (sigma + alpha * k * k)))[None]
    kx = np.broadcast_to(sp.wavenumbers(g.nx, g.Lx)[None, :], g.shape)
    ky = np.broadcast_to(sp.wavenumbers(g.ny, g.Ly)[:, None], g.shape)
    k2 = kx * kx + ky * ky
    rx, ry = np.fft.fft2(r[0]), np.fft.fft2(r[1])
    proj = np.where(k2 > 0, (kx * rx + ky * ry) / np.where(k2 > 0, k2, 1.0), 0.0)
    px, py = kx * proj, ky * proj
    zx = (rx - px) / sigma + px / (sigma + alpha * k2)
    zy = (ry - py) / sigma + py / (sigma + alpha * k2)
    return np.stack([np.real(np.fft.ifft2(zx)), np.real(np.fft.ifft2(zy))])


def solve_A_assembled(sigma, alpha, r, g):
    """A^{-1} r in 2D by solving the assembled 2x2 symbol at every mode (a plain
    library solve); used only to pin solve_A on well-conditioned cases."""
    kx = sp.wavenumbers(g.nx, g.Lx)[None, :]
    ky = sp.wavenumbers(g.ny, g.Ly)[:, None]
    KX = np.broadcast_to(kx, g.shape)
    KY = np.broadcast_to(ky, g.shape)
    M = np.empty(g.shape + (2, 2))
    M[..., 0, 0] = sigma + alpha * KX * KX
    M[..., 0, 1] = alpha * KX * KY
    M[..., 1, 0] = alpha * KX * KY
    M[..., 1, 1] = sigma + alpha * KY * KY
    rh = np.stack([np.fft.fft2(r[0]), np.fft.fft2(r[1])], axis=-1)
    zh = np.linalg.solve(M.astype(np.complex128), rh[..., None])[..., 0]
    return np.stack([np.real(np.fft.ifft2(zh[..., 0])), np.real(np.fft.ifft2(zh[..., 1]))])


def coefficients(eta, grad_h, flat, kind="optimal"):
    """(sigma*, alpha*, kappa_ub) of section 4.

    flat:     sigma* = eta_max, alpha* = eta_max^3 / 3, kappa_ub = (eta_max/eta_min)^3
              (Eq:FlatbathCoeff)
    variable: sigma* = max_x (eta + lambda_+ eta |grad h|^2), alpha* = lambda_+ eta_max^3,
              kappa_ub = max(sigma*/eta_min, (lambda_+/lambda_-)(eta_max/eta_min)^3)
              (Eq:Optcoeff, Eq:Optcoeffb)
    kind="replacement" gives sigma**, alpha** and their looser bound (Remark 4.2).
    """
    eta_min = float(np.min(eta))
    eta_max = float(np.max(eta))
    if eta_min <= 0.0 or not np.isfinite(eta_min) or not np.isfinite(eta_max):
        raise ValueError("total depth must be positive and finite (section 3.1)")
    ratio3 = (eta_max / eta_min) ** 3
    if flat:
        return eta_max, eta_max ** 3 / 3.0, ratio3
    g2 = np.sum(grad_h * grad_h, axis=0)
    alpha = LAMBDA_PLUS * eta_max ** 3
    if kind == "optimal":
        sigma = float(np.max(eta + LAMBDA_PLUS * eta * g2))
        kappa = max(sigma / eta_min, (LAMBDA_PLUS / LAMBDA_MINUS) * ratio3)
    elif kind == "replacement":
        gmax2 = float(np.max(g2))
        sigma = eta_max * (1.0 + LAMBDA_PLUS * gmax2)
        kappa = max((eta_max / eta_min) * (1.0 + LAMBDA_PLUS * gmax2),
                    (LAMBDA_PLUS / LAMBDA_MINUS) * ratio3)
    else:
        raise ValueError(kind)
    return sigma, alpha, kappa


def pointwise_M(eta, grad_h):
    """The (d+1) x (d+1) coefficient matrix M(x) of B (Appendix A, Def:MatrixM),
    returned with shape (..., d+1, d+1) over the grid."""
    d = grad_h.shape[0]
    shp = eta.shape
    M = np.zeros(shp + (d + 1, d + 1))
    gh = np.moveaxis(grad_h, 0, -1)                     # (..., d)
    M[..., :d, :d] = (np.eye(d) + gh[..., :, None] * gh[..., None, :])
    M[..., :d, d] = 0.5 * eta[..., None] * gh
    M[..., d, :d] = 0.5 * eta[..., None] * gh
    M[..., d, d] = eta ** 2 / 3.0
    return eta[..., None, None] * M
