"""Spectral derivative on an equispaced periodic grid (section 6.1).

D = F^{-1} (i K) F with wavenumbers k_j = 2 pi j / L, j = -n/2+1 .. n/2-1, and the
n/2 (Nyquist) wavenumber set to zero.  In 2D, D_x and D_y act along their own
axis and each zeroes its own Nyquist wavenumber (tensor-product extension,
end of section 6.1).  Test infrastructure only.
"""
from __future__ import annotations

import numpy as np


def wavenumbers(n: int, L: float) -> np.ndarray:
    """k_j in FFT order (j = 0..n-1), Nyquist (j = n/2) set to 0 (section 6.1)."""
    j = np.arange(n)
    m = np.where(j < n // 2, j, j - n).astype(np.float64)  # signed mode index
    if n % 2 == 0:
        m[n // 2] = 0.0
    return 2.0 * np.pi * m / L


def deriv(f: np.ndarray, L: float, axis: int = -1) -> np.ndarray:
    """Spectral derivative of a real periodic field along `axis` (section 6.1)."""
    n = f.shape[axis]
    k = wavenumbers(n, L)
    shape = [1] * f.ndim
    shape[axis] = n
    fh = np.fft.fft(f, axis=axis)
    return np.real(np.fft.ifft(1j * k.reshape(shape) * fh, axis=axis))


def dx(f, g):
    """d/dx on grid g (x is the last axis)."""
    return deriv(f, g.Lx, axis=-1)


def dy(f, g):
    """d/dy on grid g (y is the second-to-last axis, 2D only)."""
    return deriv(f, g.Ly, axis=-2)


def grad(f, g):
    """Spectral gradient, component-major (d, ...)."""
    if g.d == 1:
        return dx(f, g)[None]
    return np.stack([dx(f, g), dy(f, g)])


def div(u, g):
    """Spectral divergence of a component-major vector field."""
    if g.d == 1:
        return dx(u[0], g)
    return dx(u[0], g) + dy(u[1], g)


def dense_D(n: int, L: float) -> np.ndarray:
    """Dense n x n matrix of D = F^{-1} (iK) F built from the DFT matrix (small n only)."""
    j = np.arange(n)
    F = np.exp(-2j * np.pi * np.outer(j, j) / n)
    Finv = np.conj(F) / n
    K = np.diag(1j * wavenumbers(n, L))
    return np.real(Finv @ K @ F)


def dense_Dx_Dy(nx: int, ny: int, Lx: float, Ly: float):
    """Dense 2D derivative matrices on fields flattened in (y, x) row-major order."""
    Dx1 = dense_D(nx, Lx)
    Dy1 = dense_D(ny, Ly)
    Dx = np.kron(np.eye(ny), Dx1)
    Dy = np.kron(Dy1, np.eye(nx))
    return Dx, Dy
