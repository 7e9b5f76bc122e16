"""The identities behind the 2D wall solve on the grid's own points, checked in
NumPy against SciPy's type-II DCT/DST (CPU only; the kernels themselves are
checked against the oracle in tests/test_gpu_walls.py).

A line f_0..f_{n-1} read in the order v_i = f_{2i} (i < n/2), v_i = f_{2(n-1-i)+1}
(i >= n/2) has a DFT V with w_k V_k = C_k - i C_{n-k}, w_k = exp(-i pi k / 2n), for
the cosine sums C_k = sum_j f_j cos(pi k (2j+1) / 2n) (C_n = 0); read with the
sign (-1)^j, which is -1 exactly on the second half of that order, its cosine sums
are the sine sums: C_{n-m} = sum_j f_j sin(pi m (2j+1) / 2n).  In 2D the columns of
the row transforms hold C_k - i C_{nx-k} of every row, and the pair of column
FFT values (F[q], F[ny-q]) gives the four amplitudes of slots (k, nx-k) x (q, ny-q).
"""
import numpy as np
import pytest
import scipy.fft as sf


def _order(n):
    i = np.arange(n)
    return np.where(i < n // 2, 2 * i, 2 * (n - 1 - i) + 1)


def _sign(n):
    return np.where(np.arange(n) >= n // 2, -1.0, 1.0)


def _w(n, k):
    return np.exp(-1j * np.pi * np.asarray(k) / (2 * n))


@pytest.mark.parametrize("n", [2, 4, 8, 64, 512])
def test_reordered_dft_gives_the_cosine_sums(n):
    rng = np.random.default_rng(n)
    f = rng.normal(size=n)
    V = np.fft.fft(f[_order(n)])
    k = np.arange(n)
    z = _w(n, k) * V
    C = sf.dct(f, type=2) / 2.0                       # sum_j f_j cos(pi k (2j+1) / 2n)
    Cn = np.concatenate([C, [0.0]])
    np.testing.assert_allclose(z.real, C, atol=1e-12 * np.abs(f).sum())
    np.testing.assert_allclose(-z.imag, Cn[n - k], atol=1e-12 * np.abs(f).sum())


@pytest.mark.parametrize("n", [2, 4, 8, 64, 512])
def test_signed_reordered_line_gives_the_sine_sums(n):
    rng = np.random.default_rng(n + 1)
    f = rng.normal(size=n)
    g = f[_order(n)] * _sign(n)                       # = ((-1)^j f_j) in the order
    np.testing.assert_array_equal(g, ((-1.0) ** np.arange(n) * f)[_order(n)])
    z = _w(n, np.arange(n)) * np.fft.fft(g)
    S = sf.dst(f, type=2) / 2.0                       # S[m-1] = sum_j f_j sin(pi m (2j+1) / 2n), m = 1..n
    m = np.arange(1, n + 1)
    np.testing.assert_allclose(z.real[n - m[:-1]], S[:-1], atol=1e-12 * np.abs(f).sum())
    np.testing.assert_allclose(z.real[0], S[-1], atol=1e-12 * np.abs(f).sum())   # the Nyquist sine mode


@pytest.mark.parametrize("ny,nx", [(2, 2), (4, 8), (16, 4), (32, 32)])
@pytest.mark.parametrize("xs,ys", [(False, False), (True, False), (False, True), (True, True)])
def test_column_pairs_give_the_2d_slot_amplitudes(ny, nx, xs, ys):
    """Real 2D DFT of the ordered (and signed) field, then per column k and pair
    (q, ny-q): P_a = (F[q] + conj F[ny-q]) / 2 and P_b = i (F[q] - conj F[ny-q]) / 2
    after the x twiddle, then w_q P = E_q - i E_{ny-q}: the unnormalised cosine /
    sine amplitudes at slots (k, q), (k, ny-q), (nx-k, q), (nx-k, ny-q), mode m at
    slot m mod n."""
    rng = np.random.default_rng(nx * 100 + ny)
    f = rng.normal(size=(ny, nx))
    g = f[_order(ny)][:, _order(nx)]
    if xs:
        g = g * _sign(nx)[None, :]
    if ys:
        g = g * _sign(ny)[:, None]
    F = np.fft.fft(np.fft.rfft(g, axis=1), axis=0)

    def amp(sx, sy):
        jx, jy = np.arange(nx), np.arange(ny)
        mx = sx if (sx or not xs) else nx
        my = sy if (sy or not ys) else ny
        bx = np.sin(np.pi * mx * (2 * jx + 1) / (2 * nx)) if xs else np.cos(np.pi * mx * (2 * jx + 1) / (2 * nx))
        by = np.sin(np.pi * my * (2 * jy + 1) / (2 * ny)) if ys else np.cos(np.pi * my * (2 * jy + 1) / (2 * ny))
        return by @ f @ bx

    tol = 1e-11 * np.abs(f).sum()
    for k in range(nx // 2 + 1):
        for q in range(ny // 2 + 1):
            m = (ny - q) % ny
            F1, F2 = _w(nx, k) * F[q, k], _w(nx, k) * F[m, k]
            ua = _w(ny, q) * 0.5 * (F1 + np.conj(F2))
            ub = _w(ny, q) * 0.5j * (F1 - np.conj(F2))
            # x-line sums of index k and nx-k; a sine line's sums of index j are the modes nx-j
            xa, xb = (k, (nx - k) % nx) if not xs else ((nx - k) % nx, k)
            ya_q, ya_m = (q, m) if not ys else (m, q)
            assert abs(ua.real - amp(xa, ya_q)) <= tol
            if k != 0:
                assert abs(ub.real - amp(xb, ya_q)) <= tol
            if q != m:
                assert abs(-ua.imag - amp(xa, ya_m)) <= tol
                if k != 0:
                    assert abs(-ub.imag - amp(xb, ya_m)) <= tol
