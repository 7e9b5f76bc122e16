"""Pins of the oracle's spectral derivative against closed forms and the DFT
matrix (section 6.1), not against itself."""
import json
import math
import os

import numpy as np
import pytest

from oracle import spectral as sp
from paper_2506_16045_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("n,L", [(16, 1.0), (64, 2 * math.pi), (256, 80.0), (512, 400.0)])
def test_derivative_of_trig_modes(n, L):
    g = I.grid1d(n, L)
    x = I.coords(g)
    for m in range(1, n // 2):
        k = 2 * math.pi * m / L
        f = np.sin(k * x) + 0.5 * np.cos(k * x)
        exact = k * np.cos(k * x) - 0.5 * k * np.sin(k * x)
        assert np.max(np.abs(sp.dx(f, g) - exact)) <= 1e-12 * max(1.0, k) * n


@pytest.mark.parametrize("n", [8, 32, 128])
def test_nyquist_mode_is_annihilated(n):
    g = I.grid1d(n, 3.0)
    x = I.coords(g)
    f = np.cos(math.pi * n * x / 3.0)           # the n/2 mode, +-1 on the grid
    assert np.max(np.abs(f)) == pytest.approx(1.0)
    assert np.max(np.abs(sp.dx(f, g))) < 1e-12
    assert np.max(np.abs(sp.dx(np.ones(n), g))) < 1e-13


@pytest.mark.parametrize("n", [8, 16, 33 - 1])
def test_dense_D_real_antisymmetric_and_matches_fft(n, rng):
    D = sp.dense_D(n, 2.0)
    assert np.max(np.abs(D + D.T)) < 1e-12
    f = rng.normal(size=n)
    g = I.grid1d(n, 2.0)
    assert np.max(np.abs(D @ f - sp.dx(f, g))) < 1e-11


def test_2d_partial_derivatives():
    g = I.grid2d(32, 16, 2.0, 3.0)
    X, Y = I.coords(g)
    a, b = 3, 2
    ph = 2 * math.pi * (a * X / g.Lx + b * Y / g.Ly)
    f = np.sin(ph)
    assert np.max(np.abs(sp.dx(f, g) - 2 * math.pi * a / g.Lx * np.cos(ph))) < 1e-11
    assert np.max(np.abs(sp.dy(f, g) - 2 * math.pi * b / g.Ly * np.cos(ph))) < 1e-11
    # y-Nyquist row mode killed by dy but not by dx
    f2 = np.cos(math.pi * g.ny * Y / g.Ly) * np.sin(2 * math.pi * X / g.Lx)
    assert np.max(np.abs(sp.dy(f2, g))) < 1e-11
    assert np.max(np.abs(sp.dx(f2, g))) > 1.0


def test_golden_test_problem_slope():
    """Section 6.2 prints |h_x|_max = sqrt(2)/(e^{1/2} sigma) |h0| ~ 17.2 |h0| for the
    test bathymetry h = 1 + h0 exp(-(x-1/2)^2/sigma^2), sigma = 1/20."""
    with open(os.path.join(GOLDEN, "paper_numbers.json")) as fh:
        gold = json.load(fh)
    printed = gold["test_problem_max_slope_per_h0"]["value"]
    g, eta, h, b = I.pcg_test_problem_1d(4096, 1.0, 1.0)
    slope = np.max(np.abs(sp.dx(h, g)))
    assert abs(slope - printed) / printed < 5e-3          # the paper's 3-digit value
    closed = math.sqrt(2.0) / (math.exp(0.5) * (1.0 / 20.0))
    assert abs(slope - closed) / closed < 1e-4            # its closed form
