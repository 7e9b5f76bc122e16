"""Pins of the oracle's right-hand side f(w, p):

* the exact flat-bottom solitary wave (section 6, ExSleta/ExSlu) is a travelling
  wave, so eta_t = -c eta_x and U_t = -c (G u)_x must come out of f;
* the forcing F of Def:bigF must agree with the eta-multiplied momentum equation
  Eq:MomEq through the commutation U_t = G u_t + (dG/dt) u of section 2.2;
* the energy of Remark 2.1 (with the bathymetry terms of B[u, u]) is conserved
  by the semi-discrete system, which singles out the reading
  (u.grad)^2 h = u.grad(u.grad h) over the Hessian reading.
"""
import math

import numpy as np
import pytest

from oracle import operators as op
from oracle import rhs as R
from oracle import spectral as sp
from paper_2506_16045_amd import inputs as I


@pytest.mark.parametrize("d", [1, 2])
def test_solitary_wave_is_a_travelling_solution(d):
    h0, a = 1.0, 0.2
    c, _ = I.solitary_speed_width(h0, a)
    g = I.grid1d(256, 80.0) if d == 1 else I.grid2d(256, 4, 80.0, 2.0)
    eta, u = I.solitary_wave(g, h0, a, 35.0)
    h = np.full(g.shape, h0)
    gh, fl = op.bathy_gradient(h, g)
    eta_t, U_t = R.rhs(eta, u, h, gh, g)
    U = op.apply_G(eta, gh, u, g)
    assert np.max(np.abs(eta_t + c * sp.dx(eta, g))) < 1e-11
    assert np.max(np.abs(U_t + c * sp.dx(U, g))) < 1e-10
    # and the travelling-wave rate is not trivially small
    assert np.max(np.abs(U_t)) > 1e-2


def _band_limited(g):
    if g.d == 1:
        x = I.coords(g)
        eta = 1.5 + 0.2 * np.cos(x) + 0.1 * np.sin(2 * x)
        u = (0.3 * np.sin(x) + 0.2 * np.cos(2 * x))[None]
        h = 0.8 + 0.15 * np.cos(x + 0.3)
        return eta, u, h
    X, Y = I.coords(g)
    eta = 1.5 + 0.2 * np.cos(X) + 0.1 * np.sin(Y + 0.4) + 0.05 * np.cos(X - Y)
    u = np.stack([0.3 * np.sin(X) + 0.1 * np.cos(Y), 0.2 * np.cos(X + Y) - 0.1 * np.sin(Y)])
    h = 0.8 + 0.15 * np.cos(X + 0.3) + 0.1 * np.sin(Y)
    return eta, u, h


def _dG(eta, gh, u, g, etadot):
    """Directional derivative of G_{eta,h} u in eta along etadot: G is a cubic
    polynomial in eta, so the Richardson-combined central difference is exact
    up to rounding."""
    def cd(e):
        return (op.apply_G(eta + e * etadot, gh, u, g) - op.apply_G(eta - e * etadot, gh, u, g)) / (2 * e)
    e = 1e-3
    return (4 * cd(e / 2) - cd(e)) / 3


GRIDS = [I.grid1d(128, 2 * math.pi), I.grid2d(64, 64, 2 * math.pi, 2 * math.pi)]


@pytest.mark.parametrize("g", GRIDS, ids=["1d", "2d"])
def test_forcing_agrees_with_momentum_equation(g):
    eta, u, h = _band_limited(g)
    gh, fl = op.bathy_gradient(h, g)
    eta_t, U_t = R.rhs(eta, u, h, gh, g)
    Gu_t = R.momentum_rhs(eta, u, h, gh, g)            # = G u_t by Eq:MomEq
    rhs2 = Gu_t + _dG(eta, gh, u, g, eta_t)           # (G u)_t = G u_t + G_{eta_t} u
    scale = np.max(np.abs(U_t))
    assert np.max(np.abs(U_t - rhs2)) <= 1e-10 * scale


def _energy_rate(rhs_fn, g):
    eta, u, h = _band_limited(g)
    gh, fl = op.bathy_gradient(h, g)
    eta_t, U_t = rhs_fn(eta, u, h, gh, g)
    zeta = eta - h
    # dE/dt = int zeta eta_t + u . U_t - 1/2 u . (dG/dt) u   (G symmetric)
    rate = np.sum(zeta * eta_t) + np.sum(u * U_t) - 0.5 * np.sum(u * _dG(eta, gh, u, g, eta_t))
    scale = np.sum(np.abs(u * U_t)) + np.sum(np.abs(zeta * eta_t))
    return rate * g.cell, scale * g.cell


@pytest.mark.parametrize("g", GRIDS, ids=["1d", "2d"])
def test_energy_conserved_over_bathymetry_with_material_reading(g):
    rate, scale = _energy_rate(R.rhs, g)
    assert abs(rate) <= 1e-11 * scale
    rate_h, _ = _energy_rate(R.rhs_hessian_reading, g)
    assert abs(rate_h) > 1e-4 * scale


def test_mass_rate_is_zero(rng):
    g = I.grid2d(32, 16, 3.0, 2.0)
    eta = I.random_positive_depth(g, rng)
    u = np.stack([I.random_smooth_field(g, rng), I.random_smooth_field(g, rng)])
    h = 1.0 + 0.1 * I.random_smooth_field(g, rng)
    gh, _ = op.bathy_gradient(h, g)
    eta_t, _ = R.rhs(eta, u, h, gh, g)
    assert abs(np.sum(eta_t)) < 1e-12 * np.sum(np.abs(eta_t))
