"""Pins of the oracle's time integrators (section 5):

* the exact flat-bottom solitary wave (section 6) is reproduced at the design
  order of each scheme (RK4: 4, AB_s: s, SBDF2: 2; section 6.4 reports the
  same rates for Test 1);
* mass (Remark 2.1) is conserved to rounding;
* energy (Remark 2.1 with the bathymetry terms of B) drifts at the scheme's
  order;
* with dt = 0 the SBDF2 constraint recursion of Eq:MM decays at the rate set by
  the roots of the characteristic equation Eq:CharEq, c(z) - b(z) + lambda b(z) = 0,
  for the generalised eigenvalues lambda of (G, A) (section 5.4).
"""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import diagnostics as dg
from oracle import operators as op
from oracle import stepping as st
from paper_2506_16045_amd import inputs as I

H0, AMP, X0, TF = 1.0, 0.2, 30.0, 1.0


def _run(scheme, dt):
    g = I.grid1d(256, 80.0)
    eta0, u0 = I.solitary_wave(g, H0, AMP, X0)
    h = np.full(g.shape, H0)
    pb = st.Problem.from_h(g, h, tol=1e-13)
    U0 = pb.G(eta0, u0)
    n = int(round(TF / dt))
    if scheme == "rk4":
        e, U, u = st.run_rk4(pb, eta0, U0, u0, dt, n)
    elif scheme.startswith("ab"):
        e, U, u = st.run_ab(pb, int(scheme[2]), eta0, U0, u0, dt, n)
    else:
        e, U, u = st.run_sbdf2(pb, eta0, U0, u0, dt, n)
    ee, ue = I.solitary_wave(g, H0, AMP, X0, t=TF)
    assert abs(dg.mass(e, h, g) - dg.mass(eta0, h, g)) < 1e-13 * 80
    return np.max(np.abs(e - ee)), np.max(np.abs(u - ue))


@pytest.mark.parametrize("scheme,order", [("rk4", 4), ("ab2", 2), ("ab3", 3), ("ab4", 4), ("sbdf2", 2)])
def test_solitary_wave_convergence_order(scheme, order):
    e1, v1 = _run(scheme, 0.1)
    e2, v2 = _run(scheme, 0.05)
    rate = math.log2(e1 / e2)
    assert order - 0.4 <= rate <= order + 0.5, (e1, e2, rate)
    assert math.log2(v1 / v2) >= order - 0.3


def test_energy_drift_over_bathymetry_is_fourth_order():
    g = I.grid1d(64, 2 * math.pi)
    x = I.coords(g)
    h = 0.8 + 0.1 * np.cos(x)
    eta0 = h + 0.05 * np.cos(2 * x) + 0.7
    u0 = (0.05 * np.sin(x))[None]
    pb = st.Problem.from_h(g, h, tol=1e-14)
    U0 = pb.G(eta0, u0)
    E0 = dg.energy(eta0, u0, h, pb.grad_h, g)
    drift = []
    for dt in (0.1, 0.05):
        e, U, u = st.run_rk4(pb, eta0, U0, u0, dt, int(round(1.0 / dt)))
        drift.append(abs(dg.energy(e, u, h, pb.grad_h, g) - E0) / E0)
    assert drift[0] / drift[1] > 8.0, drift


def test_sbdf2_zero_stability_rate():
    g, eta, h, _ = I.pcg_test_problem_1d(32, 0.5, 0.3)
    pb = st.Problem.from_h(g, h, tol=1e-14)
    rng = np.random.default_rng(7)
    U = rng.normal(size=(1, 32))
    u0 = rng.normal(size=(1, 32))
    s, a, k = op.coefficients(eta, pb.grad_h, pb.flat)
    u_star = np.linalg.solve(op.dense_G(eta, pb.grad_h, g), U.ravel())
    lam = scipy.linalg.eigh(op.dense_G(eta, pb.grad_h, g), op.dense_A(s, a, g), eigvals_only=True)
    # SBDF2: c(z) = z^2, b(z) = 2z - 1  ->  z^2 - (1 - lambda)(2 z - 1) = 0
    rho = max(np.max(np.abs(np.roots([1.0, -2 * (1 - l), (1 - l)]))) for l in lam)
    assert rho < 1.0
    errs = {}
    for n in (60, 160):
        _, _, un = st.run_sbdf2(pb, eta, U, u0, 0.0, n, coeffs=(s, a))
        errs[n] = np.linalg.norm(un.ravel() - u_star)
    measured = (errs[160] / errs[60]) ** (1.0 / 100)
    assert measured == pytest.approx(rho, rel=0.02)


# ---------------------------------------------------------------------------
# Initial guesses of the stepper solves (a reading: the paper does not fix them)
# ---------------------------------------------------------------------------
def test_guess_history_extrapolates_linear_offsets_exactly():
    h = st.GuessHistory("extrapolate")
    h.prepare(0.1)
    base = np.array([3.0, -1.0])
    assert np.array_equal(h.guess("rk2", base), base)           # nothing recorded: the base
    a, b = np.array([0.5, 2.0]), np.array([-0.25, 0.125])
    h.record("rk2", base, base + a)                                # o_0 = a
    assert np.allclose(h.guess("rk2", base), base + a)             # one offset: held constant
    h.record("rk2", base, base + a + b)                            # o_1 = a + b
    assert np.allclose(h.guess("rk2", base), base + a + 2 * b)     # o_2 of the line, exactly
    h.record("rk2", base, base + a + 2 * b)
    assert np.allclose(h.guess("rk2", base), base + a + 3 * b)
    assert np.array_equal(h.guess("rk3", base), base)              # slots are independent
    h.prepare(0.05)                                                # a new step size clears
    assert np.array_equal(h.guess("rk2", base), base)
    p = st.GuessHistory("previous")
    p.record("ab", base, base + a)
    assert np.array_equal(p.guess("ab", base), base)
    with pytest.raises(ValueError):
        st.GuessHistory("linear")


@pytest.mark.parametrize("scheme", ["rk4", "ab3"])
def test_guess_changes_iterations_not_solution(scheme):
    """Both guesses converge to the same trajectory (to the solve tolerance);
    the extrapolated one needs fewer PCG iterations once its history is built."""
    g = I.grid1d(256, 80.0)
    rng = np.random.default_rng(I.SEED_BASE + 71)
    h = I.random_bumps1d(g, rng)
    eta_s, u0 = I.solitary_wave(g, 1.0, 0.2, 30.0)
    eta0 = h + (eta_s - 1.0)
    out, iters = {}, {}
    for mode in ("previous", "extrapolate"):
        pb = st.Problem.from_h(g, h, tol=1e-12, guess=mode)
        U0 = pb.G(eta0, u0)
        if scheme == "rk4":
            out[mode] = st.run_rk4(pb, eta0, U0, u0, 0.05, 12)
        else:
            out[mode] = st.run_ab(pb, 3, eta0, U0, u0, 0.05, 12)
        iters[mode] = sum(pb.iters[-8:])
    for a, b in zip(out["previous"], out["extrapolate"]):
        assert np.max(np.abs(a - b)) <= 1e-9 * max(1.0, np.max(np.abs(a)))
    assert iters["extrapolate"] < 0.85 * iters["previous"], iters
