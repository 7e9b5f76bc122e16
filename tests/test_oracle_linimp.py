"""Pins of the linearly implicit schemes and their zero-stability checker
(oracle/linimp.py; section 5.3 Eq:IMEX_DAE, section 5.4 Eq:CharEq,
Fig:StabilityRegion).

* The checker's stable intervals equal closed forms derived by hand: SBDF1
  (0, 2) (root 1 - lambda), SBDF2 (0, 4/3) (|z|^2 = 1 - lambda on (0, 1], a root
  at -1 at 4/3), SBDF3 (1/2, 8/7) (roots e^{+-i pi/3} at 1/2, a root at -1 at 8/7:
  Fig:StabilityRegion's caption, read for the eigenvalues of G^{-1} A).
* SBDF3(r): r = 0 is the textbook SBDF3 (BDF3 with extrapolation); the
  closed-form interval equals the checker's for several r; the order
  conditions hold (third order of (a, b) and (a, c), defect of the constraint
  recurrence O(dt^3)); a(z) satisfies the root condition.
* The recurrence of Eq:ZeroS3 iterated by brute force with a dense random
  symmetric positive pair (G, A) whose generalised eigenvalues are prescribed:
  bounded exactly when the checker says zero-stable.
* The joint choice of (r, theta) places [1/(theta kappa), 1/theta] inside D.
* On the SGN equations: the generic stepper with the SBDF2 coefficients equals
  the dedicated SBDF2 stepper; SBDF3(r) converges at third order against the
  exact flat-bottom solitary wave (section 6, ExSleta/ExSlu); over the shelf
  (kappa_ub = 339) plain SBDF3 blows up while SBDF3(r) with the chosen
  (r, theta) stays bounded, as section 5.4 predicts.
Planted mistakes in the oracle (a wrong sign of lambda in Eq:CharEq, the sum
of Eq:ZeroS3 starting at j = 1, b and c swapped in the constraint update, a
missing theta, a dropped c_j term) each fail one of these."""
import math

import numpy as np
import pytest

from oracle import diagnostics as dg
from oracle import linimp as L
from oracle import operators as op
from oracle import stepping as ost
from paper_2506_16045_amd import inputs as I


@pytest.mark.parametrize("scheme,lo,hi", [(L.SBDF1, 0.0, 2.0), (L.SBDF2, 0.0, 4.0 / 3.0),
                                          (L.SBDF3, 0.5, 8.0 / 7.0)], ids=["sbdf1", "sbdf2", "sbdf3"])
def test_stable_intervals_of_the_sbdf_family(scheme, lo, hi):
    got = L.stable_interval(scheme, lam_min=1e-6, anchor=0.9)
    assert abs(got[1] - hi) < 1e-9
    if lo == 0.0:
        assert got[0] <= 1.001e-6      # stable down to the smallest eigenvalue sampled
    else:
        assert abs(got[0] - lo) < 1e-9
    assert L.root_condition(scheme.a)


def test_boundary_roots_of_sbdf3():
    """At lambda = 1/2 two roots sit at e^{+-i pi/3} (and one at 1/2); at 8/7 one at -1."""
    r = np.sort_complex(L.char_roots(L.SBDF3, 0.5))
    assert np.allclose(sorted(np.abs(r)), [0.5, 1.0, 1.0], atol=1e-12)
    on = r[np.abs(np.abs(r) - 1.0) < 1e-9]
    assert np.allclose(sorted(np.angle(on)), [-math.pi / 3, math.pi / 3], atol=1e-9)
    assert np.min(np.abs(L.char_roots(L.SBDF3, 8.0 / 7.0) + 1.0)) < 1e-9


def test_sbdf2_decay_rate():
    """|z| = sqrt(1 - lambda) for lambda in (0, 1): both roots of z^2 - 2(1-l)z + (1-l)."""
    for lam in (0.01, 0.3, 0.9):
        assert np.allclose(np.abs(L.char_roots(L.SBDF2, lam)), math.sqrt(1.0 - lam), atol=1e-12)


def test_sbdf3r_is_sbdf3_at_r0():
    s = L.sbdf3r(0.0)
    assert np.allclose(s.a, L.SBDF3.a, atol=1e-14)
    assert np.allclose(s.b, L.SBDF3.b, atol=1e-14)
    assert np.allclose(s.c, L.SBDF3.c, atol=1e-14)


@pytest.mark.parametrize("r", [0.0, 0.3, 0.6, 0.85, 0.95])
def test_sbdf3r_interval_and_order_conditions(r):
    s = L.sbdf3r(r)
    lo, hi = L.sbdf3r_interval(r)
    got = L.stable_interval(s, anchor=math.sqrt(lo * hi))
    assert abs(got[0] - lo) < 1e-9 * max(1.0, lo) and abs(got[1] - hi) < 1e-9 * hi
    a, b, c = np.array(s.a), np.array(list(s.b) + [0.0]), np.array(s.c)
    j = np.arange(4, dtype=float)
    # explicit (a, b) and implicit (a, c) pairs of order 3; the k = 4 condition fails
    for k in range(0, 4):
        lhs = np.sum(a * j ** k)
        assert abs(lhs - (k * np.sum(b * j ** (k - 1)) if k else 0.0)) < 1e-12
        assert abs(lhs - (k * np.sum(c * j ** (k - 1)) if k else 0.0)) < 1e-12
    assert abs(np.sum(a * j ** 4) - 4 * np.sum(b * j ** 3)) > 1e-6
    # constraint defect: sum (c_j - b_j) j^k = 0 for k = 0, 1, 2, not for k = 3
    for k in range(3):
        assert abs(np.sum((c - b) * j ** k)) < 1e-12
    assert abs(np.sum((c - b) * j ** 3)) > 1e-6
    assert L.root_condition(s.a)


def test_order_three_schemes_are_unstable_near_zero():
    """For a third-order constraint recurrence c - b has a triple root at 1, so a
    root leaves the unit disk as lambda -> 0: D never reaches down to 0."""
    for r in (0.0, 0.5, 0.9):
        assert not L.zero_stable(L.sbdf3r(r), 1e-4)
    assert L.zero_stable(L.SBDF2, 1e-4)


def _pair(eigs, rng):
    """Dense SPD A and G = A^{1/2} Q diag(eigs) Q^T A^{1/2}: generalised eigenvalues eigs."""
    n = len(eigs)
    M = rng.normal(size=(n, n))
    A = M @ M.T + n * np.eye(n)
    w, V = np.linalg.eigh(A)
    Ah = V @ np.diag(np.sqrt(w)) @ V.T
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    G = Ah @ Q @ np.diag(eigs) @ Q.T @ Ah
    return A, G


def _recurrence_growth(scheme, A, G, steps, rng, theta=1.0):
    """Iterate Eq:ZeroS3 (dt = 0, w = 0) with A -> theta A: c_s theta A p_{n+s} =
    sum_j b_j (theta A - G) p_{n+j} - sum_{j<s} c_j theta A p_{n+j}."""
    s = scheme.steps
    At = theta * A
    ps = [rng.normal(size=A.shape[0]) for _ in range(s)]
    n0 = max(np.linalg.norm(p) for p in ps)
    for _ in range(steps):
        rhs = sum(scheme.b[j] * ((At - G) @ ps[j]) for j in range(s)) - sum(scheme.c[j] * (At @ ps[j])
                                                                            for j in range(s))
        ps = ps[1:] + [np.linalg.solve(scheme.c[s] * At, rhs)]
    return max(np.linalg.norm(p) for p in ps) / n0


def test_brute_force_recurrence_agrees_with_the_checker():
    rng = np.random.default_rng(I.SEED_BASE + 90)
    inside = np.array([0.55, 0.7, 0.9, 1.0, 1.1])     # within SBDF3's (1/2, 8/7)
    outside = np.array([0.3, 0.7, 0.9, 1.0])          # 0.3 < 1/2
    A, G = _pair(inside, rng)
    assert _recurrence_growth(L.SBDF3, A, G, 400, rng) < 1e-3
    A, G = _pair(outside, rng)
    assert _recurrence_growth(L.SBDF3, A, G, 400, rng) > 1e6
    # SBDF3(r) with the joint choice for kappa = 1/0.3 damps the same pair
    r, th = L.choose_sbdf3r(1.0 / 0.3)
    assert _recurrence_growth(L.sbdf3r(r), A, G, 400, rng, theta=th) < 0.05
    # and SBDF2 is stable for any eigenvalue in (0, 1]
    A, G = _pair(np.array([1e-3, 0.01, 0.5, 1.0]), rng)
    assert _recurrence_growth(L.SBDF2, A, G, 400, rng) < 10.0


@pytest.mark.parametrize("kappa", [1.0, 1.728, 5.0, 17.6, 67.0, 338.9])
def test_joint_choice_places_the_spectrum_inside_D(kappa):
    margin = 1.1
    r, th = L.choose_sbdf3r(kappa, margin)
    lo, hi = L.sbdf3r_interval(r)
    e_lo, e_hi = 1.0 / (th * kappa), 1.0 / th
    assert e_lo >= lo * margin * (1 - 1e-9) and e_hi <= hi / margin * (1 + 1e-9)
    # the smallest such r: a slightly smaller one is too narrow (unless r = 0)
    if r > 0:
        assert L.sbdf3r_ratio(r - 1e-6) < kappa * margin * margin
    s = L.sbdf3r(r)
    for lam in np.geomspace(e_lo, e_hi, 25):
        assert L.zero_stable(s, lam)


def _flat_wave():
    g = I.grid1d(256, 80.0)
    h = np.ones(g.shape)
    eta, u = I.solitary_wave(g, 1.0, 0.2, 20.0)
    return g, h, eta, u


def test_generic_stepper_with_sbdf2_coefficients_equals_eq_mm():
    g = I.grid1d(512, 80.0)
    x = I.coords(g)
    h = 1.0 - 0.4 * np.exp(-((x - 45.0) / 6.0) ** 2)
    es, u = I.solitary_wave(g, 1.0, 0.3, 35.0)
    eta = h + es - 1.0
    pb1 = ost.Problem.from_h(g, h, tol=1e-12)
    pb2 = ost.Problem.from_h(g, h, tol=1e-12)
    U0 = pb1.G(eta, u)
    a = ost.run_sbdf2(pb1, eta, U0, u, 0.05, 8)
    b = L.run_linimp(pb2, L.SBDF2, eta, U0, u, 0.05, 8)
    for x1, x2 in zip(a, b):
        assert np.array_equal(x1, x2)


@pytest.mark.parametrize("member", ["chosen", "r=0.5"])
def test_sbdf3r_converges_at_third_order_on_the_exact_solitary_wave(member):
    g, h, eta, u = _flat_wave()
    T = 2.0
    e_x, u_x = I.solitary_wave(g, 1.0, 0.2, 20.0, t=T)
    pb = ost.Problem.from_h(g, h, tol=1e-13)
    _, _, kap = op.coefficients(eta, pb.grad_h, pb.flat)
    if member == "chosen":
        r, th = L.choose_sbdf3r(kap)
        assert r == 0.0                  # flat bottom, kappa_ub = 1.2^3: plain SBDF3 with a scaled A
    else:
        r = 0.5                          # a member with c_0, c_1, c_2 != 0, A centred in its D
        lo, hi = L.sbdf3r_interval(r)
        th = 1.0 / math.sqrt(lo * hi * kap)
    errs = []
    for dt in (0.1, 0.05, 0.025):
        pb = ost.Problem.from_h(g, h, tol=1e-13)
        e, U, uu = L.run_linimp(pb, L.sbdf3r(r), eta, pb.G(eta, u), u, dt, int(round(T / dt)), theta=th)
        errs.append(dg.rel_l2(e - 1.0, e_x - 1.0))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(2.8 < q < 3.3 for q in rates), (errs, rates)


@pytest.mark.parametrize("r", [0.0, 0.6, 0.9])
def test_sbdf3r_conserves_mass_to_rounding(r):
    """Remark 2.1: the mass integral of zeta is conserved; the update keeps it to
    rounding over many steps (its coefficients satisfy a(1) = 0 exactly)."""
    g = I.grid1d(512, 80.0)
    x = I.coords(g)
    h = 1.0 - 0.4 * np.exp(-((x - 45.0) / 6.0) ** 2)
    es, u = I.solitary_wave(g, 1.0, 0.3, 35.0)
    eta = h + es - 1.0
    pb = ost.Problem.from_h(g, h, tol=1e-12)
    lo, hi = L.sbdf3r_interval(r)
    _, _, kap = op.coefficients(eta, pb.grad_h, pb.flat)
    th = 1.0 / math.sqrt(lo * hi * min(kap, 0.8 * hi / lo))
    e, _, _ = L.run_linimp(pb, L.sbdf3r(r), eta, pb.G(eta, u), u, 0.05, 60, theta=th)
    m0 = dg.mass(eta, h, g)
    assert abs(dg.mass(e, h, g) - m0) <= 1e-12


@pytest.mark.slow
def test_plain_sbdf3_blows_up_over_the_shelf_while_the_joint_choice_does_not():
    c = I.config_c2()
    g = c["grid"]
    pb = ost.Problem.from_h(g, c["h"], tol=1e-12)
    _, _, kap = op.coefficients(c["eta"], pb.grad_h, pb.flat)
    assert kap > 300
    U0 = pb.G(c["eta"], c["u"])
    with np.errstate(all="ignore"):
        e, _, _ = L.run_linimp(ost.Problem.from_h(g, c["h"], tol=1e-12), L.SBDF3, c["eta"], U0, c["u"], 0.02, 400)
    assert not np.all(np.isfinite(e)) or np.max(np.abs(e - c["h"])) > 10.0
    r, th = L.choose_sbdf3r(kap)
    e, _, u = L.run_linimp(ost.Problem.from_h(g, c["h"], tol=1e-12), L.sbdf3r(r), c["eta"], U0, c["u"], 0.02, 400,
                           theta=th)
    assert np.all(np.isfinite(e)) and np.max(np.abs(e - c["h"])) < 0.35
