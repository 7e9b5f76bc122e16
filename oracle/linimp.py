"""Linearly implicit multistep schemes for the SGN DAE and their zero-stability
(section 5.3 Subsec:IMEX_LMM, Eq:IMEX_DAE, Eq:MM; section 5.4
subsec:zerostability, Eq:PolynomialCoeff, Eq:CharEq, Fig:StabilityRegion).
Test infrastructure only.

A scheme of s steps is given by coefficients a_j, c_j (j = 0..s) and b_j
(j = 0..s-1):
    sum_j a_j w_{n+j} = dt sum_j b_j f(w_{n+j}, p_{n+j})
    sum_j c_j A p_{n+j} = sum_j b_j (A p_{n+j} - G_{n+j} p_{n+j} + U_{n+j})
(Eq:IMEX_DAE with g = G p - U; the sum on the right of the zero-stability
recurrence starts at j = 0, the printed j = 1 being read as a typo).  Applied
with dt = 0 to a linear constraint, a mode of A^{-1} G with eigenvalue lambda
evolves by the roots z of
    c(z) - b(z) + lambda b(z) = 0                        (Eq:CharEq)
and the scheme is zero-stable if every such root lies in |z| < 1 for every
eigenvalue, given that a(z) satisfies the root condition.  Theorem 4.1 puts the
eigenvalues of A^{-1} G in [1/kappa_ub, 1].

SBDF1 and SBDF2 contain (0, 1]; SBDF3 only (1/2, 8/7), so it fails once an
eigenvalue falls below 1/2 (Fig:StabilityRegion: "lambda > 2" read for the
eigenvalues of G^{-1} A).  The paper leaves the higher-order construction to
the joint choice of A and the coefficients.  The reading built here (a
one-parameter family, "SBDF3(r)"):
    c(z) = (z - r)^3,   b(z) = c(z) - (z - 1)^3,   a(z) from the third-order
    conditions  sum_j a_j j^k = k sum_j c_j j^(k-1),  k = 0..3,
so that (a, b) is a third-order explicit pair, (a, c) a third-order implicit
one, and the constraint recurrence has defect O(dt^3) (c - b has a triple root
at 1).  r = 0 is SBDF3.  On the real axis
    D = ( 1 / (1 + (1 + r)^3),  1 / (1 - ((1 + r) / 2)^3) ),
and A is scaled by theta so that [1/(theta kappa), 1/theta] sits inside D with
a margin on both sides.  The width of D grows without bound as r -> 1, at the
price of a larger error constant.

Derivation of D for SBDF3(r): lambda (z - r)^3 + (1 - lambda)(z - 1)^3 = 0,
i.e. ((z - r)/(z - 1))^3 = -(1 - lambda)/lambda =: t^3.  From z - r = t (z - 1),
|z| < 1 iff |t - r| < |t - 1| iff Re t < (1 + r)/2.  For lambda in (0, 1] the
cube roots t = rho e^{i pi/3}, rho e^{-i pi/3}, -rho with
rho = ((1 - lambda)/lambda)^{1/3} give the condition rho/2 < (1 + r)/2; for
lambda > 1 the roots t = rho, rho e^{+-2 pi i/3} give rho < (1 + r)/2.
"""
from __future__ import annotations

from dataclasses import dataclass
from math import sqrt

import numpy as np

from . import stepping as st


@dataclass(frozen=True)
class Scheme:
    """Coefficients of an s-step linearly implicit scheme, lowest index first:
    a, c of length s + 1, b of length s."""

    name: str
    a: tuple
    b: tuple
    c: tuple

    @property
    def steps(self) -> int:
        return len(self.a) - 1


# Table LMMCoeffs (SBDF2) and the first- and third-order members of the family
# shown in Fig:StabilityRegion (BDF coefficients with extrapolated explicit terms)
SBDF1 = Scheme("SBDF1", (-1.0, 1.0), (1.0,), (0.0, 1.0))
SBDF2 = Scheme("SBDF2", (0.5, -2.0, 1.5), (-1.0, 2.0), (0.0, 0.0, 1.0))
SBDF3 = Scheme("SBDF3", (-1.0 / 3.0, 1.5, -3.0, 11.0 / 6.0), (1.0, -3.0, 3.0), (0.0, 0.0, 0.0, 1.0))


def poly(coeffs, z):
    """sum_j coeffs[j] z^j."""
    return sum(cj * z ** j for j, cj in enumerate(coeffs))


def char_roots(scheme: Scheme, lam: float):
    """Roots of c(z) - b(z) + lam b(z) (Eq:CharEq)."""
    p = np.array(scheme.c, dtype=np.complex128)
    p[: len(scheme.b)] -= (1.0 - lam) * np.asarray(scheme.b)
    return np.roots(p[::-1])


def zero_stable(scheme: Scheme, lam: float, strict: float = 0.0) -> bool:
    """Every root of Eq:CharEq has |z| < 1 - strict."""
    return bool(np.max(np.abs(char_roots(scheme, lam))) < 1.0 - strict)


def root_condition(a, tol: float = 1e-9) -> bool:
    """Roots of a(z) in the closed unit disk, those on the circle simple."""
    r = np.roots(np.asarray(a, dtype=np.float64)[::-1])
    if np.any(np.abs(r) > 1.0 + tol):
        return False
    on = r[np.abs(np.abs(r) - 1.0) <= tol]
    for i in range(len(on)):
        for j in range(i + 1, len(on)):
            if abs(on[i] - on[j]) <= 1e-6:
                return False
    return True


def stable_interval(scheme: Scheme, lam_min: float = 1e-6, lam_max: float = 1e3, samples: int = 4000,
                    anchor: float | None = None):
    """The real interval of lambda around `anchor` on which the scheme is zero-stable
    (sampled on a log grid, ends refined by bisection).  None if the anchor is
    unstable.  anchor defaults to the geometric centre of the stable samples."""
    lam = np.geomspace(lam_min, lam_max, samples)
    ok = np.array([zero_stable(scheme, l) for l in lam])
    if not ok.any():
        return None
    if anchor is None:
        idx = np.where(ok)[0]
        runs = np.split(idx, np.where(np.diff(idx) != 1)[0] + 1)
        run = max(runs, key=len)
        i0, i1 = run[0], run[-1]
    else:
        if not zero_stable(scheme, anchor):
            return None
        i = int(np.searchsorted(lam, anchor))
        i0 = i1 = min(i, samples - 1)
        while i0 > 0 and ok[i0 - 1]:
            i0 -= 1
        while i1 < samples - 1 and ok[i1 + 1]:
            i1 += 1

    def bisect(good, bad):
        for _ in range(80):
            mid = sqrt(good * bad)
            if zero_stable(scheme, mid):
                good = mid
            else:
                bad = mid
        return good

    lo = lam[i0] if i0 == 0 else bisect(lam[i0], lam[i0 - 1])
    hi = lam[i1] if i1 == samples - 1 else bisect(lam[i1], lam[i1 + 1])
    return float(lo), float(hi)


# ---------------------------------------------------------------------------
# The SBDF3(r) family and the joint choice of (r, theta)
# ---------------------------------------------------------------------------

def sbdf3r(r: float) -> Scheme:
    """c(z) = (z - r)^3, b(z) = c(z) - (z - 1)^3 and a(z) from the third-order
    conditions sum_j a_j j^k = k sum_j c_j j^(k-1), k = 0..3."""
    if not 0.0 <= r < 1.0:
        raise ValueError("r must lie in [0, 1)")
    c = np.array([-r ** 3, 3.0 * r * r, -3.0 * r, 1.0])
    cube = np.array([-1.0, 3.0, -3.0, 1.0])            # (z - 1)^3
    b = (c - cube)[:3]
    # k = 0: sum a_j = 0; k >= 1: sum a_j j^k = k sum c_j j^(k-1) (with 0^0 = 1)
    M = np.array([[float(j) ** k if (j or k) else 1.0 for j in range(4)] for k in range(4)])
    rhs = np.zeros(4)
    for k in range(1, 4):
        rhs[k] = k * sum(c[j] * (float(j) ** (k - 1) if (j or k - 1) else 1.0) for j in range(4))
    a = np.linalg.solve(M, rhs)
    # consistency a(1) = 0 held exactly in floating point, in the order the update
    # sums its terms, so that a constant level (and the mass, Remark 2.1) is kept
    a[3] = -((a[0] + a[1]) + a[2])
    return Scheme(f"SBDF3(r={r:g})", tuple(a), tuple(b), tuple(c))


def sbdf3r_interval(r: float):
    """Closed form of D on the real axis for SBDF3(r) (module docstring)."""
    return 1.0 / (1.0 + (1.0 + r) ** 3), 1.0 / (1.0 - (0.5 * (1.0 + r)) ** 3)


def sbdf3r_ratio(r: float) -> float:
    lo, hi = sbdf3r_interval(r)
    return hi / lo


def choose_sbdf3r(kappa: float, margin: float = 1.1):
    """Joint choice of the scheme and of A's scale for eigenvalues of A^{-1} G in
    [1/kappa, 1] (Theorem 4.1): the smallest r whose interval D is at least
    kappa margin^2 wide, and theta with A -> theta A placing the scaled interval
    [1/(theta kappa), 1/theta] at the geometric centre of D (a factor of at least
    `margin` from either end).  Returns (r, theta)."""
    if not (kappa >= 1.0 and margin >= 1.0):
        raise ValueError("kappa >= 1 and margin >= 1 required")
    need = kappa * margin * margin
    if sbdf3r_ratio(0.0) >= need:
        r = 0.0
    else:
        lo, hi = 0.0, 1.0 - 1e-15
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if sbdf3r_ratio(mid) >= need:
                hi = mid
            else:
                lo = mid
        r = hi
    lam_lo, lam_hi = sbdf3r_interval(r)
    theta = 1.0 / sqrt(lam_lo * lam_hi * kappa)
    return r, theta


def error_constant(scheme: Scheme, p: int) -> float:
    """Error constant of the explicit pair (a, b) of order p, normalised by b(1):
    (sum a_j j^(p+1)/(p+1)! - sum b_j j^p/p!) / sum b_j."""
    from math import factorial
    a, b = scheme.a, scheme.b
    C = (sum(a[j] * float(j) ** (p + 1) for j in range(len(a))) / factorial(p + 1)
         - sum(b[j] * float(j) ** p for j in range(len(b))) / factorial(p))
    return C / sum(b)


# ---------------------------------------------------------------------------
# Stepping (Eq:IMEX_DAE applied to the SGN constraint form, Eq:MM for SBDF2)
# ---------------------------------------------------------------------------

def run_linimp(pb: st.Problem, scheme: Scheme, eta, U, u, dt, nsteps, coeffs=None, theta: float = 1.0):
    """nsteps steps of the linearly implicit scheme, the first s-1 of them RK4
    start-up steps with the same dt (reading: the paper states no start-up).
    A = theta (sigma I - alpha grad div) with (sigma, alpha) = coeffs, or the
    coefficients of the initial eta (section 6.5 keeps them fixed over the run).
        w_{n+s}   = (-sum_{j<s} a_j w_{n+j} + dt sum_j b_j f_{n+j}) / a_s
        A u_{n+s} = (sum_j b_j R_{n+j} - sum_{j<s} c_j A u_{n+j}) / c_s,
        R_k = A u_k - G_{eta_k} u_k + U_k."""
    s = scheme.steps
    a, b, c = scheme.a, scheme.b, scheme.c
    sig, alp = coeffs if coeffs is not None else st.sbdf2_coefficients(pb, eta)
    sig, alp = theta * sig, theta * alp
    if nsteps <= 0:
        return eta, U, u
    hist = []           # per level: (eta, U, f_eta, f_U, R, A u)
    done = 0

    def level(eta_k, U_k, u_k):
        fe, fU = pb.f(eta_k, u_k)
        Au = pb.A(sig, alp, u_k)
        return (eta_k, U_k, fe, fU, Au - pb.G(eta_k, u_k) + U_k, Au)

    while done < nsteps and len(hist) < s - 1:
        hist.append(level(eta, U, u))
        eta, U, u = st.rk4_step(pb, eta, U, u, dt)
        done += 1
    while done < nsteps:
        hist.append(level(eta, U, u))
        hist = hist[-s:]
        eta_n = sum(-a[j] * hist[j][0] for j in range(s)) + dt * sum(b[j] * hist[j][2] for j in range(s))
        U_n = sum(-a[j] * hist[j][1] for j in range(s)) + dt * sum(b[j] * hist[j][3] for j in range(s))
        rhs = sum(b[j] * hist[j][4] for j in range(s)) - sum(c[j] * hist[j][5] for j in range(s))
        eta, U = eta_n / a[s], U_n / a[s]
        u = pb.A_inv(sig, alp, rhs / c[s])
        done += 1
    return eta, U, u
