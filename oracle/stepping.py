"""Time integrators for the index-1 DAE  w_t = f(w, p), G_{eta,h} p = U  (section 5).

w = (eta, U), p = u.  Test infrastructure only.

rk4_step  : classical RK4 (Eq:ERK) with one PCG solve per stage.  Readings of
            the printed stage equations: the U stage starts from U_n (the text
            prints u_n), the stage constraint is G u^(i) = U^(i) (the text
            prints U^(j)), and the final update advances U (the text prints u),
            after which u_{n+1} is solved for.  Stage 1 reuses u_n, so a step
            costs 4 solves.  Initial guesses (reading: the paper leaves them
            open) come from GuessHistory: the most recent velocity, or that
            velocity plus the same solve's offset from earlier steps,
            extrapolated in time.
ab_step   : Adams-Bashforth of order s = 2, 3, 4 (Eq:AB, Table LMMCoeffs), one
            PCG solve per step; the first s-1 steps are RK4 steps with the same
            dt (reading: the paper does not state a start-up).
sbdf2_step: the linearly implicit scheme Eq:MM with the SBDF2 coefficients of
            Table LMMCoeffs: one A-solve per step, no Krylov iteration.  The
            coefficients of A are held fixed over the run, taken from the
            initial data (section 6.5); the first step is one RK4 step.
Coefficients of A for every PCG solve are recomputed from the current eta
(section 5.1 allows this).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import krylov, operators as op
from .rhs import rhs, rhs_dealiased

RK4_A = ((), (0.5,), (0.0, 0.5), (0.0, 0.0, 1.0))
RK4_B = (1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0)

# Adams-Bashforth b_j, j = 0 .. s-1 (Table LMMCoeffs); a = (0, .., -1, 1)
AB_B = {
    2: (-1.0 / 2.0, 3.0 / 2.0),
    3: (5.0 / 12.0, -16.0 / 12.0, 23.0 / 12.0),
    4: (-9.0 / 24.0, 37.0 / 24.0, -59.0 / 24.0, 55.0 / 24.0),
}
# SBDF2 (Table LMMCoeffs)
SBDF2_A = (0.5, -2.0, 1.5)
SBDF2_B = (-1.0, 2.0)


class GuessHistory:
    """Initial guesses of the constraint solves inside the steppers.

    Each solve has a slot (RK4 stages 2, 3, 4, the final RK4 solve, the
    Adams-Bashforth solve) and a base: the most recent velocity when the solve
    starts.  mode 'previous' starts every solve from its base (plain warm
    start).  mode 'extrapolate' records the slot's offset o_n = solution - base
    after every solve and starts the next solve of that slot from
    base + o_{n-1} (one offset recorded) or base + 2 o_{n-1} - o_{n-2} (two or
    more), the value at the next step of the polynomial through the recorded
    offsets.  The offsets scale with the step, so a change of dt clears them.
    A guess only changes where the Krylov iteration starts, not the solution
    it converges to (the stop test is on the residual)."""

    SLOTS = ("rk2", "rk3", "rk4", "rk_final", "ab")

    def __init__(self, mode: str = "extrapolate"):
        if mode not in ("previous", "extrapolate"):
            raise ValueError("mode must be 'previous' or 'extrapolate'")
        self.mode = mode
        self.dt = None
        self.offsets = {k: [] for k in self.SLOTS}

    def prepare(self, dt):
        if self.dt != dt:
            self.clear()
            self.dt = dt

    def clear(self, slot=None):
        for k in ([slot] if slot else self.SLOTS):
            self.offsets[k] = []

    def guess(self, slot, base):
        o = self.offsets[slot]
        if self.mode == "previous" or not o:
            return base
        if len(o) == 1:
            return base + o[-1]
        return base + (2.0 * o[-1] - o[-2])

    def record(self, slot, base, solution):
        if self.mode == "previous":
            return
        o = self.offsets[slot]
        o.append(solution - base)
        del o[:-2]


@dataclass
class Problem:
    g: object
    h: np.ndarray
    grad_h: np.ndarray
    flat: bool
    tol: float = 1e-12
    max_iter: int = 1000
    iters: list = field(default_factory=list)
    hist: GuessHistory = field(default_factory=GuessHistory)
    dealias: int = 1   # > 1: the right-hand side is the de-aliased one, padded by this factor

    @classmethod
    def from_h(cls, g, h, tol=1e-12, max_iter=1000, guess="extrapolate", dealias=1):
        gh, fl = op.bathy_gradient(h, g)
        return cls(g, np.asarray(h, dtype=np.float64), gh, fl, tol, max_iter, hist=GuessHistory(guess),
                   dealias=dealias)

    def f(self, eta, u):
        if self.dealias > 1:
            return rhs_dealiased(eta, u, self.h, self.g, self.dealias)
        return rhs(eta, u, self.h, self.grad_h, self.g)

    def G(self, eta, u):
        return op.apply_G(eta, self.grad_h, u, self.g)

    def A(self, sigma, alpha, u):
        return op.apply_A(sigma, alpha, u, self.g)

    def A_inv(self, sigma, alpha, r):
        return op.solve_A(sigma, alpha, r, self.g)

    def solve(self, eta, U, x0):
        """PCG solve of G_{eta,h} u = U, A built from the current eta."""
        s, a, _ = op.coefficients(eta, self.grad_h, self.flat)
        u, it, ok, _ = krylov.pcg(lambda v: self.G(eta, v),
                                  lambda r: self.A_inv(s, a, r),
                                  U, x0=x0, tol=self.tol, max_iter=self.max_iter)
        if not ok:
            raise RuntimeError("PCG did not converge")
        self.iters.append(it)
        return u

    def stage_solve(self, slot, eta, U, base):
        """Solve G u = U for one stepper slot, starting from the slot's guess."""
        u = self.solve(eta, U, self.hist.guess(slot, base))
        self.hist.record(slot, base, u)
        return u


def rk4_step(pb: Problem, eta, U, u, dt):
    pb.hist.prepare(dt)
    fe, fU = [], []
    u_last = u
    for i in range(4):
        if i == 0:
            eta_i, u_i = eta, u
        else:
            eta_i = eta.copy()
            U_i = U.copy()
            for j, aij in enumerate(RK4_A[i]):
                if aij != 0.0:
                    eta_i = eta_i + dt * aij * fe[j]
                    U_i = U_i + dt * aij * fU[j]
            u_i = pb.stage_solve(GuessHistory.SLOTS[i - 1], eta_i, U_i, u_last)
            u_last = u_i
        e_t, U_t = pb.f(eta_i, u_i)
        fe.append(e_t)
        fU.append(U_t)
    eta_new = eta + dt * (RK4_B[0] * fe[0] + RK4_B[1] * fe[1] + RK4_B[2] * fe[2] + RK4_B[3] * fe[3])
    U_new = U + dt * (RK4_B[0] * fU[0] + RK4_B[1] * fU[1] + RK4_B[2] * fU[2] + RK4_B[3] * fU[3])
    u_new = pb.stage_solve("rk_final", eta_new, U_new, u_last)
    return eta_new, U_new, u_new


def run_rk4(pb: Problem, eta, U, u, dt, nsteps):
    for _ in range(nsteps):
        eta, U, u = rk4_step(pb, eta, U, u, dt)
    return eta, U, u


def run_ab(pb: Problem, order, eta, U, u, dt, nsteps):
    """AB_s for nsteps steps in total (the first s-1 are RK4 start-up steps)."""
    b = AB_B[order]
    pb.hist.prepare(dt)
    pb.hist.clear("ab")
    hist = []                                 # (f_eta, f_U) at levels n .. n+s-1
    done = 0
    while done < nsteps:
        if len(hist) < order - 1:
            hist.append(pb.f(eta, u))
            eta, U, u = rk4_step(pb, eta, U, u, dt)
            done += 1
            continue
        hist.append(pb.f(eta, u))
        hist = hist[-order:]
        eta_new = eta.copy()
        U_new = U.copy()
        for j in range(order):
            eta_new = eta_new + dt * b[j] * hist[j][0]
            U_new = U_new + dt * b[j] * hist[j][1]
        u = pb.stage_solve("ab", eta_new, U_new, u)
        eta, U = eta_new, U_new
        done += 1
    return eta, U, u


def sbdf2_coefficients(pb: Problem, eta0):
    s, a, _ = op.coefficients(eta0, pb.grad_h, pb.flat)
    return s, a


def run_sbdf2(pb: Problem, eta, U, u, dt, nsteps, coeffs=None):
    """Linearly implicit SBDF2 (Eq:MM) for nsteps steps (the first is an RK4 step).

    w_{n+2} = (2 w_{n+1} - w_n/2 + dt (2 f_{n+1} - f_n)) / (3/2)
    A u_{n+2} = 2 R_{n+1} - R_n,  R_k = A u_k - G_{eta_k} u_k + U_k.
    """
    sig, alp = coeffs if coeffs is not None else sbdf2_coefficients(pb, eta)

    def R(eta_k, U_k, u_k):
        return pb.A(sig, alp, u_k) - pb.G(eta_k, u_k) + U_k

    if nsteps <= 0:
        return eta, U, u
    f0 = pb.f(eta, u)
    R0 = R(eta, U, u)
    w0 = (eta, U)
    eta1, U1, u1 = rk4_step(pb, eta, U, u, dt)
    done = 1
    while done < nsteps:
        f1 = pb.f(eta1, u1)
        R1 = R(eta1, U1, u1)
        a0, a1, a2 = SBDF2_A
        b0, b1 = SBDF2_B
        eta2 = (-a0 * w0[0] - a1 * eta1 + dt * (b0 * f0[0] + b1 * f1[0])) / a2
        U2 = (-a0 * w0[1] - a1 * U1 + dt * (b0 * f0[1] + b1 * f1[1])) / a2
        u2 = pb.A_inv(sig, alp, b0 * R0 + b1 * R1)
        w0, f0, R0 = (eta1, U1), f1, R1
        eta1, U1, u1 = eta2, U2, u2
        done += 1
    return eta1, U1, u1
