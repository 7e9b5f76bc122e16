"""Krylov solvers for G u = b (section 3.2).  Test infrastructure only.

pcg   : textbook preconditioned conjugate gradient, preconditioner solves only
        (section 3.2, Eq:PCGLinSyst).  Stop rule (reading; the paper does not
        state one): the recursively updated residual satisfies
        ||r_k||_2 <= tol ||b||_2, the relative-residual test of the MATLAB pcg
        routine the paper's computations used.
gmres : restarted, right-preconditioned GMRES with the same stop rule on the
        (unpreconditioned) residual.  The paper itself uses PCG only; GMRES is
        an option of the device library.  Pinned by manufactured systems and by
        its definition: every iterate (with and without restarts) and the
        iteration count equal a brute-force minimisation of the residual over
        each cycle's Krylov space on a dense tiny problem.
"""
from __future__ import annotations

import numpy as np


def _dot(a, b):
    return float(np.sum(a * b))


def pcg(apply_op, precond, b, x0=None, tol=1e-12, max_iter=1000, history=None):
    """Textbook PCG.  Returns (x, iters, converged, relres).

    iters counts operator applications inside the loop (one per iteration).
    history, if a list, receives each iterate x_k (k = 0, 1, ...).
    """
    b = np.asarray(b, dtype=np.float64)
    bnorm = np.sqrt(_dot(b, b))
    if bnorm == 0.0:
        x = np.zeros_like(b)
        if history is not None:
            history.append(x.copy())
        return x, 0, True, 0.0
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    r = b - apply_op(x) if x0 is not None else b.copy()
    if history is not None:
        history.append(x.copy())
    rnorm = np.sqrt(_dot(r, r))
    if rnorm <= tol * bnorm:
        return x, 0, True, rnorm / bnorm
    z = precond(r)
    p = z.copy()
    rho = _dot(r, z)
    for k in range(1, max_iter + 1):
        q = apply_op(p)
        alpha = rho / _dot(p, q)
        x = x + alpha * p
        r = r - alpha * q
        if history is not None:
            history.append(x.copy())
        rnorm = np.sqrt(_dot(r, r))
        if rnorm <= tol * bnorm:
            return x, k, True, rnorm / bnorm
        z = precond(r)
        rho_new = _dot(r, z)
        beta = rho_new / rho
        rho = rho_new
        p = z + beta * p
    return x, max_iter, False, rnorm / bnorm


def gmres(apply_op, precond, b, x0=None, tol=1e-12, max_iter=1000, restart=30):
    """Right-preconditioned restarted GMRES(m): solve (G M^{-1}) y = b, x = M^{-1} y.

    Arnoldi with modified Gram-Schmidt and Givens rotations.  Returns
    (x, iters, converged, relres) with iters = number of operator applications
    in Arnoldi steps.
    """
    b = np.asarray(b, dtype=np.float64)
    shape = b.shape
    bnorm = np.sqrt(_dot(b, b))
    if bnorm == 0.0:
        return np.zeros_like(b), 0, True, 0.0
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    iters = 0
    while True:
        r = b - apply_op(x) if (x0 is not None or iters > 0) else b.copy()
        beta = np.sqrt(_dot(r, r))
        if beta <= tol * bnorm:
            return x, iters, True, beta / bnorm
        if iters >= max_iter:
            return x, iters, False, beta / bnorm
        m = restart
        V = [r / beta]
        Z = []
        Hm = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        gvec = np.zeros(m + 1)
        gvec[0] = beta
        j_done = 0
        for j in range(m):
            zj = precond(V[j])
            Z.append(zj)
            w = apply_op(zj)
            iters += 1
            for i in range(j + 1):
                Hm[i, j] = _dot(w, V[i])
                w = w - Hm[i, j] * V[i]
            Hm[j + 1, j] = np.sqrt(_dot(w, w))
            V.append(w / Hm[j + 1, j] if Hm[j + 1, j] != 0.0 else w)
            for i in range(j):                       # apply previous rotations
                t = cs[i] * Hm[i, j] + sn[i] * Hm[i + 1, j]
                Hm[i + 1, j] = -sn[i] * Hm[i, j] + cs[i] * Hm[i + 1, j]
                Hm[i, j] = t
            den = np.hypot(Hm[j, j], Hm[j + 1, j])
            cs[j] = Hm[j, j] / den
            sn[j] = Hm[j + 1, j] / den
            Hm[j, j] = den
            Hm[j + 1, j] = 0.0
            gvec[j + 1] = -sn[j] * gvec[j]
            gvec[j] = cs[j] * gvec[j]
            j_done = j + 1
            if abs(gvec[j + 1]) <= tol * bnorm or iters >= max_iter:
                break
        y = np.linalg.solve(np.triu(Hm[:j_done, :j_done]), gvec[:j_done])
        for i in range(j_done):
            x = x + y[i] * Z[i]
        x = x.reshape(shape)
