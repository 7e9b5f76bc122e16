"""Pins of the oracle's wall (homogeneous Neumann) operators, oracle/walls.py:

* the cosine / sine series amplitudes of closed-form modes (the sine Nyquist
  mode included) and the derivative of closed-form fields;
* the same G, A^{-1} and grad h as the periodic oracle (pinned on its own)
  applied on the doubled periodic domain to the even / odd reflections of the
  fields and restricted back: a second construction of the same operator;
* G symmetric positive definite and equal to A for constant depth and a flat
  bottom; the eigenvalue interval of Theorem 4.1, which Sec:BoundonG states for
  walls as well; PCG reaching the tolerance on G u = b;
* the right-hand side between walls, and the RK4, Adams-Bashforth and SBDF2
  steppers built on the wall operators, equal to the periodic ones on the
  reflected fields (second construction again); the mass rate is zero.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import operators as op
from oracle import walls as W
from paper_2506_16045_amd import inputs as I


def test_series_amplitudes_of_closed_form_modes():
    g = I.grid1d_walls(16, 3.0)
    x = I.coords(g)
    A = W.to_modes(np.cos(3 * np.pi * x / g.Lx) + 0.5, "c")
    ref = np.zeros(17)
    ref[3], ref[0] = 1.0, 0.5
    assert np.max(np.abs(A - ref)) < 1e-14
    for m in (1, 5, 16):   # 16: the sine Nyquist mode, +-1 at the cell centres
        A = W.to_modes(np.sin(m * np.pi * x / g.Lx), "s")
        ref = np.zeros(17)
        ref[m] = 1.0
        assert np.max(np.abs(A - ref)) < 1e-14
        assert np.max(np.abs(W.from_modes(A, "s") - np.sin(m * np.pi * x / g.Lx))) < 1e-14


def test_derivatives_of_closed_forms():
    g = I.grid2d_walls(16, 8, 2.0, 1.5)
    X, Y = I.coords(g)
    kx, ky = 3 * np.pi / g.Lx, 2 * np.pi / g.Ly
    f = np.cos(kx * X) * np.cos(ky * Y)
    gr = W.grad(f, g)
    assert np.max(np.abs(gr[0] + kx * np.sin(kx * X) * np.cos(ky * Y))) < 1e-12
    assert np.max(np.abs(gr[1] + ky * np.cos(kx * X) * np.sin(ky * Y))) < 1e-12
    mx, my = 5 * np.pi / g.Lx, 3 * np.pi / g.Ly
    u = np.stack([np.sin(mx * X) * np.cos(ky * Y), np.cos(kx * X) * np.sin(my * Y)])
    d = W.div(u, g)
    ref = mx * np.cos(mx * X) * np.cos(ky * Y) + my * np.cos(kx * X) * np.cos(my * Y)
    assert np.max(np.abs(d - ref)) < 1e-12
    # the sine Nyquist mode has no derivative (section 6.1 convention)
    g1 = I.grid1d_walls(16, 2.0)
    x = I.coords(g1)
    assert np.max(np.abs(W.div(np.sin(16 * np.pi * x / g1.Lx)[None], g1))) < 1e-12


# ---- reflection onto the doubled periodic domain ------------------------------------
def reflect(f, kinds):
    """Even ('c') / odd ('s') reflection of samples across the walls, per axis (array
    order), onto the periodic domain of twice the length."""
    out = f
    for ax, k in enumerate(kinds):
        mirror = np.flip(out, axis=ax) * (1.0 if k == "c" else -1.0)
        out = np.concatenate([out, mirror], axis=ax)
    return out


def restrict(F, g):
    return F[..., :g.nx] if g.d == 1 else F[..., :g.ny, :g.nx]


def periodic_twin(g):
    if g.d == 1:
        return I.grid1d(2 * g.nx, 2 * g.Lx)
    return I.grid2d(2 * g.nx, 2 * g.ny, 2 * g.Lx, 2 * g.Ly)


def _fields(g, rng, flat=False):
    eta = I.random_positive_depth(g, rng, 0.6, 1.6)
    h = np.full(g.shape, 1.0) if flat else 1.0 + 0.3 * I.random_smooth_field(g, rng, modes=3)
    u = rng.normal(size=(g.d,) + g.shape)
    return eta, h, u


WALL_GRIDS = [I.grid1d_walls(32, 3.0), I.grid2d_walls(16, 8, 2.0, 1.5)]
IDS = ["1d", "2d"]


@pytest.mark.parametrize("g", WALL_GRIDS, ids=IDS)
def test_wall_operators_equal_periodic_ones_on_the_reflected_domain(g, rng):
    eta, h, u = _fields(g, rng)
    g2 = periodic_twin(g)
    sc = W.SCALAR[g.d]
    vk = W.VECTOR[g.d]
    E = lambda f: reflect(f, sc)  # noqa: E731
    Ev = lambda v: np.stack([reflect(v[c], vk[c]) for c in range(g.d)])  # noqa: E731
    gh, flat = W.bathy_gradient(h, g)
    gh2, _ = op.bathy_gradient(E(h), g2)
    assert np.max(np.abs(restrict(gh2, g) - gh)) < 1e-11
    Gu = W.apply_G(eta, gh, u, g)
    Gu2 = op.apply_G(E(eta), gh2, Ev(u), g2)
    assert np.max(np.abs(restrict(Gu2, g) - Gu)) < 1e-10 * np.max(np.abs(Gu))
    z = W.solve_A(1.3, 0.7, u, g)
    z2 = op.solve_A(1.3, 0.7, Ev(u), g2)
    assert np.max(np.abs(restrict(z2, g) - z)) < 1e-12 * np.max(np.abs(z))


@pytest.mark.parametrize("g", [I.grid1d_walls(16, 3.0), I.grid2d_walls(6, 4, 2.0, 1.5)], ids=IDS)
def test_dense_G_symmetric_positive_definite_and_A_for_flat(g, rng):
    eta, h, _ = _fields(g, rng)
    gh, _ = W.bathy_gradient(h, g)
    G = W.dense(lambda v: W.apply_G(eta, gh, v, g), g)
    assert np.max(np.abs(G - G.T)) < 1e-10 * np.max(np.abs(G))
    assert np.min(np.linalg.eigvalsh(0.5 * (G + G.T))) > 0
    c = 1.3
    G0 = W.dense(lambda v: W.apply_G(np.full(g.shape, c), np.zeros((g.d,) + g.shape), v, g), g)
    A0 = W.dense(lambda v: W.apply_A(c, c ** 3 / 3.0, v, g), g)
    assert np.max(np.abs(G0 - A0)) < 1e-11 * np.max(np.abs(A0))
    Ainv = W.dense(lambda v: W.solve_A(c, c ** 3 / 3.0, v, g), g)
    assert np.max(np.abs(Ainv @ A0 - np.eye(A0.shape[0]))) < 1e-11


@pytest.mark.parametrize("g", [I.grid1d_walls(32, 2.0), I.grid2d_walls(8, 8, 1.0, 1.0)], ids=IDS)
@pytest.mark.parametrize("flat", [True, False])
def test_theorem_4_1_eigenvalue_interval_with_walls(g, flat, rng):
    eta, h, _ = _fields(g, rng, flat)
    gh, fl = W.bathy_gradient(h, g)
    s, a, k = op.coefficients(eta, gh, fl)
    G = W.dense(lambda v: W.apply_G(eta, gh, v, g), g)
    A = W.dense(lambda v: W.apply_A(s, a, v, g), g)
    lam = scipy.linalg.eigh(0.5 * (G + G.T), 0.5 * (A + A.T), eigvals_only=True)
    assert lam.min() >= (1.0 / k) * (1 - 1e-9)
    assert lam.max() <= 1.0 + 1e-9


@pytest.mark.parametrize("g", WALL_GRIDS, ids=IDS)
def test_pcg_with_walls_reaches_the_tolerance(g, rng):
    eta, h, _ = _fields(g, rng)
    gh, fl = W.bathy_gradient(h, g)
    b = rng.normal(size=(g.d,) + g.shape)
    u, it, ok, _ = W.pcg_solve(eta, gh, fl, b, g, tol=1e-12)
    assert ok
    assert np.linalg.norm(b - W.apply_G(eta, gh, u, g)) <= 1e-12 * np.linalg.norm(b)


def _state(g, rng):
    eta, h, _ = _fields(g, rng)
    u = 0.2 * np.stack([W.from_modes(W.to_modes(c, k), k) for c, k in
                        zip(rng.normal(size=(g.d,) + g.shape), W.VECTOR[g.d])])
    return eta, h, u


@pytest.mark.parametrize("g", WALL_GRIDS, ids=IDS)
def test_wall_rhs_equals_periodic_rhs_on_the_reflected_domain(g, rng):
    from oracle import rhs as R
    eta, h, u = _state(g, rng)
    g2 = periodic_twin(g)
    sc, vk = W.SCALAR[g.d], W.VECTOR[g.d]
    E = lambda f: reflect(f, sc)  # noqa: E731
    Ev = lambda v: np.stack([reflect(v[c], vk[c]) for c in range(g.d)])  # noqa: E731
    gh, _ = W.bathy_gradient(h, g)
    et, Ut = W.rhs(eta, u, h, gh, g)
    gh2, _ = op.bathy_gradient(E(h), g2)
    et2, Ut2 = R.rhs(E(eta), Ev(u), E(h), gh2, g2)
    assert np.max(np.abs(restrict(et2, g) - et)) < 1e-10 * np.max(np.abs(et))
    assert np.max(np.abs(restrict(Ut2, g) - Ut)) < 1e-10 * np.max(np.abs(Ut))
    assert abs(np.sum(et)) < 1e-12 * np.sum(np.abs(et))      # mass rate zero


@pytest.mark.parametrize("scheme", ["rk4", "ab2", "sbdf2"])
def test_wall_steppers_equal_periodic_steppers_on_the_reflected_domain(scheme, rng):
    from oracle import stepping as ST
    g = I.grid1d_walls(64, 20.0)
    eta, h, u = _state(g, rng)
    g2 = periodic_twin(g)
    pw = W.Problem.from_h(g, h, tol=1e-13)
    pp = ST.Problem.from_h(g2, reflect(h, "c"), tol=1e-13)
    U = pw.G(eta, u)
    U2 = pp.G(reflect(eta, "c"), np.stack([reflect(u[0], "s")]))
    args_w = (eta, U, u)
    args_p = (reflect(eta, "c"), U2, np.stack([reflect(u[0], "s")]))
    if scheme == "rk4":
        rw, rp = ST.run_rk4(pw, *args_w, 0.05, 3), ST.run_rk4(pp, *args_p, 0.05, 3)
    elif scheme == "ab2":
        rw, rp = ST.run_ab(pw, 2, *args_w, 0.05, 3), ST.run_ab(pp, 2, *args_p, 0.05, 3)
    else:
        rw, rp = ST.run_sbdf2(pw, *args_w, 0.05, 3), ST.run_sbdf2(pp, *args_p, 0.05, 3)
    for a, b in zip(rw, rp):
        assert np.max(np.abs(restrict(b, g) - a)) < 1e-9 * max(1.0, np.max(np.abs(a)))
