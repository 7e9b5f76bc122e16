"""Seeded synthetic inputs for the SGN constraint solve and time stepping.

This module only builds input fields (depths, bathymetries, velocities and
right-hand sides) from closed-form recipes and seeded random draws.  It holds
none of the method's arithmetic (no derivative, no operator, no solver) and
imports neither the CPU oracle nor the HIP library, so both sides can take
their inputs from it.

Layout convention shared by every field returned here:
  * 1D scalar fields have shape (n,), the grid is x_j = j L / n (section 6.1).
  * 2D scalar fields have shape (ny, nx), x is the fast axis, x_i = i Lx / nx,
    y_j = j Ly / ny (section 6.1, doubly periodic).
  * vector fields are component-major: shape (d, n) or (d, ny, nx).

Recipes that the paper states are cited by section/equation; recipes that the
paper leaves open are marked "reading" and listed in the design notes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_BASE = 2506_16045


@dataclass(frozen=True)
class Grid:
    """Equispaced periodic grid (section 6.1).  d = 1 uses nx, Lx only."""

    d: int
    nx: int
    ny: int = 1
    Lx: float = 1.0
    Ly: float = 1.0
    bc: int = 0   # 0: periodic; 1: walls (homogeneous Neumann, cell-centred grid)

    @property
    def shape(self):
        return (self.nx,) if self.d == 1 else (self.ny, self.nx)

    @property
    def npts(self) -> int:
        return self.nx * (self.ny if self.d == 2 else 1)

    @property
    def cell(self) -> float:
        """Area element dx (1D) or dx*dy (2D)."""
        if self.d == 1:
            return self.Lx / self.nx
        return (self.Lx / self.nx) * (self.Ly / self.ny)


def grid1d(n: int, L: float) -> Grid:
    return Grid(1, n, 1, float(L), 1.0)


def grid2d(nx: int, ny: int, Lx: float, Ly: float) -> Grid:
    return Grid(2, nx, ny, float(Lx), float(Ly))


def grid1d_walls(n: int, L: float) -> Grid:
    """[0, L] between walls, cell-centred points x_j = (j + 1/2) L / n."""
    return Grid(1, n, 1, float(L), 1.0, 1)


def grid2d_walls(nx: int, ny: int, Lx: float, Ly: float) -> Grid:
    """[0, Lx] x [0, Ly] closed by walls, cell-centred points."""
    return Grid(2, nx, ny, float(Lx), float(Ly), 1)


def coords(g: Grid):
    """Grid coordinates; 1D returns x, 2D returns (X, Y) of shape (ny, nx).  A grid
    between walls has its points at the cell centres."""
    off = 0.5 if g.bc == 1 else 0.0
    x = (np.arange(g.nx, dtype=np.float64) + off) * (g.Lx / g.nx)
    if g.d == 1:
        return x
    y = (np.arange(g.ny, dtype=np.float64) + off) * (g.Ly / g.ny)
    X, Y = np.meshgrid(x, y, indexing="xy")
    return X, Y


def periodic_offset(x, x0: float, L: float):
    """Signed distance x - x0 wrapped to [-L/2, L/2) (nearest periodic image)."""
    return np.mod(x - x0 + 0.5 * L, L) - 0.5 * L


# ---------------------------------------------------------------------------
# Exact solitary wave over a flat bottom (section 6, ExSleta / ExSlu)
# ---------------------------------------------------------------------------

def solitary_speed_width(h0: float, a: float):
    """Speed c = sqrt(h0 + a) and width gamma = sqrt(3a) / (2 h0 c) (section 6)."""
    c = math.sqrt(h0 + a)
    gamma = math.sqrt(3.0 * a) / (2.0 * h0 * c)
    return c, gamma


def solitary_wave(g: Grid, h0: float, a: float, x0: float, t: float = 0.0,
                  theta: float = 0.0):
    """Total depth eta_s and velocity u_s of the SGN solitary wave.

    eta_s = h0 + a sech^2(gamma xi), u_s = w (cos theta, sin theta),
    w = c (eta_s - h0) / eta_s, xi = x cos theta + y sin theta - c t - x0
    (the crest sits at x0 + c t for theta = 0).  The periodic domain uses the
    nearest periodic image of xi along x (reading: the paper takes the domain
    large enough for the sech^2 tail to reach machine precision).
    Returns (eta, u) with u component-major, shape (d, ...).
    """
    c, gamma = solitary_speed_width(h0, a)
    if g.d == 1:
        x = coords(g)
        xi = periodic_offset(x - c * t, x0, g.Lx)
        eta = h0 + a / np.cosh(gamma * xi) ** 2
        w = c * (eta - h0) / eta
        return eta, w[None, :].copy()
    X, Y = coords(g)
    if theta != 0.0:
        raise ValueError("only theta = 0 line waves are generated on periodic 2D grids")
    xi = periodic_offset(X - c * t, x0, g.Lx)
    eta = h0 + a / np.cosh(gamma * xi) ** 2
    w = c * (eta - h0) / eta
    u = np.stack([w, np.zeros_like(w)])
    return eta, u


# ---------------------------------------------------------------------------
# Bathymetries (still-water depth h)
# ---------------------------------------------------------------------------

def flat(g: Grid, h0: float = 1.0):
    return np.full(g.shape, float(h0))


def tanh_shelf(g: Grid, h_deep: float = 1.0, drop: float = 0.5, x_up: float = 200.0,
               x_down: float = 350.0, width: float = 10.0):
    """Depth 1 -> 0.5 shelf built from tanh steps, closed periodically.

    The workload states a single step 0.25 (1 + tanh((x - 200)/10)); a single step
    is not periodic, so (reading) the shelf returns to the deep level through a
    second step at x_down and both steps are summed over the neighbouring
    periodic images:  h = h_deep - (drop/2) sum_k [tanh((x+kL-x_up)/w) - tanh((x+kL-x_down)/w)].
    """
    x = coords(g)
    L = g.Lx
    s = np.zeros_like(x)
    for k in (-1, 0, 1):
        s += np.tanh((x + k * L - x_up) / width) - np.tanh((x + k * L - x_down) / width)
    return h_deep - 0.5 * drop * s


def gaussian_bump2d(g: Grid, h0: float = 1.0, height: float = 0.5, radius: float = 10.0,
                    centre=None):
    """h = h0 - height exp(-r^2 / radius^2), r measured to the nearest periodic image."""
    X, Y = coords(g)
    cx, cy = centre if centre is not None else (0.5 * g.Lx, 0.5 * g.Ly)
    dx = periodic_offset(X, cx, g.Lx)
    dy = periodic_offset(Y, cy, g.Ly)
    return h0 - height * np.exp(-(dx * dx + dy * dy) / radius ** 2)


def random_bumps1d(g: Grid, rng, h0: float = 1.0, min_depth: float = 0.2):
    """h0 minus a sum of 1-3 Gaussian bumps, height U[0,0.5], width U[5,20].

    Centres are uniform on [0, L) with periodic distance; redrawn while
    min h < min_depth so the depth stays positive (section 3.1 assumption
    eta >= eta_min > 0).
    """
    x = coords(g)
    while True:
        m = int(rng.integers(1, 4))
        h = np.full_like(x, h0)
        for _ in range(m):
            A = rng.uniform(0.0, 0.5)
            w = rng.uniform(5.0, 20.0)
            c = rng.uniform(0.0, g.Lx)
            d = periodic_offset(x, c, g.Lx)
            h -= A * np.exp(-(d / w) ** 2)
        if h.min() >= min_depth:
            return h


def random_bumps2d(g: Grid, rng, h0: float = 1.0, min_depth: float = 0.2):
    """2D analogue: 1-3 Gaussian bumps, height U[0,0.5], radius U[5,20]."""
    X, Y = coords(g)
    while True:
        m = int(rng.integers(1, 4))
        h = np.full(g.shape, h0)
        for _ in range(m):
            A = rng.uniform(0.0, 0.5)
            w = rng.uniform(5.0, 20.0)
            cx, cy = rng.uniform(0.0, g.Lx), rng.uniform(0.0, g.Ly)
            dx = periodic_offset(X, cx, g.Lx)
            dy = periodic_offset(Y, cy, g.Ly)
            h -= A * np.exp(-(dx * dx + dy * dy) / w ** 2)
        if h.min() >= min_depth:
            return h


# ---------------------------------------------------------------------------
# Preconditioner test problems (section 6.2, 6.3)
# ---------------------------------------------------------------------------

def pcg_test_problem_1d(n: int, eta0: float, h0: float, sigma: float = 1.0 / 20.0):
    """Test problem of section 6.2 on [0, 1]: b = cos(4 pi x),
    h = 1 + h0 exp(-(x - 1/2)^2 / sigma^2), eta = 1 + eta0 cos(4 pi x)^2."""
    g = grid1d(n, 1.0)
    x = coords(g)
    h = 1.0 + h0 * np.exp(-((x - 0.5) ** 2) / sigma ** 2)
    eta = 1.0 + eta0 * np.cos(4.0 * np.pi * x) ** 2
    b = np.cos(4.0 * np.pi * x)[None, :].copy()
    return g, eta, h, b


def square_wave_depth_1d(n: int, eta0: float, hx):
    """Square-wave depth of section 6.2: 0.1 where |h_x|^2 <= 0.2, 0.1 eta0 elsewhere.
    hx is the bathymetry slope on the grid (computed by the caller)."""
    mask = np.asarray(hx) ** 2 <= 0.2
    return np.where(mask, 0.1, 0.1 * eta0)


def elliptical_bump_2d(n: int, a: float, b: float, r0: float = 0.5):
    """Elliptical bump of section 6.3 on the unit square.

    h = 1 - cos^2(pi r / (2 r0)) / 2 for r <= r0, else 1, r = sqrt(a^2 x^2 + b^2 y^2);
    (reading) the bump is centred at (1/2, 1/2) with periodic offsets.
    eta = h + exp(cos 2 pi x) + sin(4 pi y) / 4, rhs U = (cos 4 pi x, cos 4 pi y).
    """
    g = grid2d(n, n, 1.0, 1.0)
    X, Y = coords(g)
    dx = periodic_offset(X, 0.5, 1.0)
    dy = periodic_offset(Y, 0.5, 1.0)
    r = np.sqrt(a * a * dx * dx + b * b * dy * dy)
    h = np.where(r <= r0, 1.0 - 0.5 * np.cos(np.pi * r / (2.0 * r0)) ** 2, 1.0)
    eta = h + np.exp(np.cos(2.0 * np.pi * X)) + 0.25 * np.sin(4.0 * np.pi * Y)
    rhs = np.stack([np.cos(4.0 * np.pi * X), np.cos(4.0 * np.pi * Y)])
    return g, eta, h, rhs


def config_walls(n: int = 512, L: float = 200.0):
    """A closed basin for the wall solve (reading: the paper runs no test with walls):
    [0, L]^2 with walls, n x n cells, bathymetry of the 2D workload (h0 = 1, Gaussian
    bump of height 0.5 and radius 10 at the centre), a Gaussian hump of height 0.2
    and radius 15 at (L/4, L/2) on the surface, and the right-hand side U = b of
    a velocity field that vanishes on the walls: u = 0.3 sin(pi x / L) cos(pi y / L)
    * (1 + 0.2 sin(3 pi x / L)), v = 0.3 cos(pi x / L) sin(2 pi y / L), given as the
    constraint's input b = eta u (the momentum without the dispersive terms)."""
    g = grid2d_walls(n, n, L, L)
    X, Y = coords(g)
    h = 1.0 - 0.5 * np.exp(-((X - L / 2) ** 2 + (Y - L / 2) ** 2) / 10.0 ** 2)
    zeta = 0.2 * np.exp(-((X - L / 4) ** 2 + (Y - L / 2) ** 2) / 15.0 ** 2)
    eta = h + zeta
    u = 0.3 * np.sin(np.pi * X / L) * np.cos(np.pi * Y / L) * (1.0 + 0.2 * np.sin(3 * np.pi * X / L))
    v = 0.3 * np.cos(np.pi * X / L) * np.sin(2 * np.pi * Y / L)
    b = np.stack([eta * u, eta * v])
    return {"grid": g, "h": h, "eta": eta, "b": b, "tol": 1e-10}


def random_smooth_field(g: Grid, rng, modes: int = 4, amp: float = 1.0):
    """A random band-limited periodic field (a few low Fourier modes)."""
    if g.d == 1:
        x = coords(g)
        f = np.zeros_like(x)
        for m in range(1, modes + 1):
            f += amp * (rng.normal() * np.cos(2 * np.pi * m * x / g.Lx)
                        + rng.normal() * np.sin(2 * np.pi * m * x / g.Lx)) / m
        return f
    X, Y = coords(g)
    f = np.zeros(g.shape)
    for mx in range(0, modes + 1):
        for my in range(0, modes + 1):
            if mx == 0 and my == 0:
                continue
            ph = rng.uniform(0, 2 * np.pi)
            f += amp * rng.normal() * np.cos(2 * np.pi * (mx * X / g.Lx + my * Y / g.Ly) + ph) / (1 + mx + my)
    return f


def random_positive_depth(g: Grid, rng, lo: float = 0.5, hi: float = 2.0):
    """Smooth random depth with values inside [lo, hi]."""
    f = random_smooth_field(g, rng)
    f = (f - f.min()) / max(f.max() - f.min(), 1e-300)
    return lo + (hi - lo) * f


# ---------------------------------------------------------------------------
# Workload configurations (the benchmark and parity cases)
# ---------------------------------------------------------------------------

def config_c1():
    """1D flat-bottom solitary wave: N=256, L=80, h0=1, a=0.2 at x=20, RK4 dt=0.01 x 500, tol 1e-12."""
    g = grid1d(256, 80.0)
    h = flat(g, 1.0)
    eta, u = solitary_wave(g, 1.0, 0.2, 20.0)
    return dict(name="C1", grid=g, h=h, eta=eta, u=u, dt=0.01, steps=500, tol=1e-12,
                scheme="rk4", h0=1.0, a=0.2, x0=20.0)


def config_c2(n: int = 4096):
    """1D shelf: N=4096, L=400, shelf 1 -> 0.5, a=0.3 at x=100, dt=0.02 x 2000."""
    g = grid1d(n, 400.0)
    h = tanh_shelf(g)
    eta_s, u = solitary_wave(g, 1.0, 0.3, 100.0)
    # the wave sits on the deep part (h = 1 up to ~1e-9 there): eta = h + zeta
    zeta = eta_s - 1.0
    eta = h + zeta
    u = (math.sqrt(1.3) * zeta / eta)[None, :]
    return dict(name="C2", grid=g, h=h, eta=eta, u=u, dt=0.02, steps=2000, tol=1e-12,
                scheme="sbdf2", h0=1.0, a=0.3, x0=100.0)


def config_c3(n: int = 1024, L: float = 200.0):
    """2D circular bump: n x n on L x L, h0=1, bump 0.5 of radius 10 at the centre,
    line solitary wave a=0.2 in x with crest at x=50 (reading), RK4 dt=0.02 x 500, tol 1e-10."""
    g = grid2d(n, n, L, L)
    h = gaussian_bump2d(g, 1.0, 0.5, 10.0)
    eta_s, u_s = solitary_wave(g, 1.0, 0.2, 50.0)
    zeta = eta_s - 1.0
    eta = h + zeta
    c = math.sqrt(1.2)
    u = np.stack([c * zeta / eta, np.zeros_like(zeta)])
    return dict(name="C3", grid=g, h=h, eta=eta, u=u, dt=0.02, steps=500, tol=1e-10,
                scheme="rk4", h0=1.0, a=0.2, x0=50.0)


C4_SIZES = (512, 1024, 2048, 4096, 8192)


def config_c4_item(rng, L: float = 400.0, sizes=C4_SIZES):
    """One batched-ensemble item: random size, random bumps, random solitary wave.
    Returns (grid, eta, h, u_star); the right-hand side is b = G u_star, formed by
    whichever side (oracle or device) is being exercised."""
    n = int(rng.choice(np.asarray(sizes)))
    g = grid1d(n, L)
    h = random_bumps1d(g, rng)
    a = rng.uniform(0.05, 0.4)
    x0 = rng.uniform(0.0, L)
    hbar = 1.0
    c, gamma = solitary_speed_width(hbar, a)
    x = coords(g)
    zeta = a / np.cosh(gamma * periodic_offset(x, x0, L)) ** 2
    eta = h + zeta
    u = (c * zeta / eta)[None, :]
    return g, eta, h, u


def config_c4(count: int = 512, seed_offset: int = 4, sizes=C4_SIZES):
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    return [config_c4_item(rng, sizes=sizes) for _ in range(count)]


# ---------------------------------------------------------------------------
# Served request stream (reading: the sizes, mixes and step counts are
# proposals; the paper prescribes no request workload)
# ---------------------------------------------------------------------------
C5_SIZES_1D = (1024, 2048, 4096, 8192, 16384)
C5_SIZES_2D = (128, 256, 512, 1024)


def config_c5_request(rng, kind: str | None = None, dim: int | None = None, n: int | None = None):
    """One request of the served stream: 70% 1D (N in C5_SIZES_1D, L = 400, the
    batched-ensemble recipe), 30% 2D (n x n in C5_SIZES_2D on 200 x 200, 1-3
    random bumps, a line solitary wave in x); half "solve" (one constraint solve
    G u = G u* to 1e-10 from a zero guess), half "step" (10 RK4 steps from
    (eta, u), dt = min(0.02, dx / 2)).  Returns a dict with kind, grid, h, eta
    and u (u* for a solve, the initial velocity for a step), dt, nsteps, tol."""
    if dim is None:
        dim = 1 if rng.uniform() < 0.7 else 2
    if kind is None:
        kind = "solve" if rng.uniform() < 0.5 else "step"
    if dim == 1:
        sizes = (n,) if n else C5_SIZES_1D
        g, eta, h, u = config_c4_item(rng, sizes=sizes)
    else:
        nn = n if n else int(rng.choice(np.asarray(C5_SIZES_2D)))
        g = grid2d(nn, nn, 200.0, 200.0)
        h = random_bumps2d(g, rng)
        a = rng.uniform(0.05, 0.4)
        x0 = rng.uniform(0.0, 200.0)
        c, gamma = solitary_speed_width(1.0, a)
        X, _ = coords(g)
        zeta = a / np.cosh(gamma * periodic_offset(X, x0, 200.0)) ** 2
        eta = h + zeta
        u = np.stack([c * zeta / eta, np.zeros_like(zeta)])
    dx = g.Lx / g.nx
    return dict(kind=kind, grid=g, h=h, eta=eta, u=u, dt=min(0.02, 0.5 * dx), nsteps=10, tol=1e-10)
