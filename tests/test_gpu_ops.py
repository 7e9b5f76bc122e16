"""GPU parity of the operator entry points against the CPU oracle, element by
element on the same seeded inputs: bathymetry gradient, coefficients,
G_{eta,h} u (Def:G), A^{-1} (section 6.1) and the right-hand side f(w, p).
Sizes span several row/column tiles, tiny and maximum sizes, and both
dimensions."""
import numpy as np
import pytest

from oracle import operators as op
from oracle import rhs as orhs
from paper_2506_16045_amd import inputs as I

pytestmark = pytest.mark.gpu

# elementwise FP64 operators: rounding-level agreement
TOL_OP = 1e-12

GRIDS = [
    I.grid1d(2, 1.0), I.grid1d(8, 3.0), I.grid1d(256, 80.0), I.grid1d(4096, 400.0), I.grid1d(16384, 400.0),
    I.grid2d(2, 2, 1.0, 1.0), I.grid2d(8, 4, 2.0, 1.0), I.grid2d(64, 32, 5.0, 3.0), I.grid2d(32, 512, 1.0, 4.0),
    I.grid2d(512, 8, 4.0, 1.0), I.grid2d(256, 256, 20.0, 20.0), I.grid2d(1024, 1024, 200.0, 200.0),
    # rows of 1024 points (the wave-private row pass): fewer rows than the XCD remap groups, and a multiple of eight
    I.grid2d(1024, 4, 50.0, 1.0), I.grid2d(1024, 32, 100.0, 4.0),
]
IDS = [f"{g.d}d-{g.nx}x{g.ny if g.d == 2 else 1}" for g in GRIDS]


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2506_16045_amd import sgn
    assert torch.cuda.is_available()
    return sgn.Context(0)


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _n(t):
    return t.detach().cpu().numpy()


def _fields(g, seed, flat=False):
    rng = np.random.default_rng(seed)
    eta = I.random_positive_depth(g, rng, 0.6, 1.6)
    if flat:
        h = np.full(g.shape, 0.9)
    else:
        h = 1.0 + 0.2 * I.random_smooth_field(g, rng, modes=min(4, max(1, g.nx // 4)))
    u = np.stack([I.random_smooth_field(g, rng, modes=min(6, max(1, g.nx // 4))) for _ in range(g.d)])
    # add grid-scale content so every mode is exercised
    u = u + 0.05 * rng.normal(size=u.shape)
    return eta, h, u


def rel(a, b):
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


@pytest.mark.parametrize("g", GRIDS, ids=IDS)
def test_bathy_gradient(ctx, g):
    eta, h, u = _fields(g, 1)
    gh_ref, fl_ref = op.bathy_gradient(h, g)
    gh, fl = ctx.bathy_prepare(g, _t(h))
    assert fl == fl_ref
    assert rel(_n(gh), gh_ref) <= TOL_OP
    gh0, fl0 = ctx.bathy_prepare(g, _t(np.full(g.shape, 0.75)))
    assert fl0 and not np.any(_n(gh0))


@pytest.mark.parametrize("g", GRIDS, ids=IDS)
@pytest.mark.parametrize("flat", [False, True])
def test_coefficients(ctx, g, flat):
    eta, h, u = _fields(g, 2, flat)
    gh, fl = op.bathy_gradient(h, g)
    for kind in (0, 1):
        c = ctx.precond_coeffs(g, _t(eta), _t(gh), fl, kind)
        ref = op.coefficients(eta, gh, fl, kind=("optimal", "replacement")[kind])
        assert c.flat == int(fl)
        np.testing.assert_allclose([c.sigma, c.alpha, c.kappa_ub], ref, rtol=1e-14)


def test_coefficients_reject_nonpositive_depth(ctx):
    from paper_2506_16045_amd import sgn
    g = I.grid1d(64, 1.0)
    eta = np.ones(64)
    eta[17] = 0.0
    with pytest.raises(sgn.SgnError) as ei:
        ctx.precond_coeffs(g, _t(eta), _t(np.zeros((1, 64))), True)
    assert ei.value.status == sgn.EDOMAIN
    eta[17] = np.nan
    with pytest.raises(sgn.SgnError):
        ctx.precond_coeffs(g, _t(eta), _t(np.zeros((1, 64))), True)


@pytest.mark.parametrize("g", GRIDS, ids=IDS)
def test_apply_constraint(ctx, g):
    eta, h, u = _fields(g, 3)
    gh, fl = op.bathy_gradient(h, g)
    ref = op.apply_G(eta, gh, u, g)
    out = ctx.apply_constraint(g, _t(eta), _t(gh), _t(u))
    assert rel(_n(out), ref) <= TOL_OP


@pytest.mark.parametrize("g", GRIDS, ids=IDS)
def test_precond_solve(ctx, g):
    rng = np.random.default_rng(4)
    r = rng.normal(size=(g.d,) + g.shape)
    for sig, alp in ((1.3, 0.7), (2.0, 40.0)):
        ref = op.solve_A(sig, alp, r, g)
        out = ctx.precond_solve(g, sig, alp, _t(r))
        assert rel(_n(out), ref) <= TOL_OP


@pytest.mark.parametrize("g", GRIDS, ids=IDS)
def test_rhs(ctx, g):
    eta, h, u = _fields(g, 5)
    u = 0.3 * u
    gh, fl = op.bathy_gradient(h, g)
    et_ref, Ut_ref = orhs.rhs(eta, u, h, gh, g)
    et, Ut = ctx.rhs(g, _t(eta), _t(h), _t(gh), _t(u))
    assert rel(_n(et), et_ref) <= 1e-11
    assert rel(_n(Ut), Ut_ref) <= 1e-11


def test_invalid_arguments(ctx):
    import torch
    from paper_2506_16045_amd import sgn
    g = I.grid1d(48, 1.0)           # not a power of two
    x = torch.zeros(48, dtype=torch.float64, device="cuda")
    with pytest.raises(sgn.SgnError) as ei:
        ctx.apply_constraint(g, x, x.view(1, 48), x.view(1, 48).clone())
    assert ei.value.status == sgn.EUNSUPPORTED
    g = I.grid1d(64, 1.0)
    with pytest.raises(TypeError):
        ctx.apply_constraint(g, torch.zeros(64, device="cuda"), torch.zeros(1, 64, dtype=torch.float64, device="cuda"),
                             torch.zeros(1, 64, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        ctx.apply_constraint(g, torch.zeros(64, dtype=torch.float64), torch.zeros(1, 64, dtype=torch.float64),
                             torch.zeros(1, 64, dtype=torch.float64))
