"""The allocation-free Krylov solve (sgn_krylov_solve_noalloc, for callers that
cannot allocate device memory): through the C ABI, two calls in a row, the
second on a smaller grid, each equal to sgn_krylov_solve with a caller workspace
(same kernels, so the same bits and iteration counts) on the 2D row/column path
(FP64 and mixed), the one-workgroup 1D path and GMRES; a grid whose workspace
exceeds the 48 MiB scratch is refused."""
import numpy as np
import pytest

from oracle import krylov
from oracle import operators as op
from paper_2506_16045_amd import inputs as I

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _n(t):
    return t.detach().cpu().numpy()


def _elliptic(n):
    g, eta, h, b = I.elliptical_bump_2d(n, 1.0, 20.0)
    gh, _ = op.bathy_gradient(h, g)
    return g, eta, gh, b


def _ensemble_item(seed, n):
    rng = np.random.default_rng(I.SEED_BASE + seed)
    g, eta, h, u_star = I.config_c4_item(rng, sizes=(n,))
    gh, _ = op.bathy_gradient(h, g)
    return g, eta, gh, op.apply_G(eta, gh, u_star, g)


PAIRS = [
    ("2d-fp64", lambda: _elliptic(256), lambda: _elliptic(128), "fp64", "pcg"),
    ("2d-mixed", lambda: _elliptic(512), lambda: _elliptic(256), "mixed", "pcg"),
    ("1d-fp64", lambda: _ensemble_item(71, 8192), lambda: _ensemble_item(72, 2048), "fp64", "pcg"),
    ("1d-mixed", lambda: _ensemble_item(73, 16384), lambda: _ensemble_item(74, 4096), "mixed", "pcg"),
    ("2d-gmres", lambda: _elliptic(128), lambda: _elliptic(64), "fp64", "gmres"),
]


@pytest.mark.parametrize("name,big,small,precision,method", PAIRS, ids=[p[0] for p in PAIRS])
def test_noalloc_solve_equals_workspace_solve(name, big, small, precision, method):
    from paper_2506_16045_amd import sgn
    print(f"noalloc {name}", flush=True)
    ctx = sgn.Context(0)
    prec = sgn.FP64 if precision == "fp64" else sgn.MIXED
    meth = sgn.PCG if method == "pcg" else sgn.GMRES
    opts = sgn.solve_opts(tol=1e-11, precision=prec, inner_tol=1e-4, max_iter=3000, method=meth,
                          gmres_restart=40, check_every=4)
    for make in (big, small):
        g, eta, gh, b = make()
        e_d, gh_d, b_d = _t(eta), _t(gh), _t(b)
        u_ref, r_ref = ctx.krylov_solve(g, e_d, gh_d, b_d, opts=opts)
        u_na, r_na = ctx.krylov_solve_noalloc(g, e_d, gh_d, b_d, opts=opts)
        assert r_na.converged and r_ref.converged
        assert r_na.iters == r_ref.iters and r_na.outer_iters == r_ref.outer_iters
        assert np.array_equal(_n(u_na), _n(u_ref)), name
        # and the solution solves the system (the oracle's operator)
        u = _n(u_na)
        res = np.linalg.norm(b - op.apply_G(eta, gh, u, g)) / np.linalg.norm(b)
        assert res <= 1e-9, res
    ctx.close()


def test_noalloc_matches_oracle_and_reuses_scratch():
    """Two different systems in a row through the shared scratch: the second
    result does not depend on what the first left there (equal to the oracle's
    PCG iterate to 1e-10)."""
    from paper_2506_16045_amd import sgn
    ctx = sgn.Context(0)
    opts = sgn.solve_opts(tol=1e-12, max_iter=3000, check_every=4)
    for make in (lambda: _elliptic(128), lambda: _elliptic(64)):
        g, eta, gh, b = make()
        u, r = ctx.krylov_solve_noalloc(g, _t(eta), _t(gh), _t(b), opts=opts)
        fl = not np.any(gh)
        s, a, _ = op.coefficients(eta, gh, fl)
        u_ref, it, ok, _ = krylov.pcg(lambda v: op.apply_G(eta, gh, v, g), lambda q: op.solve_A(s, a, q, g), b,
                                      tol=1e-12, max_iter=3000)
        # CG in floating point: over the ~300 iterations these problems take at tol
        # 1e-12 the count depends on the rounding order of the dot products (64 x 64:
        # 323 on the device, 321 in the oracle, solutions equal to 9e-14), so the
        # counts agree to 1 %
        assert ok and abs(r.iters - it) <= max(1, it // 100), (r.iters, it)
        err = np.linalg.norm(_n(u) - u_ref) / np.linalg.norm(u_ref)
        assert err <= 1e-10, err
    ctx.close()


def test_noalloc_refuses_a_grid_beyond_the_scratch():
    from paper_2506_16045_amd import sgn
    ctx = sgn.Context(0)
    g = I.grid2d(1024, 1024, 200.0, 200.0)
    eta = np.ones(g.shape)
    gh = np.zeros((2,) + g.shape)
    b = np.ones((2,) + g.shape)
    with pytest.raises(sgn.SgnError) as e:
        ctx.krylov_solve_noalloc(g, _t(eta), _t(gh), _t(b))
    assert e.value.status == sgn.EINVAL and "scratch" in str(e.value)
    ctx.close()
