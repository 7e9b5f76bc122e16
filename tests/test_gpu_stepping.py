"""GPU parity of the time steppers (section 5) against the oracle: RK4 (Eq:ERK),
AB2-4 (Eq:AB) and the linearly implicit SBDF2 scheme (Eq:MM), in 1D and 2D,
FP64 to 1e-10 relative L2 per field (zeta, u, U) and the mixed form to 1e-9,
with both initial-guess rules of the stepper solves (the most recent velocity,
or extrapolated per-slot offsets), the same rule on both sides.
Also: Krylov iteration counts per solve agree, mass is conserved on the device."""
import math

import numpy as np
import pytest

from oracle import diagnostics as dg
from oracle import stepping as ost
from paper_2506_16045_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2506_16045_amd import sgn
    return sgn.Context(0)


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _n(t):
    return t.detach().cpu().numpy()


def case_1d_flat():
    g = I.grid1d(256, 80.0)
    eta, u = I.solitary_wave(g, 1.0, 0.2, 20.0)
    return g, np.full(g.shape, 1.0), eta, u


def case_1d_shelf():
    c = I.config_c2(1024)
    return c["grid"], c["h"], c["eta"], c["u"]


def case_1d_bump():
    g = I.grid1d(512, 80.0)
    x = I.coords(g)
    h = 1.0 - 0.4 * np.exp(-((x - 45.0) / 6.0) ** 2)
    eta_s, u = I.solitary_wave(g, 1.0, 0.3, 35.0)
    eta = h + (eta_s - 1.0)
    return g, h, eta, u


def case_2d_bump():
    g = I.grid2d(64, 64, 50.0, 50.0)
    h = I.gaussian_bump2d(g, 1.0, 0.5, 5.0)
    eta_s, u_s = I.solitary_wave(g, 1.0, 0.2, 17.0)
    zeta = eta_s - 1.0
    eta = h + zeta
    u = np.stack([math.sqrt(1.2) * zeta / eta, np.zeros_like(zeta)])
    return g, h, eta, u


def _setup(ctx, g, h, eta, u, tol, guess="extrapolate"):
    from paper_2506_16045_amd import sgn
    gh, flat = ctx.bathy_prepare(g, _t(h))
    e_d, u_d = _t(eta), _t(u)
    U_d = ctx.apply_constraint(g, e_d, gh, u_d)
    st = sgn.State(ctx, g, _t(h), gh, flat, e_d, U_d, u_d)
    pb = ost.Problem.from_h(g, h, tol=tol, guess=guess)
    U0 = pb.G(eta, u)
    return st, pb, U0


def _compare(st, h, ref, tol_rel):
    e_r, U_r, u_r = ref
    err = dg.field_errors(_n(st.eta), _n(st.U), _n(st.u), e_r, U_r, u_r, h)
    assert max(err.values()) <= tol_rel, err
    return err


SCHEMES = [("rk4", 6), ("ab2", 8), ("ab3", 8), ("ab4", 8), ("sbdf2", 10)]
CASES = [("1d-flat", case_1d_flat, 0.05), ("1d-shelf", case_1d_shelf, 0.02), ("1d-bump", case_1d_bump, 0.05),
         ("2d-bump", case_2d_bump, 0.05)]


@pytest.mark.parametrize("guess", ["previous", "extrapolate"])
@pytest.mark.parametrize("cname,make,dt", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("scheme,nsteps", SCHEMES, ids=[s[0] for s in SCHEMES])
def test_stepper_fp64_matches_oracle(ctx, cname, make, dt, scheme, nsteps, guess):
    from paper_2506_16045_amd import sgn
    g, h, eta, u = make()
    tol = 1e-12
    st, pb, U0 = _setup(ctx, g, h, eta, u, tol, guess)
    opts = sgn.solve_opts(tol=tol, check_every=4, guess=guess)
    if scheme == "rk4":
        info = st.step_rk4(dt, nsteps, opts)
        ref = ost.run_rk4(pb, eta, U0, u, dt, nsteps)
    elif scheme.startswith("ab"):
        order = int(scheme[2])
        info = st.step_ab(order, dt, nsteps, opts)
        ref = ost.run_ab(pb, order, eta, U0, u, dt, nsteps)
    else:
        info = st.step_linimp(dt, nsteps, None, opts)
        ref = ost.run_sbdf2(pb, eta, U0, u, dt, nsteps)
    assert info.converged and info.steps_done == nsteps
    assert abs(info.t - nsteps * dt) < 1e-12
    assert info.solves == len(pb.iters)
    assert abs(info.iters - sum(pb.iters)) <= len(pb.iters)
    _compare(st, h, ref, 1e-10)
    # mass (Remark 2.1) is conserved by the device steps
    assert abs(dg.mass(_n(st.eta), h, g) - dg.mass(eta, h, g)) <= 1e-12 * max(1.0, abs(dg.mass(eta, h, g)))
    st.close()


@pytest.mark.parametrize("guess", ["previous", "extrapolate"])
@pytest.mark.parametrize("cname,make,dt", [CASES[2], CASES[3]], ids=["1d-bump", "2d-bump"])
def test_rk4_mixed_matches_fp64_oracle(ctx, cname, make, dt, guess):
    from paper_2506_16045_amd import sgn
    g, h, eta, u = make()
    st, pb, U0 = _setup(ctx, g, h, eta, u, 1e-13, guess)
    info = st.step_rk4(dt, 4, sgn.solve_opts(tol=1e-11, precision=sgn.MIXED, inner_tol=1e-4, guess=guess))
    ref = ost.run_rk4(pb, eta, U0, u, dt, 4)
    assert info.converged
    _compare(st, h, ref, 1e-9)


def test_sbdf2_fixed_coefficients_and_restart(ctx):
    """Caller-fixed (sigma, alpha) (section 6.5 keeps them over the run); a second
    call continues the same history."""
    from paper_2506_16045_amd import sgn
    g, h, eta, u = case_1d_bump()
    st, pb, U0 = _setup(ctx, g, h, eta, u, 1e-12)
    s, a, _ = ost.op.coefficients(eta, pb.grad_h, pb.flat)
    fixed = sgn.Coeffs(1.2 * s, 1.2 * a, 0.0, 0)
    st.step_linimp(0.05, 3, fixed)
    st.step_linimp(0.05, 4, fixed)
    ref = ost.run_sbdf2(pb, eta, U0, u, 0.05, 7, coeffs=(1.2 * s, 1.2 * a))
    _compare(st, h, ref, 1e-10)


def test_guess_history_persists_across_calls_and_resets_on_dt(ctx):
    """Calls with the same dt continue the offset history (2 + 4 RK4 steps equal
    6 oracle steps, iteration for iteration); a new dt clears it on both sides."""
    from paper_2506_16045_amd import sgn
    g, h, eta, u = case_2d_bump()
    st, pb, U0 = _setup(ctx, g, h, eta, u, 1e-12)
    opts = sgn.solve_opts(tol=1e-12, check_every=4)
    i1 = st.step_rk4(0.05, 2, opts)
    i2 = st.step_rk4(0.05, 4, opts)
    i3 = st.step_rk4(0.04, 3, opts)
    ref = ost.run_rk4(pb, eta, U0, u, 0.05, 6)
    ref = ost.run_rk4(pb, *ref, 0.04, 3)
    assert i1.solves + i2.solves + i3.solves == len(pb.iters) == 36
    assert abs(i1.iters + i2.iters + i3.iters - sum(pb.iters)) <= len(pb.iters)
    _compare(st, h, ref, 1e-10)
    st.close()


def test_bad_guess_rule_rejected(ctx):
    from paper_2506_16045_amd import sgn
    g, h, eta, u = case_1d_flat()
    st, pb, U0 = _setup(ctx, g, h, eta, u, 1e-12)
    opts = sgn.solve_opts(tol=1e-12)
    opts.guess = 7
    with pytest.raises(sgn.SgnError) as e:
        st.step_rk4(0.05, 1, opts)
    assert e.value.status == sgn.EINVAL
    st.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_size_2d_rk4_step_matches_oracle(ctx, precision):
    """The benchmarked 2D workload at its full size (1024 x 1024, tol 1e-10): one RK4
    step from the initial data on the device against the oracle's, per field
    (zeta, u, U) to 1e-10 relative L2 in FP64 and 1e-9 in the mixed form, in the
    launch configuration the bench times.  (The oracle step takes about 10 s on
    one core.)"""
    from paper_2506_16045_amd import sgn
    cfg = I.config_c3(1024)
    g, h, eta, u = cfg["grid"], cfg["h"], cfg["eta"], cfg["u"]
    st, pb, U0 = _setup(ctx, g, h, eta, u, cfg["tol"])
    prec = sgn.FP64 if precision == "fp64" else sgn.MIXED
    info = st.step_rk4(cfg["dt"], 1, sgn.solve_opts(tol=cfg["tol"], precision=prec, check_every=8))
    assert info.converged and info.solves == 4
    ref = ost.run_rk4(pb, eta, U0, u, cfg["dt"], 1)
    _compare(st, h, ref, 1e-10 if precision == "fp64" else 1e-9)
    st.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replayed_chunks_equal_eager_launches(precision, monkeypatch):
    """With SGN_GRAPHS=1 the PCG iteration chunks are captured as HIP graphs on
    their second use and replayed afterwards; over 8 RK4 steps (each solve
    configuration runs eagerly, is captured, then replayed several times, with
    the steppers' eager work and readbacks between replays) every field equals
    the eager run bit for bit."""
    import torch
    from paper_2506_16045_amd import sgn
    g, h, eta, u = case_2d_bump()
    prec = sgn.FP64 if precision == "fp64" else sgn.MIXED
    opts = sgn.solve_opts(tol=1e-11, precision=prec, inner_tol=1e-4, check_every=2)
    out = []
    for graphs in ("0", "1"):
        monkeypatch.setenv("SGN_GRAPHS", graphs)
        c = sgn.Context(0)
        gh, flat = c.bathy_prepare(g, _t(h))
        e_d, u_d = _t(eta), _t(u)
        U_d = c.apply_constraint(g, e_d, gh, u_d)
        st = sgn.State(c, g, _t(h), gh, flat, e_d, U_d, u_d)
        fields = []
        for _ in range(8):
            info = st.step_rk4(0.05, 1, opts)
            assert info.converged
            torch.cuda.synchronize()
            fields.append((_n(st.eta), _n(st.U), _n(st.u)))
        st.close()
        c.close()
        out.append(fields)
    for a, b in zip(out[0], out[1]):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


def test_sbdf2_new_fixed_coefficients_restart_the_history(ctx):
    """Eq:MM uses one A on both sides of a step: a continuing call with other fixed
    (sigma, alpha) starts a new history (an RK4 start-up step, then SBDF2 with the
    new A), equal to the oracle run in two parts."""
    from paper_2506_16045_amd import sgn
    g, h, eta, u = case_1d_bump()
    st, pb, U0 = _setup(ctx, g, h, eta, u, 1e-12)
    s, a, _ = ost.op.coefficients(eta, pb.grad_h, pb.flat)
    st.step_linimp(0.05, 3, sgn.Coeffs(1.2 * s, 1.2 * a, 0.0, 0))
    st.step_linimp(0.05, 4, sgn.Coeffs(1.5 * s, 1.1 * a, 0.0, 0))
    ref = ost.run_sbdf2(pb, eta, U0, u, 0.05, 3, coeffs=(1.2 * s, 1.2 * a))
    ref = ost.run_sbdf2(pb, *ref, 0.05, 4, coeffs=(1.5 * s, 1.1 * a))
    _compare(st, h, ref, 1e-10)
    st.close()


def test_failed_stage_solve_leaves_the_state(ctx):
    """A step whose stage solve stops at max_iter returns SGN_ENOCONV and leaves
    the state at the last completed step: t, steps_done and eta unchanged."""
    from paper_2506_16045_amd import sgn
    g, h, eta, u = case_2d_bump()
    st, pb, U0 = _setup(ctx, g, h, eta, u, 1e-12)
    opts = sgn.solve_opts(tol=1e-12, max_iter=2, guess="previous")
    with pytest.raises(sgn.SgnError) as e:
        st.step_rk4(0.05, 1, opts)
    assert e.value.status == sgn.ENOCONV
    info = st.step_rk4(0.05, 0, opts)
    assert info.steps_done == 0 and info.t == 0.0
    assert np.array_equal(_n(st.eta), eta)
    st.close()
