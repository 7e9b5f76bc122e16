"""GPU tests of the request server (sgn_server_*): each result is the same
alone and in a mix of concurrent requests (batched 1D solves, 2D and large 1D
solves and RK4 steps on the worker lanes), results match the oracle, and
admission by HBM footprint (a budget that admits one request at a time still
completes every request; oversized and invalid requests are rejected)."""
import math

import numpy as np
import pytest

from oracle import diagnostics as dg
from oracle import krylov
from oracle import operators as op
from oracle import stepping as ost
from paper_2506_16045_amd import inputs as I

pytestmark = pytest.mark.gpu


def _solve_case(g, eta, h, u_star):
    gh, _ = op.bathy_gradient(h, g)
    return dict(kind="solve", g=g, eta=eta, gh=gh, rhs=op.apply_G(eta, gh, u_star, g))


def _step_case(g, h, eta, u, dt, nsteps):
    return dict(kind="step", g=g, h=h, eta=eta, u=u, dt=dt, nsteps=nsteps)


def _cases():
    rng = np.random.default_rng(I.SEED_BASE + 50)
    cases = [_solve_case(*I.config_c4_item(rng, sizes=(512, 1024, 2048))) for _ in range(5)]
    # a 1D solve too long for the batched kernel, a 2D solve, 2D and 1D steps
    g, eta, h, b = I.pcg_test_problem_1d(16384, 1.0, 1.0)
    gh, _ = op.bathy_gradient(h, g)
    cases.append(dict(kind="solve", g=g, eta=eta, gh=gh, rhs=b))
    g, eta, h, b = I.elliptical_bump_2d(64, 1.0, 1.0)
    gh, _ = op.bathy_gradient(h, g)
    cases.append(dict(kind="solve", g=g, eta=eta, gh=gh, rhs=b))
    g = I.grid2d(64, 64, 50.0, 50.0)
    h = I.gaussian_bump2d(g, 1.0, 0.5, 5.0)
    eta_s, _ = I.solitary_wave(g, 1.0, 0.2, 17.0)
    zeta = eta_s - 1.0
    cases.append(_step_case(g, h, h + zeta, np.stack([math.sqrt(1.2) * zeta / (h + zeta), 0 * zeta]), 0.05, 3))
    g = I.grid1d(256, 80.0)
    eta, u = I.solitary_wave(g, 1.0, 0.2, 20.0)
    cases.append(_step_case(g, np.full(g.shape, 1.0), eta, u, 0.05, 4))
    return cases


def _req(srv, c, opts):
    if c["kind"] == "solve":
        return srv.solve_request(c["g"], c["eta"], c["gh"], c["rhs"], opts=opts)
    return srv.step_request(c["g"], c["h"], c["eta"], c["u"], c["dt"], c["nsteps"], opts=opts)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_results_same_alone_and_in_the_mix(precision):
    from paper_2506_16045_amd import sgn
    prec = sgn.FP64 if precision == "fp64" else sgn.MIXED
    opts = sgn.solve_opts(tol=1e-10, precision=prec, inner_tol=1e-4, max_iter=3000)
    cases = _cases()
    srv = sgn.Server(0, lanes=3)
    alone = []
    for c in cases:
        res, out = srv.wait(srv.submit(_req(srv, c, opts)))
        assert res.done and res.status == sgn.OK, (c["kind"], res.status)
        alone.append(out)
    # the same requests submitted together, twice over, with the order shuffled
    order = list(range(len(cases))) * 2
    np.random.default_rng(5).shuffle(order)
    ids = [(i, srv.submit(_req(srv, cases[i], opts))) for i in order]
    batch_sizes = []
    for i, rid in ids:
        res, out = srv.wait(rid)
        assert res.done and res.status == sgn.OK
        for k in out:
            assert np.array_equal(out[k], alone[i][k]), (i, k)
        if res.batched:
            batch_sizes.append(res.batch_size)
    assert batch_sizes and max(batch_sizes) > 1        # small solves shared launches
    st = srv.stats()
    assert st["bytes_in_use"] == 0 and st["queued"] == 0 and st["admitted"] == st["completed"]
    srv.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_results_match_the_oracle(precision):
    """Every served result against the FP64 oracle, the error stated per result:
    solves by relative L2 distance to the oracle's PCG solution and by true
    residual, RK4 runs per field (zeta, u, U); 1e-10 for the FP64 path, 1e-9 for
    the mixed one (FP32 inner solves inside FP64 refinement)."""
    from paper_2506_16045_amd import sgn
    cases = _cases()
    tol = 1e-11
    prec = sgn.FP64 if precision == "fp64" else sgn.MIXED
    gate = 1e-10 if precision == "fp64" else 1e-9
    opts = sgn.solve_opts(tol=tol, max_iter=3000, precision=prec, inner_tol=1e-4)
    srv = sgn.Server(0)
    ids = [srv.submit(_req(srv, c, opts)) for c in cases]
    for i, (c, rid) in enumerate(zip(cases, ids)):
        res, out = srv.wait(rid)
        assert res.status == sgn.OK
        g = c["g"]
        if c["kind"] == "solve":
            gh, eta, b, u = c["gh"], c["eta"], c["rhs"], out["u"]
            fl = not np.any(gh)
            s, a, _ = op.coefficients(eta, gh, fl)
            u_ref, it, ok, _ = krylov.pcg(lambda v: op.apply_G(eta, gh, v, g), lambda r: op.solve_A(s, a, r, g), b,
                                          tol=tol, max_iter=3000)
            bn = np.linalg.norm(b)
            r = np.linalg.norm(b - op.apply_G(eta, gh, u, g))
            r_ref = np.linalg.norm(b - op.apply_G(eta, gh, u_ref, g))
            err = dg.rel_l2(u, u_ref)
            print(f"  result {i}: solve {g.d}D n={g.nx} {precision} error vs oracle {err:.2e} "
                  f"relres {r / bn:.2e}", flush=True)
            assert r <= 2.0 * max(r_ref, tol * bn)
            assert err <= gate, err
            if precision == "fp64":
                assert abs(res.iters - it) <= 1
        else:
            pb = ost.Problem.from_h(g, c["h"], tol=tol)
            U0 = pb.G(c["eta"], c["u"])
            e_r, U_r, u_r = ost.run_rk4(pb, c["eta"], U0, c["u"], c["dt"], c["nsteps"])
            err = dg.field_errors(out["eta"], pb.G(out["eta"], out["u"]), out["u"], e_r, U_r, u_r, c["h"])
            print(f"  result {i}: {c['nsteps']} RK4 steps {g.d}D n={g.nx} {precision} error vs oracle "
                  f"{max(err.values()):.2e}", flush=True)
            assert max(err.values()) <= gate, err
            assert res.solves == 4 * c["nsteps"]
    srv.close()


def test_admission_by_footprint():
    from paper_2506_16045_amd import sgn
    cases = _cases()
    opts = sgn.solve_opts(tol=1e-10, max_iter=3000)
    probe = sgn.Server(0)
    fps = [sgn.Server.footprint(_req(probe, c, opts)) for c in cases]
    probe.close()
    assert all(f > 0 for f in fps)
    budget = int(1.2 * max(fps))
    srv = sgn.Server(0, hbm_budget=budget, lanes=2)
    ids = [srv.submit(_req(srv, c, opts)) for c in cases]
    spans = []
    for rid, fp in zip(ids, fps):
        res, out = srv.wait(rid)
        assert res.status == sgn.OK and res.t_submit <= res.t_admit <= res.t_start <= res.t_done
        spans.append((res.t_admit, res.t_done, fp, res.t_submit))
    # at no time did the admitted requests' footprints exceed the budget
    for t0, _, _, _ in spans:
        live = sum(fp for a, d, fp, _ in spans if a <= t0 < d)
        assert live <= budget, (live, budget)
    # the budget held requests back: at least one waited for admission
    assert any(a > s for a, _, _, s in spans)
    st = srv.stats()
    assert st["budget"] == budget and st["bytes_in_use"] == 0 and st["completed"] == len(cases)
    assert 0 < st["bytes_held"] <= budget
    # a request larger than the whole budget is refused at submission
    big = dict(cases[6])
    g = I.grid2d(1024, 1024, 200.0, 200.0)
    big.update(g=g, eta=np.ones(g.shape), gh=np.zeros((2,) + g.shape), rhs=np.zeros((2,) + g.shape))
    with pytest.raises(sgn.SgnError) as e:
        srv.submit(_req(srv, big, opts))
    assert e.value.status == sgn.ENOMEM
    # an invalid grid is refused
    bad = dict(cases[0])
    bad["g"] = I.grid1d(3, 10.0)
    bad.update(eta=np.ones(3), gh=np.zeros((1, 3)), rhs=np.zeros((1, 3)))
    with pytest.raises(sgn.SgnError) as e:
        srv.submit(_req(srv, bad, opts))
    assert e.value.status == sgn.EINVAL
    srv.close()


def test_failed_request_does_not_disturb_others():
    from paper_2506_16045_amd import sgn
    cases = _cases()
    opts = sgn.solve_opts(tol=1e-10, max_iter=3000)
    srv = sgn.Server(0)
    ref = [srv.wait(srv.submit(_req(srv, c, opts)))[1] for c in cases[:3]]
    dry = dict(cases[1])
    eta = dry["eta"].copy()
    eta[3] = -0.5
    dry["eta"] = eta
    ids = [srv.submit(_req(srv, c, opts)) for c in (cases[0], dry, cases[2])]
    out = [srv.wait(rid) for rid in ids]
    assert out[1][0].status == sgn.EDOMAIN
    assert out[0][0].status == sgn.OK and out[2][0].status == sgn.OK
    assert np.array_equal(out[0][1]["u"], ref[0]["u"]) and np.array_equal(out[2][1]["u"], ref[2]["u"])
    srv.close()
