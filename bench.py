#!/usr/bin/env python
"""Benchmark of the SGN hot path on one MI355X.

Workload (the 2D configuration the grid-point-steps metric is quoted on):
2D doubly periodic SGN over a Gaussian bump, 1024 x 1024 grid on 200 x 200,
still-water depth 1, bump height 0.5 and radius 10 at the centre, line
solitary wave a = 0.2 travelling in x (crest at x = 50), classical RK4 with
dt = 0.02, preconditioned Krylov (PCG with the constant-coefficient operator
A) to a relative residual of 1e-10 at every stage, stage solves started from
extrapolated guesses.  Default precision FP64 (the faster form on this
workload); the same run also times the mixed form (FP32
operator/FFT/preconditioner inside FP64 iterative refinement) and reports it
under other_precision (--precision mixed swaps the two).

One step = one RK4 step of the whole hot path (4 right-hand sides, 4 Krylov
solves, the stage combinations).  `value` = grid points x timed steps / wall
seconds, with every field already resident in HBM.  The line also carries
the roofline of the dominant kernel (HIP events around each of its launches
over the timed region) and the CPU oracle timed on the host on one RK4 step of
the same workload.

    python bench.py [--steps K] [--warmup W] [--precision mixed|fp64]

--workload batch measures the batched-ensemble workload instead: 512
independent 1D constraint solves G u = b with sizes drawn from
{512, ..., 8192} on L = 400, random Gaussian bumps and random solitary waves,
b = G u* formed on the device, all solved in one launch per step (a step is
one batched solve of the whole ensemble from a zero guess, to 1e-10).

--workload c1 runs the 1D flat-bottom solitary wave (N = 256 on L = 80, a = 0.2
at x = 20, RK4 dt = 0.01, PCG tol 1e-12) for its stated 500 steps (--steps
overrides), FP64; the oracle runs the same 500 steps on the host and both are
compared with each other and with the exact travelling wave.

--workload c2 runs the 1D shelf (N = 4096 on L = 400, a = 0.3 at x = 100,
dt = 0.02, tol 1e-12) for its stated 2000 steps per leg: the linearly implicit
SBDF2 (one constant-coefficient FFT solve per step), AB3+PCG and RK4+PCG, each
in FP64 and mixed precision; the oracle runs the first 200 steps of each leg,
against a device run of the same length.

--workload serve measures the request server: Poisson arrivals at each rate
of --rates (requests per second), --serve-requests requests per rate, 70% 1D
(N 1024..16384) and 30% 2D (128^2..1024^2) grids, half single constraint
solves and half 10-step RK4 runs, admitted by HBM footprint; the line reports
throughput and p50/p99 latency (submission to result on the host) per rate,
for the FP64 and the mixed-precision path.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0    # MI355X HBM3E, 8 TB/s


PROFILES = os.path.join(ROOT, "profiles")
# kernel code and the launch shapes chosen for it
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2506_16045_amd", "csrc", f)
                  for f in ("sgn_device.h", "sgn_kernels.h", "sgn_wave.h", "sgn_lib.hip")]


def kernel_bytes(kind: str, d: int, nx: int, ny: int, word: int) -> float:
    """Algorithmic HBM bytes of one launch of a PCG kernel family: every field
    the kernel must read once plus every field it must write once.
    NS = (nx/2+1) ny complex modes per spectral field (2 words), N = nx ny points."""
    ns = (nx // 2 + 1) * ny
    n = nx * ny
    cw = 2 * word
    base = kind.replace("_f32", "")
    if base == "pcg_c1":      # read r_hat, p_hat (2d fields); write p_hat (d) and d+1 transformed fields
        return (2 * d + d + (d + 1)) * ns * cw
    if base == "pcg_r1":      # read/write d+1 half-spectral fields; read eta and grad h (1 + d reals)
        return 2 * (d + 1) * ns * cw + (1 + d) * n * word
    if base == "pcg_c2":      # read d+1 half-spectral fields and p, x, r hats (3d); write x, r hats (2d)
        return ((d + 1) + 3 * d + 2 * d) * ns * cw
    if base == "pcg_init":    # read r hat (d)
        return d * ns * cw
    # 2D right-hand side (word = 8): the passes of one evaluation of f(w, p); in 2D
    # the diagonal momentum fluxes are folded into S_x = S - eta u_x^2 and
    # S_y = S - eta u_y^2 by the inverse pass, so one flux field is transformed
    ns_s = 2 if d == 2 else 1   # S spectra: S_x, S_y (2D) or S (1D)
    # periodic 2D rows of 1024 points: the inverse row pass forms d_x delta, d_x eta
    # and d_x beta from spectra it reads anyway, so the column pass writes 3 fewer
    dxr = 3 if (d == 2 and nx == 1024) else 0
    if base == "rhs_rows_fwd":  # read eta, u (d), grad h (d); write [u, eta u, eta, eta u_1 u_d, beta] spectra
        return (1 + 2 * d) * n * word + ((2 * d + 1) + 2) * ns * cw
    if base == "rhs_cols":      # read u, eta u, eta, beta spectra; write delta, grad delta, m, grad eta, grad beta
        return ((2 * d + 1) + 1) * ns * cw + ((2 * d + 2) + d - dxr) * ns * cw
    if base == "rhs_rows_inv":  # read those spectra (delta's once) and eta, u, grad h; write eta_t, U_t, S spectra
        return (3 * d + 2 - (1 if dxr else 0)) * ns * cw + (1 + 2 * d) * n * word + (1 + d) * n * word + ns_s * ns * cw
    if base == "rhs_flux":      # read the S spectra and the flux spectrum; write grad S - div(flux) (d)
        return (ns_s + 1) * ns * cw + d * ns * cw
    raise ValueError(kind)


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kind: str, n: int):
    """HBM bytes per launch from the committed counter runs, if they were taken on
    the current kernel sources (else None)."""
    path = os.path.join(PROFILES, "pcg_traffic_2d_1024.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha") != kernel_source_hash() or rec.get("n") != n:
        return None
    prec_key = "f32" if kind.endswith("_f32") else "f64"
    ent = rec.get("kernels", {}).get(prec_key, {}).get(kind.replace("_f32", ""))
    return ent.get("hbm_bytes_per_launch") if ent else None


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def cpu_baseline(cfg, steps: int = 1, device_fields=None, dealias: bool = False):
    """The oracle, as it stands, on `steps` RK4 steps of the same workload from its
    initial data.  device_fields = (eta, U, u) of the device after the same steps
    adds the relative L2 difference per field (zeta = eta - h, U, u)."""
    import numpy as np
    from oracle import stepping as ost
    pb = ost.Problem.from_h(cfg["grid"], cfg["h"], tol=cfg["tol"], dealias=2 if dealias else 1)
    U0 = pb.G(cfg["eta"], cfg["u"])
    t0 = time.perf_counter()
    e_r, U_r, u_r = ost.run_rk4(pb, cfg["eta"], U0, cfg["u"], cfg["dt"], steps)
    dt = time.perf_counter() - t0
    g = cfg["grid"]
    out = {"value": g.npts * steps / dt, "unit": "grid-pt-steps/s", "cores": 1, "kind": "oracle",
           "sample": f"{steps} RK4 step(s) of the {g.nx}x{g.ny} workload from its initial data "
                     f"({dt:.1f} s, FP64 NumPy, single thread; iterations/solve "
                     f"{np.mean(pb.iters):.1f})"}
    if device_fields is not None:
        e_d, U_d, u_d = device_fields
        rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
        out["device_vs_oracle_rel_l2"] = {"zeta": rel(e_d - cfg["h"], e_r - cfg["h"]), "U": rel(U_d, U_r),
                                          "u": rel(u_d, u_r), "steps": steps}
    return out


def batch_bytes(sizes, res, mixed: bool) -> float:
    """Algorithmic HBM bytes of one batched launch: per system, the inputs eta,
    h_x, b and the output u in FP64, 13 words per point for every PCG iteration
    (x, r, p read and written, q and z formed on chip, eta and h_x read; the
    transforms stay in LDS) in the working precision, and in mixed mode 7 FP64
    words per point for each refinement step's residual."""
    tot = 0.0
    w = 4 if mixed else 8
    for n, r in zip(sizes, res):
        tot += n * (4 * 8 + r.iters * 13 * w + (r.outer_iters * 7 * 8 if mixed else 0))
    return tot


COEFF_SWEEP = [(n, eta0) for n in (512, 16384) for eta0 in (1.0, 0.5, 0.2, 0.1, 0.05)]


def cpu_baseline_coeffs():
    """The oracle's PCG, as it stands, on every case of the coefficient sweep (both
    coefficient kinds); its iteration counts are reported beside the device's."""
    from oracle import krylov
    from oracle import operators as op
    from paper_2506_16045_amd import inputs as I
    its, nsolves = {}, 0
    t0 = time.perf_counter()
    for n, eta0 in COEFF_SWEEP:
        g, _, h, b = I.pcg_test_problem_1d(n, 1.0, 1.0)
        gh, fl = op.bathy_gradient(h, g)
        eta = I.square_wave_depth_1d(n, eta0, gh[0])
        for kind in ("optimal", "replacement"):
            s_, a_, _ = op.coefficients(eta, gh, fl, kind=kind)
            _, it, ok, _ = krylov.pcg(lambda v: op.apply_G(eta, gh, v, g), lambda r: op.solve_A(s_, a_, r, g), b,
                                      tol=1e-8, max_iter=20000)
            its[f"{n}/{eta0}/{kind}"] = it if ok else None
            nsolves += 1
    dt = time.perf_counter() - t0
    return {"value": nsolves / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"the {nsolves} solves of the sweep ({dt:.1f} s, FP64 NumPy, single thread)",
            "iters": its}


def bench_coeffs(args):
    """Optimal (Eq:Optcoeff) against replacement (Remark 4.2) coefficients: PCG to
    1e-8 on the square-wave depth of section 6.2 over a sweep of its contrast eta0
    (the depth is small where the slope is large for eta0 < 1)."""
    import numpy as np
    import torch

    from paper_2506_16045_amd import inputs as I
    from paper_2506_16045_amd import sgn

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    ctx = sgn.Context(0)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    rows = []
    for n, eta0 in COEFF_SWEEP:
        g, _, h, b = I.pcg_test_problem_1d(n, 1.0, 1.0)
        gh_d, _ = ctx.bathy_prepare(g, to(h))
        eta = I.square_wave_depth_1d(n, eta0, gh_d[0].cpu().numpy())
        e_d, b_d = to(eta), to(b)
        row = {"n": n, "eta0": eta0}
        for kind, ck in (("optimal", sgn.COEFF_OPTIMAL), ("replacement", sgn.COEFF_REPLACEMENT)):
            opts = sgn.solve_opts(tol=1e-8, max_iter=20000, check_every=8, coeff_kind=ck)
            ctx.krylov_solve(g, e_d, gh_d, b_d, opts=opts)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            reps = 5
            for _ in range(reps):
                _, res = ctx.krylov_solve(g, e_d, gh_d, b_d, opts=opts)
            torch.cuda.synchronize()
            row[kind] = {"iters": res.iters, "converged": res.converged, "relres": res.relres,
                         "ms_per_solve": round(1e3 * (time.perf_counter() - t0) / reps, 3),
                         "sigma": res.sigma, "alpha": res.alpha}
        row["ratio"] = row["replacement"]["iters"] / max(row["optimal"]["iters"], 1)
        print(f"n={n} eta0={eta0}: optimal {row['optimal']['iters']} / replacement "
              f"{row['replacement']['iters']} iterations", file=sys.stderr, flush=True)
        rows.append(row)
    head = next(r for r in rows if r["n"] == 512 and r["eta0"] == 0.05)
    out = {"metric": "PCG iterations to 1e-8 on the square-wave depth: replacement / optimal coefficients",
           "value": head["ratio"], "unit": "iteration ratio (n=512, eta0=0.05)", "n_gpus": 1,
           "steps": 5, "warmup": 1, "higher_is_better": False, "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "section 6.2 test problem (h0 = 1, b = cos 4 pi x on [0, 1]) with the square-wave "
                                  "depth 0.1 / 0.1 eta0, tol 1e-8, zero initial guess"},
           "sweep": rows, "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline_coeffs(),
           "device": torch.cuda.get_device_name(0)}
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


def cpu_baseline_walls(cfg):
    """The oracle's wall PCG (cosine / sine series), as it stands, on the same solve."""
    from oracle import walls as W
    g = cfg["grid"]
    gh, fl = W.bathy_gradient(cfg["h"], g)
    t0 = time.perf_counter()
    _, it, ok, _ = W.pcg_solve(cfg["eta"], gh, fl, cfg["b"], g, tol=cfg["tol"])
    dt = time.perf_counter() - t0
    return {"value": 1.0 / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"one solve ({dt:.1f} s, FP64 NumPy/SciPy DCT-DST, single thread; {it} iterations)"}


def bench_walls(args):
    """Constraint solves in a closed basin (walls): solves/s of the library's wall path,
    FP64 (PCG on the basin's own points in cosine / sine amplitudes) and mixed
    (reflection onto the periodic twin), with the PCG kernels timed; then FP64 RK4
    steps of the basin through a wall stepping state (on the basin's points)."""
    import numpy as np
    import torch

    from paper_2506_16045_amd import inputs as I
    from paper_2506_16045_amd import sgn

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    cfg = I.config_walls(args.n // 2 if args.n > 512 else args.n)
    g = cfg["grid"]
    ctx = sgn.Context(0)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    gh, flat = ctx.bathy_prepare(g, to(cfg["h"]))
    e_d, b_d = to(cfg["eta"]), to(cfg["b"])
    res_by = {}
    for prec_name, prec in (("fp64", sgn.FP64), ("mixed", sgn.MIXED)):
        opts = sgn.solve_opts(tol=cfg["tol"], precision=prec, check_every=args.check_every, inner_tol=args.inner_tol)
        for _ in range(max(args.warmup, 1)):
            ctx.krylov_solve(g, e_d, gh, b_d, opts=opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            u, res = ctx.krylov_solve(g, e_d, gh, b_d, opts=opts)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ctx.profile_begin()
        ctx.krylov_solve(g, e_d, gh, b_d, opts=opts)
        prof = ctx.profile_end()
        res_by[prec_name] = {"solves_per_s": args.steps / el, "ms_per_solve": 1e3 * el / args.steps,
                             "iters": res.iters, "outer_iters": res.outer_iters, "relres": res.relres,
                             "converged": res.converged,
                             "kernel_avg_us": {k: round(1e3 * v[1] / v[0], 2) for k, v in prof.items() if v[0]}}
    # RK4 steps of the basin (the hump released from rest) through a wall stepping state
    h_d = to(cfg["h"])
    u0 = torch.zeros((2,) + g.shape, dtype=torch.float64, device=e_d.device)
    U0 = ctx.apply_constraint(g, e_d, gh, u0)
    st = sgn.State(ctx, g, h_d, gh, flat, e_d.clone(), U0, u0)
    sopts = sgn.solve_opts(tol=cfg["tol"], check_every=args.check_every)
    st.step_rk4(0.05, max(args.warmup, 1), sopts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sinfo = st.step_rk4(0.05, args.steps, sopts)
    torch.cuda.synchronize()
    sel = time.perf_counter() - t0
    stepping = {"scheme": "rk4", "dt": 0.05, "steps": args.steps, "ms_per_step": 1e3 * sel / args.steps,
                "grid_pt_steps_per_s": g.npts * args.steps / sel, "krylov_iters_per_solve": sinfo.iters / max(sinfo.solves, 1),
                "converged": bool(sinfo.converged)}
    st.close()
    main = res_by["fp64"]
    kind = "pcg_r1"
    twin = (2 * g.nx, 2 * g.ny)
    nbytes = kernel_bytes(kind, 2, g.nx, g.ny, 8)   # the FP64 row pass runs on the basin's own points
    avg = main["kernel_avg_us"].get(kind)
    roof = None
    if avg:
        ach = nbytes / (avg * 1e-6) / 1e9
        roof = {"bound": "hbm", "kernel": kind, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None, "bytes_per_launch": nbytes,
                "avg_launch_us": avg, "timing": "HIP events around every launch of one further solve"}
    out = {"metric": "constraint solves/s in a closed basin (walls)", "value": main["solves_per_s"],
           "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": main["ms_per_solve"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"walls basin {g.nx}x{g.ny} cells on {g.Lx:g}x{g.Ly:g} (FP64 PCG solves and "
                                  f"FP64 RK4 steps on the cells in cosine / sine amplitudes; mixed precision on the "
                                  f"periodic twin {twin[0]}x{twin[1]}), Gaussian bump bathymetry, surface hump, "
                                  f"tol {cfg['tol']:g}, zero initial guess", "parallelism": "single GPU"},
           "precisions": res_by, "stepping": stepping, "roofline": roof,
           "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline_walls(cfg),
           "device": torch.cuda.get_device_name(0)}
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


def bench_batch(args):
    import numpy as np
    import torch

    from paper_2506_16045_amd import inputs as I
    from paper_2506_16045_amd import sgn

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    prec = sgn.MIXED if args.precision == "mixed" else sgn.FP64
    tol = 1e-10
    opts = sgn.solve_opts(tol=tol, precision=prec, inner_tol=args.inner_tol if prec == sgn.MIXED else 1e-5,
                          max_iter=5000, max_outer=40)
    systems = I.config_c4(args.count)
    ctx = sgn.Context(0)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    etas, ghs, bs, ustars, sizes, periods = [], [], [], [], [], []
    for g, eta, h, u_star in systems:
        gh, _ = ctx.bathy_prepare(g, to(h))
        e = to(eta)
        us = to(u_star)
        bs.append(ctx.apply_constraint(g, e, gh, us).reshape(-1))
        etas.append(e)
        ghs.append(gh.reshape(-1))
        ustars.append(us.reshape(-1))
        sizes.append(g.nx)
        periods.append(g.Lx)
    eta_p, gh_p, b_p, us_p = (torch.cat(x) for x in (etas, ghs, bs, ustars))
    npts = int(sum(sizes))
    u = torch.zeros(npts, dtype=torch.float64, device=dev)
    for _ in range(max(args.warmup, 1)):
        u.zero_()
        ctx.batch_solve(sizes, periods, eta_p, gh_p, b_p, u, opts)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        u.zero_()
        _, res, _ = ctx.batch_solve(sizes, periods, eta_p, gh_p, b_p, u, opts)
        lat.append((time.perf_counter() - s0) * 1e3)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = {"batch": (0, 0.0)}
    if not args.no_kernel_timing:
        ctx.profile_begin()
        for _ in range(args.timing_steps):
            u.zero_()
            ctx.batch_solve(sizes, periods, eta_p, gh_p, b_p, u, opts)
        prof = ctx.profile_end()
    # accuracy against the exact discrete solutions u* (b = G u*)
    err = []
    o = 0
    for n in sizes:
        d = torch.linalg.vector_norm(u[o:o + n] - us_p[o:o + n]) / torch.linalg.vector_norm(us_p[o:o + n])
        err.append(float(d.item()))
        o += n
    iters = [r.iters for r in res]
    roofline = None
    nl, ms = prof["batch"]
    if nl:
        avg_us = 1e3 * ms / nl
        nbytes = batch_bytes(sizes, res, prec == sgn.MIXED)
        achieved = nbytes / (avg_us * 1e-6) / 1e9
        roofline = {"bound": "hbm", "kernel": "k_batch_solve", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                    "bytes_per_launch": nbytes, "avg_launch_us": round(avg_us, 2),
                    "timing": f"HIP events around {nl} launches"}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_batch(systems, tol, args.cpu_sample)
    out = {
        "metric": "batched 1D SGN constraint solves/s (ragged N, per-system convergence); Krylov iters/solve; "
                  "p50/p99 latency",
        "value": len(sizes) * args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec == sgn.MIXED else "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"{len(sizes)} independent 1D constraint solves in one launch, N from "
                         f"{{512..8192}} on L=400, 1-3 random Gaussian bumps, random solitary waves, "
                         f"b = G u*, tol {tol:g}, zero initial guess"),
            "precision": args.precision, "systems": len(sizes), "points": npts, "tol": tol,
            "parallelism": "single GPU",
        },
        "points_per_s": npts * args.steps / elapsed,
        "krylov_iters_per_solve": float(np.mean(iters)),
        "krylov_iters_max": int(max(iters)),
        "outer_per_solve": float(np.mean([r.outer_iters for r in res])),
        "batch_latency_ms": {"p50": percentile(lat, 0.5), "p99": percentile(lat, 0.99)},
        "checks": {"max_rel_err_vs_exact": max(err), "all_converged": all(r.converged for r in res)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "device": torch.cuda.get_device_name(0),
    }
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


def bench_serve(args):
    import numpy as np
    import torch

    from paper_2506_16045_amd import inputs as I
    from paper_2506_16045_amd import sgn

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    rates = [float(r) for r in args.rates.split(",")]
    nreq = args.serve_requests
    rng = np.random.default_rng(I.SEED_BASE + 5)
    ctx = sgn.Context(0)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    # a few distinct payloads per (kind, dim, size), built before any timing;
    # solve right-hand sides b = G u* and grad h are formed on the device
    per = 3
    pool = {}
    for dim, sizes in ((1, I.C5_SIZES_1D), (2, I.C5_SIZES_2D)):
        for n in sizes:
            for kind in ("solve", "step"):
                lst = []
                for _ in range(per):
                    r = I.config_c5_request(rng, kind=kind, dim=dim, n=n)
                    g = r["grid"]
                    gh, _ = ctx.bathy_prepare(g, to(r["h"]))
                    if kind == "solve":
                        b = ctx.apply_constraint(g, to(r["eta"]), gh, to(r["u"]))
                        r["gh"] = gh.cpu().numpy()
                        r["rhs"] = b.cpu().numpy()
                    lst.append(r)
                pool[(kind, dim, n)] = lst
    ctx.close()
    torch.cuda.synchronize()
    # the request sequence (same for every precision and rate)
    seq = []
    for _ in range(nreq):
        dim = 1 if rng.uniform() < 0.7 else 2
        kind = "solve" if rng.uniform() < 0.5 else "step"
        n = int(rng.choice(np.asarray(I.C5_SIZES_1D if dim == 1 else I.C5_SIZES_2D)))
        seq.append((kind, dim, n, int(rng.integers(0, per))))

    def make(srv, key, opts):
        kind, dim, n, k = key
        r = pool[(kind, dim, n)][k]
        if kind == "solve":
            return srv.solve_request(r["grid"], r["eta"], r["gh"], r["rhs"], opts=opts)
        return srv.step_request(r["grid"], r["h"], r["eta"], r["u"], r["dt"], r["nsteps"], opts=opts)

    precs = ["fp64", "mixed"] if args.precision_serve == "both" else [args.precision_serve]
    results = {}
    served = {}   # (precision, payload key) -> output of its first served result
    for pname in precs:
        prec = sgn.MIXED if pname == "mixed" else sgn.FP64
        opts = sgn.solve_opts(tol=1e-10, precision=prec, inner_tol=args.inner_tol, max_iter=5000, max_outer=40)
        srv = sgn.Server(0, lanes=args.lanes)
        for key in sorted({(k, d, n, 0) for (k, d, n, _) in seq}):
            srv.wait(srv.submit(make(srv, key, opts)))          # warm-up: one request of each shape
        rows = []
        for rate in rates:
            gaps = np.random.default_rng(I.SEED_BASE + int(rate)).exponential(1.0 / rate, nreq)
            arrive = np.cumsum(gaps)
            ids = []
            t0 = time.perf_counter()
            for key, ta in zip(seq, arrive):
                dt = t0 + ta - time.perf_counter()
                if dt > 0:
                    time.sleep(dt)
                ids.append((key, srv.submit(make(srv, key, opts))))
            t_sub_end = time.perf_counter() - t0
            res = []
            for key, rid in ids:
                r, out = srv.wait(rid)
                served.setdefault((pname, key), out)
                if r.status != sgn.OK:
                    raise RuntimeError(f"request {key} failed with status {r.status}")
                res.append((key, r))
            lat = [1e3 * (r.t_done - r.t_submit) for _, r in res]
            t_first = min(r.t_submit for _, r in res)
            t_last = max(r.t_done for _, r in res)
            span = t_last - t_first
            pts = sum(pool[(k[0], k[1], k[2])][0]["grid"].npts * pool[(k[0], k[1], k[2])][0]["nsteps"]
                      for k, _ in res if k[0] == "step")
            row = {"rate": rate, "offered_req_s": nreq / max(t_sub_end, 1e-9), "throughput_req_s": nreq / span,
                   "p50_ms": percentile(lat, 0.5), "p99_ms": percentile(lat, 0.99),
                   "grid_pt_steps_s": pts / span,
                   "batched_fraction": sum(1 for _, r in res if r.batched) / nreq,
                   "mean_batch": float(np.mean([r.batch_size for _, r in res if r.batched] or [0]))}
            for kind in ("solve", "step"):
                lk = [1e3 * (r.t_done - r.t_submit) for k, r in res if k[0] == kind]
                row[f"{kind}_p50_ms"] = percentile(lk, 0.5)
                row[f"{kind}_p99_ms"] = percentile(lk, 0.99)
            # per request shape: count, mean time on a lane or in a batched launch
            # (start to done), the share of the summed service time, mean batch
            shapes = {}
            for k, r in res:
                e = shapes.setdefault(f"{k[0]}-{k[1]}d-{k[2]}", {"count": 0, "service_ms": 0.0, "batch": 0.0})
                e["count"] += 1
                e["service_ms"] += 1e3 * (r.t_done - r.t_start)
                e["batch"] += r.batch_size if r.batched else 1
            tot_service = sum(e["service_ms"] for e in shapes.values())
            row["per_shape"] = {name: {"count": e["count"], "mean_service_ms": round(e["service_ms"] / e["count"], 3),
                                       "service_share": round(e["service_ms"] / max(tot_service, 1e-9), 3),
                                       "mean_batch": round(e["batch"] / e["count"], 2)}
                                for name, e in sorted(shapes.items())}
            rows.append(row)
            print(json.dumps({"serve_progress": pname, **{k: round(v, 3) for k, v in row.items() if k != "per_shape"}}),
                  file=sys.stderr, flush=True)
        srv.close()
        results[pname] = rows
    best = max(results, key=lambda p: results[p][-1]["throughput_req_s"])
    out = {
        "metric": "served SGN requests: throughput and p50/p99 latency per Poisson arrival rate",
        "value": results[best][-1]["throughput_req_s"],
        "unit": "req/s",
        "n_gpus": 1,
        "steps": nreq,
        "warmup": 1,
        "ms_per_step": 1e3 / results[best][-1]["throughput_req_s"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if best == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": (f"served stream: {nreq} requests per rate, 70% 1D N 1024..16384 / 30% 2D "
                                "128^2..1024^2, half solves (tol 1e-10) and half 10-step RK4 runs, Poisson "
                                f"arrivals at {args.rates} req/s, {args.lanes} worker lanes + 2 batching lanes (1D solves, 1D RK4 runs)"),
                   "rates": rates, "requests_per_rate": nreq, "parallelism": "single GPU",
                   "hw_queues": int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))},
        "value_precision": best,
        "per_rate": results,
        "roofline": None,
        "cpu_baseline": None if args.no_cpu_baseline else serve_cpu_baseline(pool, served, precs),
        "device": torch.cuda.get_device_name(0),
    }
    print(json.dumps(out), flush=True)
    return 0


def serve_cpu_baseline(pool, served, precs):
    """The FP64 oracle on a bounded sample of the served payloads (every 1D
    payload, the 2D 128^2 ones and the first 2D 256^2 one of each kind), timed
    on the host, and the error of each sampled served result against it.  Every
    request of a payload returned the same result bit for bit (alone or in the
    mix, tested), so the error of a payload is that of each of its requests.
    The oracle forms its own inputs from the seeded fields (h, eta and u* for a
    solve, h, eta and u for a run) and solves to tol 1e-12."""
    import numpy as np
    from oracle import diagnostics as dg
    from oracle import krylov
    from oracle import operators as op
    from oracle import stepping as ost
    keys = sorted({k for _, k in served})
    sample = [k for k in keys if k[1] == 1 or k[2] == 128 or (k[2] == 256 and k[3] == 0)]
    errs = {}
    t0 = time.perf_counter()
    for key in sample:
        kind, dim, n, i = key
        r = pool[(kind, dim, n)][i]
        g = r["grid"]
        name = f"{kind}-{dim}d-{n}-#{i}"
        if kind == "solve":
            gh, fl = op.bathy_gradient(r["h"], g)
            b = op.apply_G(r["eta"], gh, r["u"], g)
            sg, al, _ = op.coefficients(r["eta"], gh, fl)
            u_ref, _, _, _ = krylov.pcg(lambda v: op.apply_G(r["eta"], gh, v, g),
                                        lambda q: op.solve_A(sg, al, q, g), b, tol=1e-12, max_iter=5000)
            for p in precs:
                if (p, key) in served:
                    u = served[(p, key)]["u"].reshape(u_ref.shape)
                    errs.setdefault(name, {})[p] = float(dg.rel_l2(u, u_ref))
        else:
            pb = ost.Problem.from_h(g, r["h"], tol=1e-12)
            e_r, U_r, u_r = ost.run_rk4(pb, r["eta"], pb.G(r["eta"], r["u"]), r["u"], r["dt"], r["nsteps"])
            for p in precs:
                if (p, key) in served:
                    o = served[(p, key)]
                    e, u = o["eta"].reshape(e_r.shape), o["u"].reshape(u_r.shape)
                    fe = dg.field_errors(e, pb.G(e, u), u, e_r, U_r, u_r, r["h"])
                    errs.setdefault(name, {})[p] = float(max(fe.values()))
    dt = time.perf_counter() - t0
    worst = {p: max((v[p] for v in errs.values() if p in v), default=None) for p in precs}
    return {"value": len(sample) / dt, "unit": "req/s", "cores": 1, "kind": "oracle",
            "sample": (f"{len(sample)} distinct served payloads (all 1D, 2D 128^2, one 2D 256^2 per kind), "
                       f"FP64 NumPy, single thread, {dt:.1f} s"),
            "per_result_error_vs_oracle": errs, "max_error_vs_oracle": worst}


def _state_1d(ctx, cfg, to):
    from paper_2506_16045_amd import sgn
    g = cfg["grid"]
    h = to(cfg["h"])
    gh, flat = ctx.bathy_prepare(g, h)
    eta, u = to(cfg["eta"]), to(cfg["u"])
    U = ctx.apply_constraint(g, eta, gh, u)
    return sgn.State(ctx, g, h, gh, flat, eta, U, u)


def _leg_step(st, leg, dt, n, opts):
    if leg == "rk4":
        return st.step_rk4(dt, n, opts)
    if leg == "ab3":
        return st.step_ab(3, dt, n, opts)
    return st.step_linimp(dt, n, None, opts)


def _oracle_leg(cfg, leg, steps):
    from oracle import stepping as ost
    pb = ost.Problem.from_h(cfg["grid"], cfg["h"], tol=cfg["tol"])
    U0 = pb.G(cfg["eta"], cfg["u"])
    t0 = time.perf_counter()
    if leg == "rk4":
        out = ost.run_rk4(pb, cfg["eta"], U0, cfg["u"], cfg["dt"], steps)
    elif leg == "ab3":
        out = ost.run_ab(pb, 3, cfg["eta"], U0, cfg["u"], cfg["dt"], steps)
    else:
        out = ost.run_sbdf2(pb, cfg["eta"], U0, cfg["u"], cfg["dt"], steps)
    return out, time.perf_counter() - t0, pb.iters


def _rel_fields(dev, ref, h):
    import numpy as np
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    return {"zeta": rel(dev[0] - h, ref[0] - h), "U": rel(dev[1], ref[1]), "u": rel(dev[2], ref[2])}


def bench_c1(args):
    """1D flat solitary wave, RK4, the stated 500 steps (section 6, ExSleta/ExSlu)."""
    import numpy as np
    import torch
    from paper_2506_16045_amd import inputs as I
    from paper_2506_16045_amd import sgn
    dev = torch.device("cuda", 0)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    cfg = I.config_c1()
    g = cfg["grid"]
    steps = args.steps if args.steps is not None else cfg["steps"]
    ctx = sgn.Context(0)
    opts = sgn.solve_opts(tol=cfg["tol"], check_every=args.check_every)
    for _ in range(max(args.warmup, 0)):
        st = _state_1d(ctx, cfg, to)
        st.step_rk4(cfg["dt"], steps, opts)
        st.close()
    st = _state_1d(ctx, cfg, to)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = st.step_rk4(cfg["dt"], steps, opts)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    if not info.converged:
        raise RuntimeError("a Krylov solve did not converge")
    fields = tuple(t.detach().cpu().numpy() for t in (st.eta, st.U, st.u))
    st.close()
    T = cfg["dt"] * steps
    e_x, u_x = I.solitary_wave(g, cfg["h0"], cfg["a"], cfg["x0"], t=T)
    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    cpu = None
    if not args.no_cpu_baseline:
        ref, sec, iters = _oracle_leg(cfg, "rk4", steps)
        cpu = {"value": g.npts * steps / sec, "unit": "grid-pt-steps/s", "cores": 1, "kind": "oracle",
               "sample": f"the whole run, {steps} RK4 steps ({sec:.1f} s, FP64 NumPy, single thread; "
                         f"iterations/solve {np.mean(iters):.2f})",
               "device_vs_oracle_rel_l2": _rel_fields(fields, ref, cfg["h"])}
    out = {"metric": "1D SGN grid-pt-steps/s at 1e-10 rel err; Krylov iters/solve",
           "value": g.npts * steps / el, "unit": "grid-pt-steps/s", "n_gpus": 1, "steps": steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * el / steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "1D flat solitary wave: N=256 on L=80, h0=1, a=0.2 at x=20, RK4 dt=0.01, "
                                  f"{steps} steps, PCG tol 1e-12", "scheme": "rk4"},
           "krylov_iters_per_solve": info.iters / max(info.solves, 1), "solves": info.solves,
           "vs_exact_solitary_wave": {"zeta": rel(fields[0] - 1.0, e_x - 1.0), "u": rel(fields[2], u_x),
                                      "t": T},
           "cpu_baseline": cpu, "device": torch.cuda.get_device_name(0)}
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


def bench_c2(args):
    """1D shelf: SBDF2 (Eq:MM), AB3+PCG (Eq:AB), RK4+PCG (Eq:ERK), FP64 and mixed,
    the stated 2000 steps per leg."""
    import numpy as np
    import torch
    from paper_2506_16045_amd import inputs as I
    from paper_2506_16045_amd import sgn
    dev = torch.device("cuda", 0)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    cfg = I.config_c2()
    g = cfg["grid"]
    steps = args.steps if args.steps is not None else cfg["steps"]
    ctx = sgn.Context(0)
    legs = {}
    for leg in ("sbdf2", "ab3", "rk4"):
        for precision in ("fp64", "mixed"):
            prec = sgn.FP64 if precision == "fp64" else sgn.MIXED
            opts = sgn.solve_opts(tol=cfg["tol"], precision=prec, check_every=args.check_every,
                                  inner_tol=args.inner_tol)
            if args.warmup > 0:
                st = _state_1d(ctx, cfg, to)
                _leg_step(st, leg, cfg["dt"], min(args.warmup, steps), opts)
                st.close()
            st = _state_1d(ctx, cfg, to)
            m0 = float(torch.sum(st.eta - st._keep[0]).item())
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = _leg_step(st, leg, cfg["dt"], steps, opts)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            m1 = float(torch.sum(st.eta - st._keep[0]).item())
            st.close()
            legs[f"{leg}-{precision}"] = {"value": g.npts * steps / el, "ms_per_step": 1e3 * el / steps,
                                          "solves": info.solves,
                                          "krylov_iters_per_solve": info.iters / max(info.solves, 1),
                                          "mass_rel_drift": abs(m1 - m0) / abs(m0)}
    cpu = None
    if not args.no_cpu_baseline:
        sample = min(200, steps)
        cpu = {"unit": "grid-pt-steps/s", "cores": 1, "kind": "oracle",
               "sample": f"the first {sample} steps of each leg (FP64 NumPy, single thread), against a device "
                         f"run of the same length", "legs": {}}
        tot_sec = 0.0
        for leg in ("sbdf2", "ab3", "rk4"):
            ref, sec, _ = _oracle_leg(cfg, leg, sample)
            tot_sec += sec
            rec = {"value": g.npts * sample / sec}
            for precision in ("fp64", "mixed"):
                prec = sgn.FP64 if precision == "fp64" else sgn.MIXED
                st = _state_1d(ctx, cfg, to)
                _leg_step(st, leg, cfg["dt"], sample, sgn.solve_opts(tol=cfg["tol"], precision=prec,
                                                                     inner_tol=args.inner_tol))
                fields = tuple(t.detach().cpu().numpy() for t in (st.eta, st.U, st.u))
                st.close()
                rec[f"device_{precision}_vs_oracle_rel_l2"] = _rel_fields(fields, ref, cfg["h"])
            cpu["legs"][leg] = rec
        cpu["value"] = g.npts * 3 * sample / tot_sec
    main = legs["sbdf2-fp64"]
    out = {"metric": "1D SGN grid-pt-steps/s at 1e-10 rel err; Krylov iters/solve",
           "value": main["value"], "unit": "grid-pt-steps/s", "n_gpus": 1, "steps": steps,
           "warmup": args.warmup, "ms_per_step": main["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "1D shelf: N=4096 on L=400, depth 1 -> 0.5 (tanh steps), solitary wave a=0.3 "
                                  f"at x=100, dt=0.02, {steps} steps per leg, PCG tol 1e-12; value: the linearly "
                                  "implicit SBDF2 leg in FP64", "scheme": "sbdf2 | ab3 | rk4"},
           "legs": legs, "cpu_baseline": cpu, "device": torch.cuda.get_device_name(0)}
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


def cpu_baseline_batch(systems, tol, count):
    """The oracle's PCG, as it stands, on the first `count` systems of the ensemble
    (forming b = G u* is not timed)."""
    from oracle import krylov
    from oracle import operators as op
    dt = 0.0
    its = []
    for g, eta, h, u_star in systems[:count]:
        gh, _ = op.bathy_gradient(h, g)
        fl = not gh.any()
        b = op.apply_G(eta, gh, u_star, g)
        sg, al, _ = op.coefficients(eta, gh, fl)
        t1 = time.perf_counter()
        _, it, ok, _ = krylov.pcg(lambda v: op.apply_G(eta, gh, v, g), lambda r: op.solve_A(sg, al, r, g), b,
                                  tol=tol, max_iter=5000)
        dt += time.perf_counter() - t1
        its.append(it)
    return {"value": count / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"the first {count} systems of the ensemble, FP64 NumPy, single thread ({dt:.1f} s; "
                      f"iterations/solve {sum(its) / max(len(its), 1):.1f})"}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["rk4-2d", "c1", "c2", "batch", "serve", "coeffs", "walls"],
                    default="rk4-2d")
    ap.add_argument("--rates", default="50,100,200,500,1000,2000", help="arrival rates of the serve workload")
    ap.add_argument("--serve-requests", type=int, default=1000, help="requests per rate (serve workload)")
    ap.add_argument("--lanes", type=int, default=6, help="worker lanes of the server (serve workload)")
    ap.add_argument("--precision-serve", choices=["both", "fp64", "mixed"], default="both")
    ap.add_argument("--count", type=int, default=512, help="systems of the batched workload")
    ap.add_argument("--cpu-sample", type=int, default=512, help="systems the CPU oracle solves for its baseline")
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 40; the stated run length for c1 and c2)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="fp64")
    ap.add_argument("--no-compare", action="store_true", help="skip timing the other precision")
    ap.add_argument("--n", type=int, default=1024, help="grid points per side (default 1024)")
    ap.add_argument("--check-every", type=int, default=8)
    ap.add_argument("--dealias", action="store_true",
                    help="rk4-2d with the de-aliased right-hand side (nonlinear terms on the 2x padded grid)")
    ap.add_argument("--inner-tol", type=float, default=1e-5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-timing", action="store_true", help="skip the per-kernel HIP-event timing pass")
    ap.add_argument("--timing-steps", type=int, default=5, help="steps of the per-kernel timing pass")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB before the timed region "
                         "(reference kernel for scaling the HBM byte counters of a profiler run)")
    ap.add_argument("--summarize-kernels", metavar="DB", help="write a kernel-duration summary of a "
                    "rocprofv3 --kernel-trace results database (no GPU needed) and exit")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="HBM bytes per launch of the PCG passes from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE "
                         "runs of this script with --calib-copy-mib (no GPU needed) and exit")
    ap.add_argument("--traffic-pattern", help="with --summarize-traffic: bytes per dispatch of the kernels "
                    "matching this regular expression, per launch shape, instead of the PCG loop families")
    ap.add_argument("--command", default="", help="command line recorded in a summary")
    ap.add_argument("--out", help="summary output path")
    args = ap.parse_args(argv)

    if args.summarize_kernels or args.summarize_traffic:
        from paper_2506_16045_amd import profiling
        if args.summarize_kernels:
            text = profiling.kernel_summary_md(args.summarize_kernels, args.command,
                                               f"Kernel durations: {args.precision}, {args.n}x{args.n} RK4 workload")
        elif args.traffic_pattern:
            rec = profiling.traffic_by_kernel(args.summarize_traffic[0], args.summarize_traffic[1],
                                              args.calib_copy_mib * (1 << 20), args.traffic_pattern)
            rec.update({"n": args.n, "kernel_source_sha": kernel_source_hash(), "command": args.command})
            text = json.dumps(rec, indent=1) + "\n"
        else:
            rec = profiling.traffic(args.summarize_traffic[0], args.summarize_traffic[1],
                                    args.calib_copy_mib * (1 << 20), args.n)
            rec.update({"n": args.n, "kernel_source_sha": kernel_source_hash(), "command": args.command})
            text = json.dumps(rec, indent=1) + "\n"
        if args.out:
            with open(args.out, "w") as fh:
                fh.write(text)
        print(text)
        return 0

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library's path is single-GPU "
              "(how it would shard across GPUs is described in the design notes; it is not run)", file=sys.stderr)
        return 2

    if args.workload == "c1":
        return bench_c1(args)
    if args.workload == "c2":
        return bench_c2(args)
    if args.steps is None:
        args.steps = 40
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        # the server's lanes overlap on the device only with a hardware queue
        # each; HIP's default of 4 queues per process makes 2 batching lanes and
        # the worker lanes share them.  Read when the HIP runtime starts, so set here.
        need = args.lanes + 2
        try:
            have = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
        except ValueError:
            have = 4
        if have < need:
            os.environ["GPU_MAX_HW_QUEUES"] = str(need)
        return bench_serve(args)
    if args.workload == "coeffs":
        return bench_coeffs(args)
    if args.workload == "walls":
        return bench_walls(args)

    import numpy as np
    import torch

    from paper_2506_16045_amd import inputs as I
    from paper_2506_16045_amd import profiling, sgn

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    cfg = I.config_c3(args.n)
    g = cfg["grid"]
    ctx = sgn.Context(0)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    h = to(cfg["h"])
    gh, flat = ctx.bathy_prepare(g, h)

    def new_state():
        eta = to(cfg["eta"])
        u = to(cfg["u"])
        U = ctx.apply_constraint(g, eta, gh, u)
        st = sgn.State(ctx, g, h, gh, flat, eta, U, u)
        if args.dealias:
            st.set_dealias(True)
        return st

    if args.calib_copy_mib > 0:
        nel = args.calib_copy_mib * (1 << 20) // 8
        src_c = torch.rand(nel, dtype=torch.float64, device=dev)
        dst_c = torch.empty_like(src_c)
        torch.cuda.synchronize()
        dst_c.copy_(src_c)
        torch.cuda.synchronize()
        del src_c, dst_c

    def run(precision: str, kernel_timing: bool):
        prec = sgn.MIXED if precision == "mixed" else sgn.FP64
        opts = sgn.solve_opts(tol=cfg["tol"], precision=prec, check_every=args.check_every,
                              inner_tol=args.inner_tol)
        state = new_state()
        mass0 = float(torch.sum(state.eta - h).item())
        if args.warmup > 0:
            state.step_rk4(cfg["dt"], args.warmup, opts)
        torch.cuda.synchronize()
        # timed region: K steps in one stepping call, no instrumentation
        t0 = time.perf_counter()
        info = state.step_rk4(cfg["dt"], args.steps, opts)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        solves, iters, max_iters = info.solves, info.iters, info.max_iters
        if not info.converged:
            raise RuntimeError("a Krylov solve did not converge")
        # per-step latency: further steps, one call each, synchronised after each
        lat = []
        for _ in range(min(args.steps, 20)):
            s0 = time.perf_counter()
            info = state.step_rk4(cfg["dt"], 1, opts)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - s0) * 1e3)
            if not info.converged:
                raise RuntimeError("a Krylov solve did not converge")
        # kernel timing: HIP events around every launch of each kernel family on the
        # library's stream, over further steps of the same run (events between
        # launches slow the step down, so they stay out of the timed region above)
        prof = {k: (0, 0.0) for k in ctx.KERNEL_KINDS}
        launches = {k: [] for k in ctx.KERNEL_KINDS}
        if kernel_timing and args.timing_steps > 0:
            ctx.profile_begin()
            state.step_rk4(cfg["dt"], args.timing_steps, opts)
            prof = ctx.profile_end()
            launches = ctx.profile_launches()
        # device-side property checks of the final state (not part of the timed region)
        Gu = ctx.apply_constraint(g, state.eta, gh, state.u)
        relres = float((torch.linalg.vector_norm(Gu - state.U) / torch.linalg.vector_norm(state.U)).item())
        drift = abs(float(torch.sum(state.eta - h).item()) - mass0) / max(abs(mass0), 1e-300)
        state.close()
        return {"precision": precision, "prec": prec, "elapsed": elapsed, "lat": lat, "solves": solves,
                "iters": iters, "max_iters": max_iters, "prof": prof, "launches": launches, "relres": relres,
                "drift": drift,
                "value": g.npts * args.steps / elapsed, "ms_per_step": 1e3 * elapsed / args.steps}

    main_run = run(args.precision, not args.no_kernel_timing)
    other = None
    if not args.no_compare:
        o = run("mixed" if args.precision == "fp64" else "fp64", False)
        other = {"precision": o["precision"], "value": o["value"], "ms_per_step": o["ms_per_step"],
                 "krylov_iters_per_solve": o["iters"] / max(o["solves"], 1),
                 "checks": {"constraint_relres": o["relres"], "mass_rel_drift": o["drift"]}}
    prec = main_run["prec"]
    prof = main_run["prof"]
    word = 4 if prec == sgn.MIXED else 8
    kstats = {}
    kinds = ("pcg_c1_f32", "pcg_r1_f32", "pcg_c2_f32", "pcg_init_f32") if prec == sgn.MIXED else \
        ("pcg_c1", "pcg_r1", "pcg_c2", "pcg_init")
    rhs_kinds = ("rhs_rows_fwd", "rhs_cols", "rhs_rows_inv", "rhs_flux") if not args.dealias else ()
    for kind in kinds + rhs_kinds:
        n_launch, ms = prof[kind]
        if n_launch:
            # a Krylov pass launched after its solve has converged returns at once:
            # those launches move none of the pass's bytes, so the roofline prices
            # the full launches only (the counter runs exclude them likewise)
            full, early = profiling.split_launches(main_run["launches"][kind])
            avg_full = 1e3 * sum(full) / len(full) if full else 1e3 * ms / n_launch
            kstats[kind] = {"launches": n_launch, "early_exit_launches": len(early), "avg_us": avg_full,
                            "avg_all_us": 1e3 * ms / n_launch, "total_ms": ms}
    # every timed family against the HBM roofline (algorithmic bytes per launch over its
    # event-timed average); `roofline` is the family with the largest total time
    # (FP32 inner passes in mixed mode; the FP64 residual passes are separate families;
    # the right-hand side is FP64 in both precisions)
    rooflines = {}
    for kind, st_ in kstats.items():
        if kind.startswith("pcg_init"):
            continue
        w_k = 8 if kind.startswith("rhs_") else word
        nbytes = kernel_bytes(kind, g.d, g.nx, g.ny, w_k)
        achieved = nbytes / (st_["avg_us"] * 1e-6) / 1e9
        rooflines[kind] = {"bound": "hbm", "kernel": kind, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                           "traffic": measured_traffic(kind, args.n), "bytes_per_launch": nbytes,
                           "avg_launch_us": round(st_["avg_us"], 2), "launches": st_["launches"],
                           "early_exit_launches": st_["early_exit_launches"],
                           "avg_all_launches_us": round(st_["avg_all_us"], 2), "total_ms": round(st_["total_ms"], 4)}
    roofline = None
    if rooflines:
        dom = max(rooflines, key=lambda k: rooflines[k]["total_ms"])
        roofline = dict(rooflines[dom])
        roofline["timing"] = (f"HIP events around every launch over {args.timing_steps} further steps; "
                              "avg_launch_us over the full launches (early exits after convergence excluded)")
        del roofline["total_ms"]

    cpu = None
    if not args.no_cpu_baseline:
        # one device step from the initial data, compared with the oracle's step inside the baseline leg
        st1 = new_state()
        st1.step_rk4(cfg["dt"], 1, sgn.solve_opts(tol=cfg["tol"], precision=prec, check_every=args.check_every,
                                                   inner_tol=args.inner_tol))
        dev_fields = tuple(t.detach().cpu().numpy() for t in (st1.eta, st1.U, st1.u))
        st1.close()
        cpu = cpu_baseline(cfg, 1, dev_fields, args.dealias)

    lat = main_run["lat"]
    out = {
        "metric": "2D SGN grid-pt-steps/s at 1e-9 rel err; Krylov iters/solve; p50/p99 latency",
        "value": main_run["value"],
        "unit": "grid-pt-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec == sgn.MIXED else "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"2D SGN over a Gaussian bump, RK4: {g.nx}x{g.ny} grid on {g.Lx:g}x{g.Ly:g}, "
                         "h0=1, bump height 0.5 radius 10 at the centre, line solitary wave a=0.2 at x=50, "
                         f"dt={cfg['dt']}, Krylov tol {cfg['tol']:g}"
                         + (", de-aliased right-hand side (2x zero-padded grid)" if args.dealias else "")),
            "scheme": "rk4", "rhs": "dealiased-2x" if args.dealias else "plain", "precision": args.precision, "grid": [g.nx, g.ny], "dt": cfg["dt"],
            "tol": cfg["tol"], "initial_guess": "extrapolated per stage", "parallelism": "single GPU",
        },
        "krylov_iters_per_solve": main_run["iters"] / max(main_run["solves"], 1),
        "krylov_max_iters": main_run["max_iters"],
        "solves": main_run["solves"],
        "step_latency_ms": {"p50": percentile(lat, 0.5), "p99": percentile(lat, 0.99)},
        "checks": {"constraint_relres": main_run["relres"], "mass_rel_drift": main_run["drift"]},
        "other_precision": other,
        "kernels": kstats,
        "kernel_families_ms_per_step": {k: round(v[1] / max(args.timing_steps, 1), 4)
                                         for k, v in prof.items() if v[0]},
        "roofline": roofline,
        "rooflines": rooflines,
        "cpu_baseline": cpu,
        "device": torch.cuda.get_device_name(0),
    }
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
