"""Write the stored oracle trajectories that the long GPU parity tests compare with.

    python tests/golden/make_stepping_golden.py            # everything (~15 min, one core)
    python tests/golden/make_stepping_golden.py c2 c3      # selected parts

Calls only the CPU oracle (oracle/) and the seeded input generators; nothing
here touches the HIP library.  Outputs, next to this file:

  c2_legs.npz       the 1D shelf workload (N = 4096 on L = 400, a = 0.3 at
                    x = 100, dt = 0.02, 2000 steps, PCG tol 1e-12) after the
                    whole run of each leg: RK4+PCG (Eq:ERK), AB3+PCG (Eq:AB)
                    and the linearly implicit SBDF2 (Eq:MM); eta, U, u per leg
                    and the oracle's Krylov iteration totals.
  c3_256_rk4.npz    the 2D bump workload at 256 x 256 (same domain, bump,
                    wave, dt = 0.02) after 500 RK4 steps: at the workload's
                    tol 1e-10 (eta, U, u, iters) and at tol 1e-13 (*_tight).
  stepping_checks.json
                    what the runs show about the readings: SBDF2 at dt = 0.02
                    on the shelf stays bounded and within O(dt^2) of RK4 (the
                    stability check the linearly implicit leg needs before its
                    GPU run); the 1D flat run's crest position and error against
                    the exact solitary wave; the drift between the oracle at
                    tol 1e-10 and at tol 1e-13 (256 x 256 over 500 steps and
                    1024 x 1024 over 5 steps), which bounds how far two correct
                    solvers at the workload's tolerance can differ.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import diagnostics as dg  # noqa: E402
from oracle import stepping as ost  # noqa: E402
from paper_2506_16045_amd import inputs as I  # noqa: E402

C2_STEPS = 2000
C3_SMALL_N = 256
C3_SMALL_STEPS = 500
C3_FULL_STEPS = 5


def _checks_path():
    return os.path.join(HERE, "stepping_checks.json")


def _load_checks():
    p = _checks_path()
    if os.path.exists(p):
        with open(p) as fh:
            return json.load(fh)
    return {}


def _save_checks(d):
    with open(_checks_path(), "w") as fh:
        json.dump(d, fh, indent=2, sort_keys=True)
        fh.write("\n")


def run_leg(cfg, leg, steps, tol=None):
    g = cfg["grid"]
    pb = ost.Problem.from_h(g, cfg["h"], tol=cfg["tol"] if tol is None else tol)
    U0 = pb.G(cfg["eta"], cfg["u"])
    if leg == "rk4":
        out = ost.run_rk4(pb, cfg["eta"], U0, cfg["u"], cfg["dt"], steps)
    elif leg == "ab3":
        out = ost.run_ab(pb, 3, cfg["eta"], U0, cfg["u"], cfg["dt"], steps)
    elif leg == "sbdf2":
        out = ost.run_sbdf2(pb, cfg["eta"], U0, cfg["u"], cfg["dt"], steps)
    else:
        raise ValueError(leg)
    return out, pb.iters


def crest_position(eta, g):
    """Crest of a 1D wave: vertex of the parabola through the grid maximum and its neighbours."""
    i = int(np.argmax(eta))
    n = g.nx
    ym, y0, yp = eta[(i - 1) % n], eta[i], eta[(i + 1) % n]
    den = ym - 2.0 * y0 + yp
    off = 0.5 * (ym - yp) / den if den != 0.0 else 0.0
    return (i + off) * g.Lx / n


def make_c1(checks):
    cfg = I.config_c1()
    t0 = time.time()
    (e, U, u), iters = run_leg(cfg, "rk4", cfg["steps"])
    g = cfg["grid"]
    T = cfg["dt"] * cfg["steps"]
    e_x, u_x = I.solitary_wave(g, cfg["h0"], cfg["a"], cfg["x0"], t=T)
    c, _ = I.solitary_speed_width(cfg["h0"], cfg["a"])
    checks["c1_rk4_500"] = {
        "t": T,
        "crest_exact": cfg["x0"] + c * T,
        "crest_oracle": crest_position(e, g),
        "zeta_rel_l2_vs_exact": dg.rel_l2(e - 1.0, e_x - 1.0),
        "u_rel_l2_vs_exact": dg.rel_l2(u, u_x),
        "iters_per_solve": float(np.mean(iters)),
        "seconds": time.time() - t0,
    }
    print("c1", checks["c1_rk4_500"], flush=True)


def make_c2(checks):
    cfg = I.config_c2()
    out = {}
    info = {}
    for leg in ("rk4", "ab3", "sbdf2"):
        t0 = time.time()
        (e, U, u), iters = run_leg(cfg, leg, C2_STEPS)
        out[f"{leg}_eta"], out[f"{leg}_U"], out[f"{leg}_u"] = e, U, u
        out[f"{leg}_iters"] = np.array([len(iters), int(np.sum(iters))], dtype=np.int64)
        info[leg] = {"solves": len(iters), "iters": int(np.sum(iters)), "seconds": time.time() - t0,
                     "max_abs_zeta": float(np.max(np.abs(e - cfg["h"])))}
        print("c2", leg, info[leg], flush=True)
    np.savez_compressed(os.path.join(HERE, "c2_legs.npz"), **out)
    h = cfg["h"]
    g = cfg["grid"]
    T = cfg["dt"] * C2_STEPS
    e_x, u_x = I.solitary_wave(g, 1.0, cfg["a"], cfg["x0"], t=T)
    checks["c2_legs"] = {
        "steps": C2_STEPS, "dt": cfg["dt"], "t": T,
        "legs": info,
        "sbdf2_vs_rk4": dg.field_errors(out["sbdf2_eta"], out["sbdf2_U"], out["sbdf2_u"],
                                        out["rk4_eta"], out["rk4_U"], out["rk4_u"], h),
        "ab3_vs_rk4": dg.field_errors(out["ab3_eta"], out["ab3_U"], out["ab3_u"],
                                      out["rk4_eta"], out["rk4_U"], out["rk4_u"], h),
        "rk4_zeta_rel_l2_vs_flat_exact": dg.rel_l2(out["rk4_eta"] - h, e_x - 1.0),
        "sbdf2_zeta_rel_l2_vs_flat_exact": dg.rel_l2(out["sbdf2_eta"] - h, e_x - 1.0),
        "mass_rel_drift_sbdf2": abs(dg.mass(out["sbdf2_eta"], h, g) - dg.mass(cfg["eta"], h, g))
        / abs(dg.mass(cfg["eta"], h, g)),
    }


def make_c3_small(checks):
    cfg = I.config_c3(C3_SMALL_N)
    t0 = time.time()
    (e, U, u), iters = run_leg(cfg, "rk4", C3_SMALL_STEPS)
    sec = time.time() - t0
    print("c3-256 tol 1e-10 done", sec, flush=True)
    (e2, U2, u2), iters2 = run_leg(cfg, "rk4", C3_SMALL_STEPS, tol=1e-13)
    np.savez_compressed(os.path.join(HERE, "c3_256_rk4.npz"), eta=e, U=U, u=u,
                        iters=np.array([len(iters), int(np.sum(iters))], dtype=np.int64),
                        eta_tight=e2, U_tight=U2, u_tight=u2,
                        iters_tight=np.array([len(iters2), int(np.sum(iters2))], dtype=np.int64))
    checks["c3_256_rk4_500"] = {
        "steps": C3_SMALL_STEPS, "tol": cfg["tol"], "seconds": sec,
        "iters_per_solve": float(np.mean(iters)),
        "drift_tol_1e-10_vs_1e-13": dg.field_errors(e, U, u, e2, U2, u2, cfg["h"]),
        "iters_per_solve_tol_1e-13": float(np.mean(iters2)),
    }
    print("c3-256", checks["c3_256_rk4_500"], flush=True)


def make_c3_full(checks):
    cfg = I.config_c3(1024)
    t0 = time.time()
    (e, U, u), iters = run_leg(cfg, "rk4", C3_FULL_STEPS)
    sec = time.time() - t0
    (e2, U2, u2), iters2 = run_leg(cfg, "rk4", C3_FULL_STEPS, tol=1e-13)
    checks["c3_1024_rk4_5"] = {
        "steps": C3_FULL_STEPS, "tol": cfg["tol"], "seconds": sec,
        "iters_per_solve": float(np.mean(iters)),
        "drift_tol_1e-10_vs_1e-13": dg.field_errors(e, U, u, e2, U2, u2, cfg["h"]),
        "iters_per_solve_tol_1e-13": float(np.mean(iters2)),
    }
    print("c3-1024", checks["c3_1024_rk4_5"], flush=True)


PARTS = {"c1": make_c1, "c2": make_c2, "c3": make_c3_small, "c3full": make_c3_full}


def main(argv):
    parts = argv or list(PARTS)
    checks = _load_checks()
    for p in parts:
        PARTS[p](checks)
        _save_checks(checks)


if __name__ == "__main__":
    main(sys.argv[1:])
