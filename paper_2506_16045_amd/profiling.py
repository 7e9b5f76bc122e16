"""Summaries of rocprofv3 output (SQLite results databases) for the kernels of
libsgn: per-kernel duration statistics of a --kernel-trace run, and HBM bytes
per launch from --pmc FETCH_SIZE / WRITE_SIZE runs scaled by a reference copy
of known size recorded in the same process.  Used by `bench.py --summarize-*`;
nothing here touches the GPU.
"""
from __future__ import annotations

import collections
import re
import sqlite3
import subprocess


def demangle(names):
    names = list(names)
    if not names:
        return {}
    try:
        out = subprocess.run(["c++filt"], input="\n".join(names), capture_output=True, text=True).stdout
        dem = out.strip().split("\n")
        if len(dem) == len(names):
            return dict(zip(names, dem))
    except OSError:
        pass
    return {n: n for n in names}


def kernel_family(demangled: str, grid_size: int = 0, n: int = 0):
    """(family, precision) of a PCG loop or 2D right-hand-side kernel name, e.g.
    ('pcg_r1', 'f32') or ('rhs_rows_inv', 'f64'), else None.  The right-hand side's
    two column launches share one kernel; they are told apart by their job count
    (grid_size work-items over 256-thread blocks of n/2 + 1 columns per job)."""
    if re.search(r"k_rhs_rows_fwd<2,", demangled):
        return "rhs_rows_fwd", "f64"
    if re.search(r"k_rhs_rows_inv<2,|k_rhs_rows_inv_w\b", demangled):
        return "rhs_rows_inv", "f64"
    if re.search(r"k_cols_lin_jobs<double, 4, [34], 3>", demangled) and n:
        jobs = round(grid_size / (256 * (n // 2 + 1)))
        return ("rhs_cols", "f64") if jobs == 3 else ("rhs_flux", "f64") if jobs == 1 else None
    m = re.search(r"k_pcg_(c1|r1|c2|init)w?<(double|float)(?:, (\d+))?(?:, (\d+))?(?:, (\d+|true|false))?", demangled)
    if not m:
        return None
    fam, typ = m.group(1), m.group(2)   # k_pcg_r1w, k_pcg_c1w, k_pcg_c2w: the wave-private passes
    mode = m.group(5)
    if fam == "c1" and mode not in (None, "0"):
        return None           # initial-residual copy mode, not the loop pass
    if fam == "c2" and mode not in (None, "3"):
        return None           # residual / store modes, not the loop pass
    return "pcg_" + fam, ("f64" if typ == "double" else "f32")


def kernel_stats(db_path: str):
    db = sqlite3.connect(db_path)
    rows = db.execute("select name, end - start from kernels").fetchall()
    agg = collections.defaultdict(list)
    for name, dur in rows:
        agg[name].append(dur)
    dem = demangle(agg)
    out = []
    for name, durs in agg.items():
        # only the Krylov loop passes return early; other kernels' durations vary
        # with their arguments (field counts), not with convergence
        loop = re.search(r"k_pcg_(c1|r1|c2)w?<", dem[name]) is not None
        full, early = split_launches(durs) if loop else (durs, [])
        out.append({"name": dem[name], "calls": len(durs), "total_ns": sum(durs),
                    "avg_ns": sum(durs) / len(durs), "min_ns": min(durs), "max_ns": max(durs),
                    "early": len(early), "avg_full_ns": sum(full) / len(full) if full else 0.0})
    out.sort(key=lambda r: -r["total_ns"])
    return out


def kernel_summary_md(db_path: str, command: str, title: str, top: int = 25) -> str:
    st = kernel_stats(db_path)
    total = sum(r["total_ns"] for r in st)
    lines = [f"# {title}", "", "Command:", "", "```", command, "```", "",
             f"Kernels: {len(st)} distinct, total GPU kernel time {total / 1e6:.2f} ms.", "",
             "Early exits (Krylov loop passes only): launches shorter than half the kernel's median (a",
             "pass launched after its solve has converged returns at once); `avg us (full)` averages the",
             "other launches, the figure the bench's roofline prices with the bytes of a full pass.", "",
             "| kernel | calls | total ms | avg us | min us | max us | share | early exits | avg us (full) |",
             "|---|---|---|---|---|---|---|---|---|"]
    for r in st[:top]:
        nm = r["name"].split("(")[0].replace("|", "/")
        lines.append(f"| `{nm}` | {r['calls']} | {r['total_ns'] / 1e6:.3f} | {r['avg_ns'] / 1e3:.2f} | "
                     f"{r['min_ns'] / 1e3:.2f} | {r['max_ns'] / 1e3:.2f} | {100 * r['total_ns'] / total:.1f}% | "
                     f"{r['early']} | {r['avg_full_ns'] / 1e3:.2f} |")
    return "\n".join(lines) + "\n"


def counter_means(db_path: str, counter: str):
    db = sqlite3.connect(db_path)
    rows = db.execute("select kernel_name, value, grid_size from counters_collection where counter_name = ?",
                      (counter,)).fetchall()
    return rows


def traffic(fetch_db: str, write_db: str, calib_bytes: int, n: int = 0):
    """HBM bytes per launch of each PCG loop family and precision (and of the 2D
    right-hand-side passes when n, the grid side, is given), from FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch) scaled so that the reference copy of
    calib_bytes reads and writes exactly calib_bytes."""
    fr = counter_means(fetch_db, "FETCH_SIZE")
    wr = counter_means(write_db, "WRITE_SIZE")
    kib = calib_bytes / 1024.0
    # reference copy: the copy dispatch whose WRITE_SIZE is closest to the copied size
    cw = [v for n, v, g in wr if "copy" in n.lower()]
    cf = [v for n, v, g in fr if "copy" in n.lower()]
    if not cw or not cf:
        raise RuntimeError("reference copy kernel not found in the counter runs")
    w_ref = min(cw, key=lambda v: abs(v - kib))
    f_ref = max(cf)
    scale_w = kib / w_ref
    scale_f = kib / f_ref
    dem = demangle({n for n, _, _ in fr} | {n for n, _, _ in wr})
    acc = collections.defaultdict(lambda: {"fetch": [], "write": []})
    for nm, v, g in fr:
        fam = kernel_family(dem[nm], g, n)
        if fam:
            acc[fam]["fetch"].append(v)
    for nm, v, g in wr:
        fam = kernel_family(dem[nm], g, n)
        if fam:
            acc[fam]["write"].append(v)
    out = {"scale_fetch": scale_f, "scale_write": scale_w, "reference_copy_bytes": calib_bytes,
           "reference_fetch_kib": f_ref, "reference_write_kib": w_ref, "kernels": {},
           "note": "dispatches that returned at once (the solve had already converged) are excluded"}

    def working(vals):
        top = max(vals)
        return [v for v in vals if v >= 0.5 * top]

    for (fam, prec), d in acc.items():
        if not d["fetch"] or not d["write"]:
            continue
        fv, wv = working(d["fetch"]), working(d["write"])
        f = sum(fv) / len(fv) * scale_f * 1024.0
        w = sum(wv) / len(wv) * scale_w * 1024.0
        out["kernels"].setdefault(prec, {})[fam] = {"fetch_bytes": f, "write_bytes": w,
                                                    "hbm_bytes_per_launch": f + w,
                                                    "dispatches": len(fv)}
    return out


def traffic_by_kernel(fetch_db: str, write_db: str, calib_bytes: int, pattern: str):
    """HBM bytes per dispatch of every kernel whose demangled name matches
    `pattern`, per launch shape (grid size), scaled by the reference copy as in
    traffic()."""
    fr = counter_means(fetch_db, "FETCH_SIZE")
    wr = counter_means(write_db, "WRITE_SIZE")
    kib = calib_bytes / 1024.0
    cw = [v for n, v, g in wr if "copy" in n.lower()]
    cf = [v for n, v, g in fr if "copy" in n.lower()]
    if not cw or not cf:
        raise RuntimeError("reference copy kernel not found in the counter runs")
    scale_w = kib / min(cw, key=lambda v: abs(v - kib))
    scale_f = kib / max(cf)
    dem = demangle({n for n, _, _ in fr} | {n for n, _, _ in wr})
    acc = collections.defaultdict(lambda: {"fetch": [], "write": []})
    for rows, key in ((fr, "fetch"), (wr, "write")):
        for n, v, g in rows:
            nm = dem[n].split("(")[0]
            if re.search(pattern, nm):
                acc[(nm, g)][key].append(v)
    out = {"scale_fetch": scale_f, "scale_write": scale_w, "reference_copy_bytes": calib_bytes, "kernels": []}
    for (nm, g), d in sorted(acc.items()):
        if not d["fetch"] or not d["write"]:
            continue
        f = sum(d["fetch"]) / len(d["fetch"]) * scale_f * 1024.0
        w = sum(d["write"]) / len(d["write"]) * scale_w * 1024.0
        out["kernels"].append({"kernel": nm, "grid_size": g, "dispatches": len(d["fetch"]),
                               "fetch_bytes": f, "write_bytes": w, "hbm_bytes_per_launch": f + w})
    return out


def split_launches(durations):
    """(full, early) launches of one kernel family: a Krylov pass launched after
    its solve has converged returns at once, so a family's durations are bimodal;
    launches shorter than half the family's median are the early exits.  (The
    median is a full launch as long as fewer than half return early, which the
    chunk sizing of the solves keeps so.)"""
    ds = sorted(durations)
    if not ds:
        return [], []
    med = ds[len(ds) // 2]
    full = [d for d in durations if d >= 0.5 * med]
    early = [d for d in durations if d < 0.5 * med]
    return full, early
