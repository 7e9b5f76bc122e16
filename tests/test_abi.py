"""The C-ABI library loads on a machine without a GPU and exports every symbol
include/sgn.h declares; host-only entry points (sizes, version) answer without
touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2506_16045_amd", "libsgn.so")
HEADER = os.path.join(ROOT, "include", "sgn.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(sgn_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libsgn.so is not built (run __graft_entry__.build())")
    import torch  # noqa: F401  (same HIP runtime as the GPU path)
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n


def test_binding_signatures_cover_the_header():
    from paper_2506_16045_amd import sgn
    assert set(sgn.header_symbols()) == set(sgn._SIGS)


def test_version_and_workspace_sizes(lib):
    from paper_2506_16045_amd import sgn
    from paper_2506_16045_amd import inputs as I
    assert "gfx950" in sgn.version()
    for g in (I.grid1d(256, 80.0), I.grid1d(16384, 1.0), I.grid2d(1024, 1024, 200.0, 200.0), I.grid2d(8, 4, 1.0, 1.0)):
        a = sgn.workspace_bytes(g, sgn.FP64)
        b = sgn.workspace_bytes(g, sgn.MIXED)
        assert a > 0 and b >= a
        assert sgn.state_workspace_bytes(g) > 0
    # 2D 1024^2: about 20 spectral and 17 physical FP64 fields for the right-hand side
    big = sgn.workspace_bytes(I.grid2d(1024, 1024, 1.0, 1.0), sgn.MIXED)
    assert 100e6 < big < 1e9


def test_batch_workspace_sizes(lib):
    """Batched solves and RK4 runs: a workspace grows with the systems it holds
    (a run holds about 40 doubles per point), and an unsupported size gives 0."""
    from paper_2506_16045_amd import sgn
    for fn in (sgn._lib.sgn_batch_workspace_bytes, sgn._lib.sgn_batch_step_workspace_bytes):
        for prec in (sgn.FP64, sgn.MIXED):
            one = (ctypes.c_int32 * 1)(8192)
            many = (ctypes.c_int32 * 3)(256, 8192, 2)
            a, b = fn(1, one, prec), fn(3, many, prec)
            assert 0 < a < b
            assert fn(1, (ctypes.c_int32 * 1)(16384), prec) == 0
            assert fn(1, (ctypes.c_int32 * 1)(384), prec) == 0
    step = sgn._lib.sgn_batch_step_workspace_bytes(1, (ctypes.c_int32 * 1)(8192), sgn.MIXED)
    assert 30 * 8 * 8192 < step < 50 * 8 * 8192


@pytest.mark.parametrize("dim,nx,ny", [(1, 3, 1), (1, 32768, 1), (2, 64, 1), (2, 8192, 8), (2, 64, 2048), (3, 8, 8), (1, 0, 1)])
def test_unsupported_grids_report_zero_workspace(dim, nx, ny):
    from paper_2506_16045_amd import sgn
    g = sgn.Grid(dim, nx, ny, 1.0, 1.0)
    assert sgn._lib.sgn_workspace_bytes(ctypes.byref(g), 0) == 0


def test_binding_refuses_to_load_without_the_library(tmp_path):
    """No CPU fallback: with the library absent, importing the binding raises."""
    import subprocess
    import sys
    env = dict(os.environ, SGN_LIB=str(tmp_path / "absent" / "libsgn.so"))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "try:\n    import paper_2506_16045_amd.sgn\nexcept ImportError as e:\n"
            "    print('refused:', e); sys.exit(0)\nsys.exit(3)\n") % ROOT
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "no CPU fallback" in r.stdout


def test_product_sources_never_reach_the_oracle():
    """The package and the C sources neither import nor include anything under oracle/."""
    pkg = os.path.join(ROOT, "paper_2506_16045_amd")
    pat = re.compile(r"^\s*(from\s+oracle\b|import\s+oracle\b|from\s+\.\.oracle\b|#\s*include\s*[<\"][^>\"]*oracle)",
                     re.M)
    seen = 0
    for base, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                seen += 1
                text = open(os.path.join(base, f)).read()
                assert not pat.search(text), os.path.join(base, f)
                assert "importlib" not in text or "oracle" not in text, os.path.join(base, f)
    assert seen >= 8


def test_binding_constants_match_the_header():
    """Every enumerator include/sgn.h gives a value has the same value in the binding
    (SGN_X in the header is X in paper_2506_16045_amd.sgn)."""
    import paper_2506_16045_amd.sgn as S
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    pairs = re.findall(r"\bSGN_([A-Z0-9_]+)\s*=\s*(-?\d+)", text)
    assert len(pairs) >= 20
    checked = 0
    for name, val in pairs:
        if hasattr(S, name):
            assert getattr(S, name) == int(val), name
            checked += 1
    for name in ("OK", "EINVAL", "EDOMAIN", "ENOCONV", "ENOMEM", "EDEVICE", "EUNSUPPORTED",
                 "PCG", "GMRES", "FP64", "MIXED", "BC_PERIODIC", "BC_WALLS",
                 "COEFF_OPTIMAL", "COEFF_REPLACEMENT", "GUESS_PREVIOUS", "GUESS_EXTRAPOLATE"):
        assert hasattr(S, name), name
    assert checked >= 17
    assert {v: k for k, v in S.STATUS_NAMES.items()} == {
        "SGN_" + n: int(v) for n, v in pairs if n in ("OK", "EINVAL", "EDOMAIN", "ENOCONV", "ENOMEM",
                                                      "EDEVICE", "EUNSUPPORTED")}
    # the per-kernel timing families are reported in the order of sgn_kernel_kind
    kinds = {n[len("KERNEL_"):].lower(): int(v) for n, v in pairs if n.startswith("KERNEL_")}
    n_kinds = kinds.pop("kinds")
    assert len(S.Context.KERNEL_KINDS) == n_kinds
    assert {k: i for i, k in enumerate(S.Context.KERNEL_KINDS)} == kinds


def test_linimp3_choice_equals_the_oracles():
    """The library's joint choice of (r, theta) for the third-order linearly
    implicit scheme (host only) equals the oracle's, written independently."""
    from oracle import linimp as L
    from paper_2506_16045_amd import sgn
    for kappa in (1.0, 1.728, 5.0, 17.6, 266.5, 338.9, 1e4):
        for margin in (1.0, 1.1, 1.5):
            r, th = sgn.linimp3_choose(kappa, margin)
            r_o, th_o = L.choose_sbdf3r(kappa, margin)
            assert abs(r - r_o) <= 1e-12 and abs(th - th_o) <= 1e-12 * th_o, (kappa, margin)
    with pytest.raises(sgn.SgnError):
        sgn.linimp3_choose(0.5)


def test_launch_split_separates_early_exits():
    """The bench prices full Krylov launches only: a family's bimodal durations
    split at half the median (early exits of converged solves below it)."""
    from paper_2506_16045_amd import profiling
    full, early = profiling.split_launches([21.0, 4.1, 22.5, 20.8, 3.9, 24.0, 21.7])
    assert sorted(early) == [3.9, 4.1] and len(full) == 5
    assert profiling.split_launches([]) == ([], [])
    full, early = profiling.split_launches([10.0, 10.5, 9.8])
    assert early == [] and len(full) == 3


def test_kernel_family_names_the_right_hand_side_launches():
    """The rocprof summaries map the right-hand side's column launches by their
    job count: three jobs (derivatives) and one (flux) at 1024^2."""
    from paper_2506_16045_amd import profiling
    name = "void sgn::k_cols_lin_jobs<double, 4, 3, 3>(sgn::ColGeom, ...)"
    cols = 256 * 513
    assert profiling.kernel_family(name, 3 * cols, 1024) == ("rhs_cols", "f64")
    assert profiling.kernel_family(name, cols, 1024) == ("rhs_flux", "f64")
    assert profiling.kernel_family("void sgn::k_pcg_r1w<float, 2>(int, ...)") == ("pcg_r1", "f32")
