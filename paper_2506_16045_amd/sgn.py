"""Thin Python binding of libsgn.so (include/sgn.h).

Argument marshalling only: PyTorch tensors on the GPU are passed to the C ABI as
device pointers, the current PyTorch HIP stream is passed as the library's
stream, and workspaces are PyTorch allocations owned by a Context.  Every step
of the computation runs in the library's HIP kernels; there is no CPU fallback.
If libsgn.so is missing or cannot be loaded, importing this module raises.

Field layout (as in the C header): scalar fields (nx,) in 1D and (ny, nx) in 2D,
vector fields (d, nx) / (d, ny, nx), all float64 and contiguous.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

import torch  # loaded first so libsgn.so binds to the same HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SGN_LIB", os.path.join(_HERE, "libsgn.so"))
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "sgn.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libsgn.so not found at {LIB_PATH}; build it with "
                      "`python -m paper_2506_16045_amd.build` (no CPU fallback exists)")
_lib = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_GLOBAL)

# ---- status codes and enums -------------------------------------------------
OK, EINVAL, EDOMAIN, ENOCONV, ENOMEM, EDEVICE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "SGN_OK", -1: "SGN_EINVAL", -2: "SGN_EDOMAIN", -3: "SGN_ENOCONV",
                -4: "SGN_ENOMEM", -5: "SGN_EDEVICE", -6: "SGN_EUNSUPPORTED"}
PCG, GMRES = 0, 1
FP64, MIXED = 0, 1
COEFF_OPTIMAL, COEFF_REPLACEMENT = 0, 1
BC_PERIODIC, BC_WALLS = 0, 1
GUESS_PREVIOUS, GUESS_EXTRAPOLATE = 0, 1


class SgnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("Lx", ctypes.c_double), ("Ly", ctypes.c_double), ("bc", ctypes.c_int32)]


class Coeffs(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("alpha", ctypes.c_double),
                ("kappa_ub", ctypes.c_double), ("flat", ctypes.c_int32)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("precision", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("x0_is_guess", ctypes.c_int32),
                ("gmres_restart", ctypes.c_int32), ("inner_tol", ctypes.c_double),
                ("max_outer", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("coeff_kind", ctypes.c_int32), ("guess", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("outer_iters", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("relres", ctypes.c_double), ("coeffs", Coeffs)]


class StepInfo(ctypes.Structure):
    _fields_ = [("solves", ctypes.c_int64), ("iters", ctypes.c_int64), ("max_iters", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("t", ctypes.c_double), ("steps_done", ctypes.c_int64)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("lanes", ctypes.c_int32), ("max_batch", ctypes.c_int32)]


REQ_SOLVE, REQ_STEP_RK4 = 0, 1


class Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("grid", Grid), ("opts", SolveOpts),
                ("h_eta", ctypes.c_void_p), ("h_grad_h", ctypes.c_void_p), ("h_rhs", ctypes.c_void_p),
                ("h_h", ctypes.c_void_p), ("h_u0", ctypes.c_void_p), ("dt", ctypes.c_double),
                ("nsteps", ctypes.c_int32), ("h_eta_out", ctypes.c_void_p), ("h_u_out", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("done", ctypes.c_int32), ("status", ctypes.c_int32), ("iters", ctypes.c_int64),
                ("solves", ctypes.c_int64), ("relres", ctypes.c_double), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_start", ctypes.c_double), ("t_done", ctypes.c_double),
                ("batched", ctypes.c_int32), ("batch_size", ctypes.c_int32)]


_P = ctypes.c_void_p
_I = ctypes.c_int32
_D = ctypes.c_double
_S = ctypes.c_int
_SIGS = {
    "sgn_create": (_S, [ctypes.POINTER(_P), ctypes.c_int, _P]),
    "sgn_destroy": (None, [_P]),
    "sgn_set_stream": (_S, [_P, _P]),
    "sgn_last_error": (ctypes.c_char_p, [_P]),
    "sgn_version": (ctypes.c_char_p, []),
    "sgn_profile_begin": (_S, [_P]),
    "sgn_profile_end": (_S, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double), _I]),
    "sgn_profile_launches": (_S, [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_float),
                                  ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    "sgn_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Grid), _I]),
    "sgn_gmres_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Grid), _I]),
    "sgn_bathy_prepare": (_S, [_P, ctypes.POINTER(Grid), _P, _P, ctypes.POINTER(_I), _P]),
    "sgn_precond_coeffs": (_S, [_P, ctypes.POINTER(Grid), _P, _P, _I, _I, ctypes.POINTER(Coeffs), _P]),
    "sgn_apply_constraint": (_S, [_P, ctypes.POINTER(Grid), _P, _P, _P, _P, _P]),
    "sgn_precond_solve": (_S, [_P, ctypes.POINTER(Grid), ctypes.POINTER(Coeffs), _P, _P, _P]),
    "sgn_krylov_solve": (_S, [_P, ctypes.POINTER(Grid), _P, _P, _P, _P, ctypes.POINTER(Coeffs),
                              ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), _P]),
    "sgn_krylov_solve_noalloc": (_S, [_P, ctypes.POINTER(Grid), _P, _P, _P, _P, ctypes.POINTER(Coeffs),
                                      ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo)]),
    "sgn_rhs": (_S, [_P, ctypes.POINTER(Grid), _P, _P, _P, _P, _P, _P, _P]),
    "sgn_dealias_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Grid)]),
    "sgn_rhs_dealiased": (_S, [_P, ctypes.POINTER(Grid), _P, _P, _P, _P, _P, _P, _P]),
    "sgn_state_set_dealias": (_S, [_P, _P, _P]),
    "sgn_batch_workspace_bytes": (ctypes.c_size_t, [_I, ctypes.POINTER(_I), _I]),
    "sgn_request_footprint": (ctypes.c_size_t, [ctypes.POINTER(Request)]),
    "sgn_server_create": (_S, [ctypes.POINTER(_P), ctypes.c_int, ctypes.POINTER(ServerOpts)]),
    "sgn_server_destroy": (None, [_P]),
    "sgn_server_submit": (_S, [_P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]),
    "sgn_server_poll": (_S, [_P, ctypes.c_uint64, ctypes.POINTER(Result)]),
    "sgn_server_wait": (_S, [_P, ctypes.c_uint64, _D, ctypes.POINTER(Result)]),
    "sgn_server_stats": (_S, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                              ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_size_t),
                              ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
    "sgn_batch_solve": (_S, [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_D), _P, _P, _P, _P,
                             ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), _P]),
    "sgn_batch_step_workspace_bytes": (ctypes.c_size_t, [_I, ctypes.POINTER(_I), _I]),
    "sgn_batch_step_rk4": (_S, [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_D), ctypes.POINTER(_D),
                                ctypes.POINTER(_I), _P, _P, _P, ctypes.POINTER(SolveOpts), ctypes.POINTER(StepInfo),
                                ctypes.POINTER(_S), _P]),
    "sgn_state_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(Grid), _I]),
    "sgn_state_create": (_S, [_P, ctypes.POINTER(Grid), _P, _P, _I, _P, _P, _P, _P, _P, ctypes.POINTER(_P)]),
    "sgn_state_destroy": (None, [_P]),
    "sgn_step_rk4": (_S, [_P, _P, _D, _I, ctypes.POINTER(SolveOpts), ctypes.POINTER(StepInfo)]),
    "sgn_step_ab": (_S, [_P, _P, _I, _D, _I, ctypes.POINTER(SolveOpts), ctypes.POINTER(StepInfo)]),
    "sgn_step_linimp": (_S, [_P, _P, _D, _I, ctypes.POINTER(Coeffs), ctypes.POINTER(SolveOpts),
                             ctypes.POINTER(StepInfo)]),
    "sgn_step_linimp3": (_S, [_P, _P, _D, _D, _D, _I, ctypes.POINTER(Coeffs), ctypes.POINTER(SolveOpts),
                              ctypes.POINTER(StepInfo)]),
    "sgn_linimp3_choose": (_S, [_D, _D, ctypes.POINTER(_D), ctypes.POINTER(_D)]),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


def header_symbols(path: str = HEADER_PATH):
    """Names of the functions declared in include/sgn.h."""
    with open(path) as fh:
        text = fh.read()
    return sorted(set(re.findall(r"\b(sgn_[a-z0-9_]+)\s*\(", text)))


def version() -> str:
    return _lib.sgn_version().decode()


def make_grid(g) -> Grid:
    """Grid from an object with d, nx, ny, Lx, Ly (paper_2506_16045_amd.inputs.Grid)."""
    return Grid(int(g.d), int(g.nx), int(g.ny if g.d == 2 else 1), float(g.Lx), float(g.Ly if g.d == 2 else 1.0),
                int(getattr(g, "bc", BC_PERIODIC)))


def workspace_bytes(g, precision: int = FP64) -> int:
    return int(_lib.sgn_workspace_bytes(ctypes.byref(make_grid(g)), precision))


def gmres_workspace_bytes(g, restart: int = 30) -> int:
    return int(_lib.sgn_gmres_workspace_bytes(ctypes.byref(make_grid(g)), int(restart)))


def batch_workspace_bytes(sizes, precision: int = FP64) -> int:
    n = (_I * len(sizes))(*[int(v) for v in sizes])
    return int(_lib.sgn_batch_workspace_bytes(len(sizes), n, precision))


def dealias_workspace_bytes(g) -> int:
    """Workspace of the de-aliased right-hand side; 0 if the grid is too large to pad."""
    return int(_lib.sgn_dealias_workspace_bytes(ctypes.byref(make_grid(g))))


def state_workspace_bytes(g, precision: int = FP64) -> int:
    return int(_lib.sgn_state_workspace_bytes(ctypes.byref(make_grid(g)), precision))


def solve_opts(tol=1e-12, max_iter=1000, precision=FP64, x0_is_guess=False, inner_tol=1e-5,
               max_outer=20, check_every=8, coeff_kind=COEFF_OPTIMAL, method=PCG, gmres_restart=30,
               guess=GUESS_EXTRAPOLATE):
    """Solver options; guess may also be given as 'previous' or 'extrapolate'."""
    if isinstance(guess, str):
        guess = {"previous": GUESS_PREVIOUS, "extrapolate": GUESS_EXTRAPOLATE}[guess]
    return SolveOpts(method, precision, tol, max_iter, int(bool(x0_is_guess)), gmres_restart,
                     inner_tol, max_outer, check_every, coeff_kind, guess)


def _ptr(t: torch.Tensor, shape, name: str):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor (got {t.device})")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64 (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _scalar_shape(g):
    return (g.nx,) if g.d == 1 else (g.ny, g.nx)


def _vector_shape(g):
    return (g.d,) + _scalar_shape(g)


@dataclass
class SolveResult:
    iters: int
    outer_iters: int
    converged: bool
    relres: float
    sigma: float
    alpha: float
    kappa_ub: float
    flat: bool


class _BatchResults:
    """Per-system results of a batched solve, converted from the C records when read."""

    def __init__(self, infos, n):
        self._infos = infos
        self._n = n

    def __len__(self):
        return self._n

    def __getitem__(self, i):
        if isinstance(i, slice):
            return [self[k] for k in range(*i.indices(self._n))]
        if i < 0:
            i += self._n
        if not 0 <= i < self._n:
            raise IndexError(i)
        r = self._infos[i]
        return SolveResult(r.iters, r.outer_iters, bool(r.converged), r.relres, r.coeffs.sigma, r.coeffs.alpha,
                           r.coeffs.kappa_ub, bool(r.coeffs.flat))

    def __iter__(self):
        return (self[k] for k in range(self._n))

    def __eq__(self, other):
        if isinstance(other, (list, tuple, _BatchResults)):
            return list(self) == list(other)
        return NotImplemented

    def __repr__(self):
        return repr(list(self))


class Context:
    """An sgn_ctx bound to a GPU and to the PyTorch stream current at each call."""

    def __init__(self, device: int | torch.device | None = None):
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else
                           (device.index if isinstance(device, torch.device) else int(device)))
        self.device = dev
        h = _P()
        with torch.cuda.device(dev):
            st = _lib.sgn_create(ctypes.byref(h), dev.index, _P(torch.cuda.current_stream(dev).cuda_stream))
        if st != OK:
            raise SgnError(st, "sgn_create failed")
        self._h = h
        self._ws = {}
        self._gmres_ws = {}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.sgn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ---------------------------------------------------------------
    def _sync_stream(self):
        _lib.sgn_set_stream(self._h, _P(torch.cuda.current_stream(self.device).cuda_stream))

    def _check(self, st: int):
        if st != OK:
            raise SgnError(st, _lib.sgn_last_error(self._h).decode())

    def workspace(self, g, precision=FP64) -> torch.Tensor:
        key = (g.d, g.nx, g.ny if g.d == 2 else 1, int(getattr(g, "bc", BC_PERIODIC)), max(precision, MIXED))
        nb = workspace_bytes(g, MIXED)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nb:
            ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        return ws

    # -- kernel timing ---------------------------------------------------------
    KERNEL_KINDS = ("pcg_c1", "pcg_r1", "pcg_c2", "pcg_init", "rows", "cols",
                    "pcg_c1_f32", "pcg_r1_f32", "pcg_c2_f32", "pcg_init_f32", "batch",
                    "rhs_rows_fwd", "rhs_cols", "rhs_rows_inv", "rhs_flux", "batch_step", "wall_order")

    def profile_begin(self):
        self._sync_stream()
        self._check(_lib.sgn_profile_begin(self._h))

    def profile_end(self):
        """{kernel family: (launches, total milliseconds)} since profile_begin."""
        n = len(self.KERNEL_KINDS)
        cnt = (ctypes.c_int64 * n)()
        ms = (ctypes.c_double * n)()
        self._check(_lib.sgn_profile_end(self._h, cnt, ms, n))
        return {k: (int(cnt[i]), float(ms[i])) for i, k in enumerate(self.KERNEL_KINDS)}

    def profile_launches(self):
        """{kernel family: [milliseconds of each launch]} of the last profile, in launch
        order (sgn_profile_launches)."""
        count = ctypes.c_int64(0)
        self._check(_lib.sgn_profile_launches(self._h, None, None, 0, ctypes.byref(count)))
        cap = count.value
        kinds = (ctypes.c_int32 * max(cap, 1))()
        ms = (ctypes.c_float * max(cap, 1))()
        self._check(_lib.sgn_profile_launches(self._h, kinds, ms, cap, ctypes.byref(count)))
        out = {k: [] for k in self.KERNEL_KINDS}
        for i in range(min(cap, count.value)):
            if 0 <= kinds[i] < len(self.KERNEL_KINDS):
                out[self.KERNEL_KINDS[kinds[i]]].append(float(ms[i]))
        return out

    # -- entry points ----------------------------------------------------------
    def bathy_prepare(self, g, h: torch.Tensor):
        """grad h and the flat flag (sgn_bathy_prepare)."""
        self._sync_stream()
        grid = make_grid(g)
        gh = torch.empty(_vector_shape(g), dtype=torch.float64, device=self.device)
        flat = _I(0)
        self._check(_lib.sgn_bathy_prepare(self._h, ctypes.byref(grid), _ptr(h, _scalar_shape(g), "h"),
                                           _ptr(gh, _vector_shape(g), "grad_h"), ctypes.byref(flat),
                                           _P(self.workspace(g).data_ptr())))
        return gh, bool(flat.value)

    def precond_coeffs(self, g, eta, grad_h, flat: bool, kind: int = COEFF_OPTIMAL) -> Coeffs:
        self._sync_stream()
        grid = make_grid(g)
        c = Coeffs()
        self._check(_lib.sgn_precond_coeffs(self._h, ctypes.byref(grid), _ptr(eta, _scalar_shape(g), "eta"),
                                            _ptr(grad_h, _vector_shape(g), "grad_h"), int(bool(flat)), kind,
                                            ctypes.byref(c), _P(self.workspace(g).data_ptr())))
        return c

    def apply_constraint(self, g, eta, grad_h, u, out=None):
        """out = G_{eta,h} u (sgn_apply_constraint)."""
        self._sync_stream()
        grid = make_grid(g)
        if out is None:
            out = torch.empty(_vector_shape(g), dtype=torch.float64, device=self.device)
        self._check(_lib.sgn_apply_constraint(self._h, ctypes.byref(grid), _ptr(eta, _scalar_shape(g), "eta"),
                                              _ptr(grad_h, _vector_shape(g), "grad_h"),
                                              _ptr(u, _vector_shape(g), "u"), _ptr(out, _vector_shape(g), "out"),
                                              _P(self.workspace(g).data_ptr())))
        return out

    def precond_solve(self, g, sigma: float, alpha: float, rhs, out=None):
        """out = A^{-1} rhs (sgn_precond_solve)."""
        self._sync_stream()
        grid = make_grid(g)
        c = Coeffs(sigma, alpha, 0.0, 0)
        if out is None:
            out = torch.empty(_vector_shape(g), dtype=torch.float64, device=self.device)
        self._check(_lib.sgn_precond_solve(self._h, ctypes.byref(grid), ctypes.byref(c),
                                           _ptr(rhs, _vector_shape(g), "rhs"), _ptr(out, _vector_shape(g), "out"),
                                           _P(self.workspace(g).data_ptr())))
        return out

    def krylov_solve(self, g, eta, grad_h, rhs, u=None, coeffs: Coeffs | None = None, opts: SolveOpts | None = None,
                     raise_on_noconv: bool = True):
        """Solve G u = rhs (sgn_krylov_solve).  Returns (u, SolveResult)."""
        self._sync_stream()
        grid = make_grid(g)
        o = opts if opts is not None else solve_opts()
        if u is None:
            u = torch.zeros(_vector_shape(g), dtype=torch.float64, device=self.device)
        info = SolveInfo()
        if o.method == GMRES:
            # 0 for an unsupported grid or restart: the library then rejects the call before any work
            nb = max(gmres_workspace_bytes(g, o.gmres_restart), 256)
            ws = self._gmres_ws.get(nb)
            if ws is None:
                self._gmres_ws.clear()
                ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
                self._gmres_ws[nb] = ws
        else:
            ws = self.workspace(g, o.precision)
        st = _lib.sgn_krylov_solve(self._h, ctypes.byref(grid), _ptr(eta, _scalar_shape(g), "eta"),
                                   _ptr(grad_h, _vector_shape(g), "grad_h"), _ptr(rhs, _vector_shape(g), "rhs"),
                                   _ptr(u, _vector_shape(g), "u"), ctypes.byref(coeffs) if coeffs else None,
                                   ctypes.byref(o), ctypes.byref(info), _P(ws.data_ptr()))
        res = SolveResult(info.iters, info.outer_iters, bool(info.converged), info.relres, info.coeffs.sigma,
                          info.coeffs.alpha, info.coeffs.kappa_ub, bool(info.coeffs.flat))
        if st == ENOCONV and not raise_on_noconv:
            return u, res
        self._check(st)
        return u, res

    def krylov_solve_noalloc(self, g, eta, grad_h, rhs, u=None, coeffs: Coeffs | None = None,
                             opts: SolveOpts | None = None, raise_on_noconv: bool = True):
        """Solve G u = rhs with the library's static scratch as workspace
        (sgn_krylov_solve_noalloc).  Returns (u, SolveResult)."""
        self._sync_stream()
        grid = make_grid(g)
        o = opts if opts is not None else solve_opts()
        if u is None:
            u = torch.zeros(_vector_shape(g), dtype=torch.float64, device=self.device)
        info = SolveInfo()
        st = _lib.sgn_krylov_solve_noalloc(self._h, ctypes.byref(grid), _ptr(eta, _scalar_shape(g), "eta"),
                                           _ptr(grad_h, _vector_shape(g), "grad_h"),
                                           _ptr(rhs, _vector_shape(g), "rhs"), _ptr(u, _vector_shape(g), "u"),
                                           ctypes.byref(coeffs) if coeffs else None, ctypes.byref(o),
                                           ctypes.byref(info))
        res = SolveResult(info.iters, info.outer_iters, bool(info.converged), info.relres, info.coeffs.sigma,
                          info.coeffs.alpha, info.coeffs.kappa_ub, bool(info.coeffs.flat))
        if st == ENOCONV and not raise_on_noconv:
            return u, res
        self._check(st)
        return u, res

    def batch_solve(self, sizes, periods, eta, grad_h, rhs, u=None, opts: SolveOpts | None = None,
                    raise_on_error: bool = True):
        """Independent 1D solves in one launch (sgn_batch_solve).  The fields are
        packed 1D float64 tensors (system i at offset sum(sizes[:i])).  Returns
        (u, results, status); results is a sequence of SolveResult, one per system,
        each built when it is read."""
        import numpy as np
        self._sync_stream()
        n_np = np.ascontiguousarray(sizes, dtype=np.int32)
        L_np = np.ascontiguousarray(periods, dtype=np.float64)
        nitems = int(n_np.shape[0])
        total = int(n_np.sum())
        if L_np.shape[0] != nitems:
            raise ValueError("sizes and periods differ in length")
        o = opts if opts is not None else solve_opts()
        if u is None:
            u = torch.zeros(total, dtype=torch.float64, device=self.device)
        n = n_np.ctypes.data_as(ctypes.POINTER(_I))
        L = L_np.ctypes.data_as(ctypes.POINTER(_D))
        infos = (SolveInfo * max(nitems, 1))()
        nb = int(_lib.sgn_batch_workspace_bytes(nitems, n, o.precision))
        if nitems and nb == 0:
            raise SgnError(EUNSUPPORTED, "batch sizes must be powers of two in [2, 8192]")
        ws = self._ws.get("batch")
        if ws is None or ws.numel() < nb:
            ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=self.device)
            self._ws["batch"] = ws
        st = _lib.sgn_batch_solve(self._h, nitems, n, L, _ptr(eta, (total,), "eta"), _ptr(grad_h, (total,), "grad_h"),
                                  _ptr(rhs, (total,), "rhs"), _ptr(u, (total,), "u"), ctypes.byref(o), infos,
                                  _P(ws.data_ptr()))
        if raise_on_error:
            self._check(st)
        return u, _BatchResults(infos, nitems), st

    def batch_step_rk4(self, sizes, periods, dts, nsteps, h, eta, u, opts: SolveOpts | None = None,
                       raise_on_error: bool = True):
        """Independent 1D RK4 runs in one launch (sgn_batch_step_rk4).  h, eta and
        u are packed 1D float64 tensors (state i at offset sum(sizes[:i])); eta
        and u are advanced in place.  dts and nsteps: one per state.  Returns
        (infos, statuses, status): a StepInfo and an sgn_status per state."""
        import numpy as np
        self._sync_stream()
        n_np = np.ascontiguousarray(sizes, dtype=np.int32)
        nitems = int(n_np.shape[0])
        L_np = np.ascontiguousarray(periods, dtype=np.float64)
        dt_np = np.ascontiguousarray(np.broadcast_to(np.asarray(dts, dtype=np.float64), (nitems,)))
        ns_np = np.ascontiguousarray(np.broadcast_to(np.asarray(nsteps, dtype=np.int32), (nitems,)))
        if L_np.shape[0] != nitems:
            raise ValueError("sizes and periods differ in length")
        total = int(n_np.sum())
        o = opts if opts is not None else solve_opts()
        n = n_np.ctypes.data_as(ctypes.POINTER(_I))
        infos = (StepInfo * max(nitems, 1))()
        stats = (_S * max(nitems, 1))()
        nb = int(_lib.sgn_batch_step_workspace_bytes(nitems, n, o.precision))
        if nitems and nb == 0:
            raise SgnError(EUNSUPPORTED, "batch sizes must be powers of two in [2, 8192]")
        ws = self._ws.get("batch_step")
        if ws is None or ws.numel() < nb:
            ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=self.device)
            self._ws["batch_step"] = ws
        st = _lib.sgn_batch_step_rk4(self._h, nitems, n, L_np.ctypes.data_as(ctypes.POINTER(_D)),
                                     dt_np.ctypes.data_as(ctypes.POINTER(_D)), ns_np.ctypes.data_as(ctypes.POINTER(_I)),
                                     _ptr(h, (total,), "h"), _ptr(eta, (total,), "eta"), _ptr(u, (total,), "u"),
                                     ctypes.byref(o), infos, stats, _P(ws.data_ptr()))
        if raise_on_error:
            self._check(st)
        return list(infos)[:nitems], [int(x) for x in stats[:nitems]], st

    def rhs(self, g, eta, h, grad_h, u, eta_t=None, U_t=None):
        """(eta_t, U_t) = f(w, p) (sgn_rhs)."""
        self._sync_stream()
        grid = make_grid(g)
        if eta_t is None:
            eta_t = torch.empty(_scalar_shape(g), dtype=torch.float64, device=self.device)
        if U_t is None:
            U_t = torch.empty(_vector_shape(g), dtype=torch.float64, device=self.device)
        self._check(_lib.sgn_rhs(self._h, ctypes.byref(grid), _ptr(eta, _scalar_shape(g), "eta"),
                                 _ptr(h, _scalar_shape(g), "h"), _ptr(grad_h, _vector_shape(g), "grad_h"),
                                 _ptr(u, _vector_shape(g), "u"), _ptr(eta_t, _scalar_shape(g), "eta_t"),
                                 _ptr(U_t, _vector_shape(g), "U_t"), _P(self.workspace(g).data_ptr())))
        return eta_t, U_t

    def rhs_dealiased(self, g, eta, h, grad_h, u, eta_t=None, U_t=None):
        """(eta_t, U_t) = f(w, p) formed on the zero-padded grid (sgn_rhs_dealiased)."""
        self._sync_stream()
        grid = make_grid(g)
        if eta_t is None:
            eta_t = torch.empty(_scalar_shape(g), dtype=torch.float64, device=self.device)
        if U_t is None:
            U_t = torch.empty(_vector_shape(g), dtype=torch.float64, device=self.device)
        # at least 256 bytes, so that an unsupported grid reaches the library's own check
        ws = torch.empty(max(dealias_workspace_bytes(g), 256), dtype=torch.uint8, device=self.device)
        self._check(_lib.sgn_rhs_dealiased(self._h, ctypes.byref(grid), _ptr(eta, _scalar_shape(g), "eta"),
                                           _ptr(h, _scalar_shape(g), "h"), _ptr(grad_h, _vector_shape(g), "grad_h"),
                                           _ptr(u, _vector_shape(g), "u"), _ptr(eta_t, _scalar_shape(g), "eta_t"),
                                           _ptr(U_t, _vector_shape(g), "U_t"), _P(ws.data_ptr())))
        return eta_t, U_t


class State:
    """A time-stepping state (sgn_state) over caller-owned eta, U, u tensors."""

    def __init__(self, ctx: Context, g, h, grad_h, flat: bool, eta, U, u):
        self.ctx = ctx
        self.g = g
        self._keep = (h, grad_h, eta, U, u)
        self.eta, self.U, self.u = eta, U, u
        self._sws = torch.empty(state_workspace_bytes(g), dtype=torch.uint8, device=ctx.device)
        self._ws = torch.empty(workspace_bytes(g, MIXED), dtype=torch.uint8, device=ctx.device)
        grid = make_grid(g)
        h_ = _P()
        ctx._sync_stream()
        ctx._check(_lib.sgn_state_create(ctx._h, ctypes.byref(grid), _ptr(h, _scalar_shape(g), "h"),
                                         _ptr(grad_h, _vector_shape(g), "grad_h"), int(bool(flat)),
                                         _ptr(eta, _scalar_shape(g), "eta"), _ptr(U, _vector_shape(g), "U"),
                                         _ptr(u, _vector_shape(g), "u"), _P(self._sws.data_ptr()),
                                         _P(self._ws.data_ptr()), ctypes.byref(h_)))
        self._h = h_

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.sgn_state_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_dealias(self, enable: bool = True):
        """Use the de-aliased right-hand side in later steps (sgn_state_set_dealias)."""
        self.ctx._sync_stream()
        if enable:
            self._dws = torch.empty(max(dealias_workspace_bytes(self.g), 256), dtype=torch.uint8,
                                    device=self.ctx.device)
            self.ctx._check(_lib.sgn_state_set_dealias(self.ctx._h, self._h, _P(self._dws.data_ptr())))
        else:
            self.ctx._check(_lib.sgn_state_set_dealias(self.ctx._h, self._h, None))
            self._dws = None

    def step_rk4(self, dt: float, nsteps: int, opts: SolveOpts | None = None) -> StepInfo:
        self.ctx._sync_stream()
        info = StepInfo()
        self.ctx._check(_lib.sgn_step_rk4(self.ctx._h, self._h, dt, nsteps,
                                          ctypes.byref(opts) if opts else None, ctypes.byref(info)))
        return info

    def step_ab(self, order: int, dt: float, nsteps: int, opts: SolveOpts | None = None) -> StepInfo:
        self.ctx._sync_stream()
        info = StepInfo()
        self.ctx._check(_lib.sgn_step_ab(self.ctx._h, self._h, order, dt, nsteps,
                                         ctypes.byref(opts) if opts else None, ctypes.byref(info)))
        return info

    def step_linimp3(self, r: float, theta: float, dt: float, nsteps: int, fixed: Coeffs | None = None,
                     opts: SolveOpts | None = None) -> StepInfo:
        self.ctx._sync_stream()
        info = StepInfo()
        self.ctx._check(_lib.sgn_step_linimp3(self.ctx._h, self._h, r, theta, dt, nsteps,
                                              ctypes.byref(fixed) if fixed else None,
                                              ctypes.byref(opts) if opts else None, ctypes.byref(info)))
        return info

    def step_linimp(self, dt: float, nsteps: int, fixed: Coeffs | None = None,
                    opts: SolveOpts | None = None) -> StepInfo:
        self.ctx._sync_stream()
        info = StepInfo()
        self.ctx._check(_lib.sgn_step_linimp(self.ctx._h, self._h, dt, nsteps,
                                             ctypes.byref(fixed) if fixed else None,
                                             ctypes.byref(opts) if opts else None, ctypes.byref(info)))
        return info


def linimp3_choose(kappa: float, margin: float = 1.1):
    """(r, theta) of the third-order linearly implicit scheme for eigenvalues of
    A^{-1} G in [1/kappa, 1] (sgn_linimp3_choose, host only)."""
    r, th = _D(), _D()
    st = _lib.sgn_linimp3_choose(float(kappa), float(margin), ctypes.byref(r), ctypes.byref(th))
    if st != OK:
        raise SgnError(st, "kappa >= 1 and margin >= 1 required")
    return r.value, th.value


# ---- served execution ------------------------------------------------------------
class Server:
    """Request server (sgn_server_*): host numpy inputs are copied at submission;
    outputs are numpy arrays returned by wait()/poll() once the request is done."""

    def __init__(self, device: int = 0, hbm_budget: int = 0, lanes: int = 3, max_batch: int = 1024):
        import numpy as np  # noqa: F401  (inputs are numpy arrays)
        self._h = _P()
        opts = ServerOpts(int(hbm_budget), int(lanes), int(max_batch))
        st = _lib.sgn_server_create(ctypes.byref(self._h), device, ctypes.byref(opts))
        if st != OK:
            raise SgnError(st, "sgn_server_create failed")
        self._out = {}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.sgn_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _arr(a, shape, name):
        import numpy as np
        a = np.ascontiguousarray(a, dtype=np.float64)
        if tuple(a.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {a.shape}, expected {tuple(shape)}")
        return a

    def _request(self, kind, g, opts):
        req = Request()
        req.kind = kind
        req.grid = make_grid(g)
        req.opts = opts if opts is not None else solve_opts()
        return req

    def solve_request(self, g, eta, grad_h, rhs, u0=None, opts: SolveOpts | None = None):
        import numpy as np
        req = self._request(REQ_SOLVE, g, opts)
        keep = [self._arr(eta, _scalar_shape(g), "eta"), self._arr(grad_h, _vector_shape(g), "grad_h"),
                self._arr(rhs, _vector_shape(g), "rhs")]
        req.h_eta, req.h_grad_h, req.h_rhs = (k.ctypes.data for k in keep)
        if u0 is not None:
            keep.append(self._arr(u0, _vector_shape(g), "u0"))
            req.h_u0 = keep[-1].ctypes.data
        u_out = np.zeros(_vector_shape(g))
        req.h_u_out = u_out.ctypes.data
        return req, keep, {"u": u_out}

    def step_request(self, g, h, eta, u0, dt: float, nsteps: int, opts: SolveOpts | None = None):
        import numpy as np
        req = self._request(REQ_STEP_RK4, g, opts)
        keep = [self._arr(h, _scalar_shape(g), "h"), self._arr(eta, _scalar_shape(g), "eta"),
                self._arr(u0, _vector_shape(g), "u0")]
        req.h_h, req.h_eta, req.h_u0 = (k.ctypes.data for k in keep)
        req.dt = float(dt)
        req.nsteps = int(nsteps)
        out = {"eta": np.zeros(_scalar_shape(g)), "u": np.zeros(_vector_shape(g))}
        req.h_eta_out = out["eta"].ctypes.data
        req.h_u_out = out["u"].ctypes.data
        return req, keep, out

    @staticmethod
    def footprint(req_tuple) -> int:
        return int(_lib.sgn_request_footprint(ctypes.byref(req_tuple[0])))

    def submit(self, req_tuple) -> int:
        req, keep, out = req_tuple
        rid = ctypes.c_uint64()
        st = _lib.sgn_server_submit(self._h, ctypes.byref(req), ctypes.byref(rid))
        if st != OK:
            raise SgnError(st, "request rejected")
        self._out[rid.value] = out       # the output arrays stay alive until the result is read
        return rid.value

    def _finish(self, rid, res: Result):
        out = self._out.pop(rid) if res.done else None
        return res, out

    def poll(self, rid: int):
        res = Result()
        st = _lib.sgn_server_poll(self._h, rid, ctypes.byref(res))
        if st != OK:
            raise SgnError(st, "unknown request")
        return self._finish(rid, res)

    def wait(self, rid: int, timeout: float = -1.0):
        res = Result()
        st = _lib.sgn_server_wait(self._h, rid, float(timeout), ctypes.byref(res))
        if st != OK:
            raise SgnError(st, "unknown request")
        return self._finish(rid, res)

    def stats(self):
        q, a, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        used, held, budget = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        _lib.sgn_server_stats(self._h, ctypes.byref(q), ctypes.byref(a), ctypes.byref(c), ctypes.byref(used),
                              ctypes.byref(held), ctypes.byref(budget))
        return {"queued": q.value, "admitted": a.value, "completed": c.value, "bytes_in_use": used.value,
                "bytes_held": held.value, "budget": budget.value}
