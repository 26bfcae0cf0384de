"""ctypes binding of libmor.so (include/mor.h).  Argument marshalling only:
every step of the solver runs in the library's HIP kernels.  Device buffers are
torch CUDA tensors (ROCm); streams are torch's current stream unless given.
The library must be built first (``python -m paper_2103_10203_amd.build``);
importing this module raises if it is missing.
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmor.so")

MOR_OK = 0
MOR_E_INVALID_ARG = 1
MOR_E_OUT_OF_MEMORY = 2
MOR_E_DEVICE = 3
MOR_E_NOT_CONVERGED = 4
MOR_E_NONFINITE = 5
MOR_E_UNSUPPORTED = 6
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "OUT_OF_MEMORY", 3: "DEVICE", 4: "NOT_CONVERGED",
                5: "NONFINITE", 6: "UNSUPPORTED"}

GAMMA_ROTATED = 0
GAMMA_CONTINUOUS = 1
PREC_FP32 = 0
PREC_BF16X3 = 1
PREC_FP64 = 2
TRANSFORM_AUTO = 0
TRANSFORM_FFT = 1
TRANSFORM_DFT = 2


class MorError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class mor_grid(ct.Structure):
    _fields_ = [("ndim", ct.c_int32), ("pad_", ct.c_int32), ("n", ct.c_int64 * 3)]


PATTERN_ADAPTED = 0
PATTERN_RADIAL = 1


class mor_plan_opts(ct.Structure):
    _fields_ = [("gamma_kind", ct.c_int32), ("pattern_kind", ct.c_int32), ("stream", ct.c_void_p),
                ("radial_lines", ct.c_int32), ("pad_", ct.c_int32)]


class mor_plan_info(ct.Structure):
    _fields_ = [("N", ct.c_int64), ("M", ct.c_int64), ("M_actual", ct.c_int64), ("n_coeff", ct.c_int64),
                ("n_columns", ct.c_int64), ("n_last", ct.c_int64), ("inclusion_count", ct.c_int64),
                ("ncomp", ct.c_int32), ("nstress", ct.c_int32), ("pattern_kind", ct.c_int32),
                ("radial_lines", ct.c_int32)]


class mor_phase(ct.Structure):
    _fields_ = [("lambda_", ct.c_double), ("mu", ct.c_double), ("sigma_y0", ct.c_double), ("H", ct.c_double),
                ("plastic", ct.c_int32), ("pad_", ct.c_int32)]


class mor_solve_opts(ct.Structure):
    _fields_ = [("max_iter", ct.c_int32), ("precision", ct.c_int32), ("transform", ct.c_int32),
                ("check_every", ct.c_int32), ("warm_start", ct.c_void_p), ("stream", ct.c_void_p),
                ("use_graph", ct.c_int32), ("schedule", ct.c_int32)]


class mor_outputs(ct.Structure):
    _fields_ = [("eff_stress", ct.POINTER(ct.c_double)), ("strain", ct.c_void_p), ("stress", ct.c_void_p),
                ("iterations", ct.POINTER(ct.c_int32)), ("residual", ct.POINTER(ct.c_double)),
                ("coeffs", ct.c_void_p)]


# Every function declared in include/mor.h, with its ctypes signature.
_SIGS = {
    "mor_plan_create": (ct.c_int, [ct.POINTER(mor_grid), ct.c_void_p, ct.c_int64, ct.POINTER(mor_plan_opts),
                                   ct.POINTER(ct.c_void_p)]),
    "mor_plan_create_batch": (ct.c_int, [ct.POINTER(mor_grid), ct.c_int64, ct.c_void_p, ct.c_void_p,
                                         ct.POINTER(mor_plan_opts), ct.c_void_p]),
    "mor_plan_get_info": (ct.c_int, [ct.c_void_p, ct.POINTER(mor_plan_info)]),
    "mor_plan_pattern": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64, ct.POINTER(ct.c_int64)]),
    "mor_plan_coeff_index": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int64]),
    "mor_plan_destroy": (ct.c_int, [ct.c_void_p]),
    "mor_solve": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.POINTER(mor_phase), ct.c_double,
                             ct.POINTER(mor_solve_opts), ct.POINTER(mor_outputs)]),
    "mor_solve_noalloc": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.POINTER(mor_phase), ct.c_double,
                                     ct.POINTER(mor_solve_opts), ct.POINTER(mor_outputs)]),
    "mor_solve_multi": (ct.c_int, [ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_void_p, ct.c_int64,
                                   ct.POINTER(mor_phase), ct.c_double, ct.POINTER(mor_solve_opts),
                                   ct.POINTER(mor_outputs)]),
    "mor_solve_path": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int32, ct.POINTER(mor_phase), ct.c_double,
                                  ct.POINTER(mor_solve_opts), ct.c_void_p, ct.POINTER(mor_outputs)]),
    "mor_solve_path_multi": (ct.c_int, [ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int32,
                                        ct.POINTER(mor_phase), ct.c_double, ct.POINTER(mor_solve_opts), ct.c_void_p,
                                        ct.POINTER(mor_outputs)]),
    "mor_compat": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64, ct.POINTER(mor_phase),
                              ct.c_void_p, ct.POINTER(mor_solve_opts), ct.POINTER(mor_outputs)]),
    "mor_stress_error": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int64,
                                    ct.c_int32, ct.c_double, ct.c_void_p, ct.c_void_p, ct.c_void_p]),
    "mor_profile_enable": (ct.c_int, [ct.c_int32]),
    "mor_profile_reset": (ct.c_int, []),
    "mor_profile_query": (ct.c_int, [ct.c_char_p, ct.POINTER(ct.c_double), ct.POINTER(ct.c_int64),
                                     ct.POINTER(ct.c_int64), ct.POINTER(ct.c_double)]),
    "mor_mlp_create": (ct.c_int, [ct.c_int32, ct.c_int32, ct.c_int32, ct.c_uint64, ct.POINTER(ct.c_void_p)]),
    "mor_mlp_destroy": (ct.c_int, [ct.c_void_p]),
    "mor_mlp_num_params": (ct.c_int, [ct.c_void_p, ct.POINTER(ct.c_int64)]),
    "mor_mlp_get_params": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int32]),
    "mor_mlp_set_params": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int32]),
    "mor_mlp_forward": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_int32, ct.c_void_p]),
    "mor_mlp_grad": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64, ct.POINTER(ct.c_double),
                                ct.c_void_p]),
    "mor_mlp_adam": (ct.c_int, [ct.c_void_p, ct.c_float, ct.c_float, ct.c_float, ct.c_float, ct.c_void_p]),
    "mor_warm_features": (ct.c_int, [ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_void_p,
                                     ct.c_void_p]),
    "mor_warm_targets": (ct.c_int, [ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_void_p,
                                    ct.c_void_p, ct.c_void_p, ct.c_void_p]),
    "mor_warm_apply": (ct.c_int, [ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_void_p,
                                  ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p]),
    "mor_tune_variants": (ct.c_int, [ct.c_int32, ct.c_int32, ct.c_int32, ct.POINTER(ct.c_int32)]),
    "mor_tune_get": (ct.c_int, [ct.c_int32, ct.c_int32, ct.c_int32, ct.POINTER(ct.c_int32)]),
    "mor_tune_set": (ct.c_int, [ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32]),
    "mor_tune_subbatch": (ct.c_int, [ct.c_int64, ct.c_int64, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int64)]),
    "mor_autotune": (ct.c_int, [ct.c_void_p, ct.c_int64, ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_void_p,
                                ct.c_double, ct.c_int32, ct.c_void_p]),
    "mor_last_error": (ct.c_char_p, []),
    "mor_version": (ct.c_char_p, []),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2103_10203_amd.build`")
    # torch ships its own HIP runtime under the same soname as /opt/rocm's.
    # Load torch first so that libmor binds to the runtime torch already
    # holds: one process must not initialise two HSA runtimes.
    import torch  # noqa: F401
    lib = ct.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def _check(status, allow=()):
    if status != MOR_OK and status not in allow:
        raise MorError(status, lib.mor_last_error().decode())
    return status


def _np_ptr(a):
    return a.ctypes.data_as(ct.c_void_p)


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    if stream is None:
        torch = _torch()
        if torch.cuda.is_available():
            return ct.c_void_p(torch.cuda.current_stream().cuda_stream)
        return ct.c_void_p(None)
    if isinstance(stream, int):
        return ct.c_void_p(stream)
    return ct.c_void_p(stream.cuda_stream)


@dataclass(frozen=True)
class Phase:
    """Isotropic phase: Lame constants, optional J2 plasticity (linear hardening)."""
    lam: float
    mu: float
    sigma_y0: float = 0.0
    H: float = 0.0
    plastic: bool = False


def _phases(phases):
    arr = (mor_phase * 2)()
    for i, p in enumerate(phases):
        arr[i] = mor_phase(float(p.lam), float(p.mu), float(p.sigma_y0), float(p.H), 1 if p.plastic else 0, 0)
    return arr


def _grid_of(shape):
    if len(shape) not in (2, 3):
        raise ValueError("phase map must be 2D or 3D")
    grid = mor_grid()
    grid.ndim = len(shape)
    for a in range(3):
        grid.n[a] = shape[a] if a < len(shape) else 1
    return grid


_plans_closed = 0  # plans destroyed so far (invalidates cached handle arrays)


class Plan:
    """Sampling pattern of one microstructure (mor_plan_create): the adapted
    pattern of M frequencies, or with radial_lines=L the fixed radial pattern
    of L lines (M is then ignored)."""

    def __init__(self, g: np.ndarray, M: int = 1, gamma_kind: int = GAMMA_ROTATED, stream=None,
                 radial_lines: int = 0, _handle=None):
        if _handle is not None:  # a plan from mor_plan_create_batch (make_plans)
            self._adopt(_handle, tuple(g))
            return
        g = np.ascontiguousarray(g, dtype=np.uint8)
        grid = _grid_of(g.shape)
        opts = _plan_opts(gamma_kind, stream, radial_lines)
        h = ct.c_void_p()
        _check(lib.mor_plan_create(ct.byref(grid), _np_ptr(g), int(M), ct.byref(opts), ct.byref(h)))
        self._adopt(h, g.shape)

    def _adopt(self, h, shape):
        self._h = h
        self.shape = tuple(shape)
        self.ndim = len(shape)
        self._info = None

    @property
    def info(self):
        """mor_plan_get_info as a dict (fetched on first use)."""
        if self._info is None:
            inf = mor_plan_info()
            _check(lib.mor_plan_get_info(self._h, ct.byref(inf)))
            self._info = {k: getattr(inf, k) for k, _ in mor_plan_info._fields_}
        return self._info

    @property
    def handle(self):
        return self._h

    @property
    def ncomp(self):
        return self.info["ncomp"]

    @property
    def nstress(self):
        return self.info["nstress"]

    @property
    def n_coeff(self):
        return self.info["n_coeff"]

    @property
    def N(self):
        return self.info["N"]

    def pattern(self):
        m = self.info["M_actual"]
        s = np.zeros(m, np.int64)
        r = np.zeros(m, np.int64)
        ma = ct.c_int64()
        _check(lib.mor_plan_pattern(self._h, _np_ptr(s), _np_ptr(r), m, ct.byref(ma)))
        return s, r

    def coeff_index(self):
        n = self.info["n_coeff"]
        out = np.zeros(n, np.int64)
        _check(lib.mor_plan_coeff_index(self._h, _np_ptr(out), n))
        return out

    def close(self):
        global _plans_closed
        if getattr(self, "_h", None):
            lib.mor_plan_destroy(self._h)
            self._h = None
            _plans_closed += 1

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _plan_opts(gamma_kind, stream, radial_lines):
    kind = PATTERN_RADIAL if radial_lines else PATTERN_ADAPTED
    return mor_plan_opts(int(gamma_kind), kind, _stream_ptr(stream), int(radial_lines), 0)


class PlanList(list):
    """The list make_plans returns.  It keeps the arrays the batched calls
    pass to the library (plan handles, grid points and coefficient counts per
    plan), built on first use and rebuilt whenever the list's members change,
    so that repeated calls on the same plans marshal them once."""

    _arrays = None


def _plan_arrays(plans):
    """(handles, N, n_coeff) of a sequence of plans: a ctypes array of the
    handles and two int64 arrays; cached on a PlanList while its members stay
    the same objects."""
    members = tuple(plans)
    cached = getattr(plans, "_arrays", None)
    # same member objects (plans define no equality: identity) and no plan
    # closed since (a closed member must fail below, not pass a stale handle)
    if cached is not None and cached[0] == _plans_closed and cached[1] == members:
        return cached[2]
    arrs = ((ct.c_void_p * len(members))(*[p.handle.value for p in members]),
            np.fromiter((p.N for p in members), np.int64, len(members)),
            np.fromiter((p.n_coeff for p in members), np.int64, len(members)))
    if isinstance(plans, PlanList):
        plans._arrays = (_plans_closed, members, arrs)
    return arrs


def _plan_sum(counts, po):
    """Sum of a per-plan count over the RVEs' plans."""
    return int(counts[po].sum()) if len(po) else 0


def make_plans(grids, M, gamma_kind: int = GAMMA_ROTATED, stream=None, radial_lines: int = 0):
    """Plans of many microstructures: one mor_plan_create_batch call for all
    maps of the same shape, so the construction runs as a few launches over
    the whole group instead of a chain of small launches per map (the maps
    are passed by pointer, not copied here).  M: one value or one per map.
    Plans come back in input order, identical to Plan(g, M) of each map."""
    grids = [np.ascontiguousarray(g, dtype=np.uint8) for g in grids]
    Ms = [int(M)] * len(grids) if np.isscalar(M) else [int(m) for m in M]
    if len(Ms) != len(grids):
        raise ValueError("one M per grid, or a single M")
    groups = {}
    for i, g in enumerate(grids):
        groups.setdefault(g.shape, []).append(i)
    out = PlanList([None] * len(grids))
    opts = _plan_opts(gamma_kind, stream, radial_lines)
    for shape, idx in groups.items():
        grid = _grid_of(shape)
        ptrs = (ct.c_void_p * len(idx))(*[grids[i].ctypes.data for i in idx])
        marr = np.array([Ms[i] for i in idx], np.int64)
        hs = (ct.c_void_p * len(idx))()
        _check(lib.mor_plan_create_batch(ct.byref(grid), len(idx), ct.cast(ptrs, ct.c_void_p), _np_ptr(marr),
                                         ct.byref(opts), ct.cast(hs, ct.c_void_p)))
        for j, i in enumerate(idx):
            out[i] = Plan(shape, 0, _handle=ct.c_void_p(hs[j]))
    return out


@dataclass
class SolveResult:
    status: int
    eff_stress: np.ndarray
    iterations: np.ndarray
    residual: np.ndarray
    strain: object = None
    stress: object = None
    coeffs: object = None


SCHED_GRID = 0
SCHED_PERSISTENT = 1


def _check_tensor(t, name, dtype, numel):
    """A device buffer handed to the library by pointer: a contiguous CUDA
    tensor of the expected dtype and exact size, else ValueError (a wrong
    size would make the kernels read or write outside it)."""
    if t is None:
        return
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.dtype != getattr(torch, dtype):
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if t.numel() != int(numel):
        raise ValueError(f"{name} must have {int(numel)} elements, got {t.numel()}")


def _opts(max_iter, check_every, warm_start, stream, precision=PREC_FP32, transform=TRANSFORM_AUTO, use_graph=0,
          schedule=SCHED_GRID):
    ws = ct.c_void_p(warm_start.data_ptr()) if warm_start is not None else ct.c_void_p(None)
    return mor_solve_opts(int(max_iter), int(precision), int(transform), int(check_every), ws,
                          _stream_ptr(stream), int(use_graph), int(schedule))


def _outputs(B, S, eff_rows, want_fields, want_coeffs, nfield_pts, C, ncoef_total):
    torch = _torch()
    eff = np.zeros((eff_rows, S), np.float64)
    its = np.zeros(B, np.int32)
    res = np.zeros(B, np.float64)
    out = mor_outputs()
    out.eff_stress = eff.ctypes.data_as(ct.POINTER(ct.c_double))
    out.iterations = its.ctypes.data_as(ct.POINTER(ct.c_int32))
    out.residual = res.ctypes.data_as(ct.POINTER(ct.c_double))
    strain = stress = coeffs = None
    if want_fields:
        strain = torch.empty(C * nfield_pts, dtype=torch.float32, device="cuda")
        stress = torch.empty(S * nfield_pts, dtype=torch.float32, device="cuda")
        out.strain = strain.data_ptr()
        out.stress = stress.data_ptr()
    if want_coeffs:
        coeffs = torch.empty(ncoef_total, dtype=torch.complex64, device="cuda")
        out.coeffs = coeffs.data_ptr()
    return out, eff, its, res, strain, stress, coeffs


def solve(plan: Plan, macro_strain, phases, tol: float, max_iter: int = 0, warm_start=None, stream=None,
          want_fields: bool = False, want_coeffs: bool = False, check_every: int = 0,
          precision: int = PREC_FP32, transform: int = TRANSFORM_AUTO, use_graph: int = 0,
          schedule: int = SCHED_GRID, allow=(MOR_E_NOT_CONVERGED,), noalloc: bool = False) -> SolveResult:
    """mor_solve for B macro strains on one plan; macro_strain [B][ncomp].
    noalloc=True calls mor_solve_noalloc (workspace from the library's fixed
    device scratch array instead of allocations)."""
    eb = np.ascontiguousarray(np.atleast_2d(macro_strain), dtype=np.float64)
    B, C = eb.shape
    if C != plan.ncomp:
        raise ValueError(f"macro strain needs {plan.ncomp} components")
    _check_tensor(warm_start, "warm_start", "complex64", B * C * plan.n_coeff)
    S = plan.nstress
    out, eff, its, res, strain, stress, coeffs = _outputs(B, S, B, want_fields, want_coeffs, B * plan.N, C,
                                                          B * C * plan.n_coeff)
    opts = _opts(max_iter, check_every, warm_start, stream, precision, transform, use_graph, schedule)
    fn = lib.mor_solve_noalloc if noalloc else lib.mor_solve
    st = _check(fn(plan.handle, _np_ptr(eb), B, _phases(phases), float(tol), ct.byref(opts), ct.byref(out)),
                allow)
    if strain is not None:
        strain = strain.view(B, C, *plan.shape)
        stress = stress.view(B, S, *plan.shape)
    if coeffs is not None:
        coeffs = coeffs.view(B, C, plan.n_coeff)
    return SolveResult(st, eff, its, res, strain, stress, coeffs)


def solve_multi(plans, plan_of, macro_strain, phases, tol: float, max_iter: int = 0, warm_start=None, stream=None,
                want_fields: bool = False, want_coeffs: bool = False, check_every: int = 0, use_graph: int = 0,
                precision: int = PREC_FP32, transform: int = TRANSFORM_AUTO, schedule: int = SCHED_GRID,
                allow=(MOR_E_NOT_CONVERGED,)) -> SolveResult:
    """mor_solve_multi: RVE b uses plans[plan_of[b]]; outputs packed per RVE."""
    eb = np.ascontiguousarray(np.atleast_2d(macro_strain), dtype=np.float64)
    B, C = eb.shape
    po = np.ascontiguousarray(plan_of, dtype=np.int64)
    if po.shape != (B,) or (B and (po.min() < 0 or po.max() >= len(plans))):
        raise ValueError("plan_of needs one index into plans per RVE")
    handles, n_pts, n_coef = _plan_arrays(plans)
    S = plans[0].nstress
    npts = _plan_sum(n_pts, po)
    ncoef = _plan_sum(n_coef, po) * C
    _check_tensor(warm_start, "warm_start", "complex64", ncoef)
    out, eff, its, res, strain, stress, coeffs = _outputs(B, S, B, want_fields, want_coeffs, npts, C, ncoef)
    opts = _opts(max_iter, check_every, warm_start, stream, precision, transform, use_graph, schedule)
    st = _check(lib.mor_solve_multi(handles, len(plans), _np_ptr(po), _np_ptr(eb), B, _phases(phases), float(tol),
                                    ct.byref(opts), ct.byref(out)), allow)
    return SolveResult(st, eff, its, res, strain, stress, coeffs)


def solve_path(plan: Plan, macro_strains, phases, tol: float, state, max_iter: int = 0, stream=None,
               want_fields: bool = False, check_every: int = 0, use_graph: int = 0,
               precision: int = PREC_FP32, transform: int = TRANSFORM_AUTO, schedule: int = SCHED_GRID,
               allow=(MOR_E_NOT_CONVERGED,), want_coeffs: bool = False) -> SolveResult:
    """mor_solve_path: macro_strains [steps][ncomp]; state: torch float32 cuda [nstate][N] (in/out).
    Fields and coefficients (want_coeffs) are those of the last step."""
    eb = np.ascontiguousarray(np.atleast_2d(macro_strains), dtype=np.float64)
    steps, C = eb.shape
    if C != plan.ncomp:
        raise ValueError(f"macro strains need {plan.ncomp} components")
    _check_tensor(state, "state", "float32", (5 if plan.ndim == 2 else 7) * plan.N)
    S = plan.nstress
    out, eff, its, res, strain, stress, coeffs = _outputs(steps, S, steps, want_fields, want_coeffs, plan.N, C,
                                                          C * plan.n_coeff)
    opts = _opts(max_iter, check_every, None, stream, precision, transform, use_graph, schedule)
    st = _check(lib.mor_solve_path(plan.handle, _np_ptr(eb), steps, _phases(phases), float(tol), ct.byref(opts),
                                   ct.c_void_p(state.data_ptr()), ct.byref(out)), allow)
    if strain is not None:
        strain = strain.view(C, *plan.shape)
        stress = stress.view(S, *plan.shape)
    if coeffs is not None:
        coeffs = coeffs.view(C, plan.n_coeff)
    return SolveResult(st, eff, its, res, strain, stress, coeffs)


def solve_path_multi(plans, plan_of, macro_strains, phases, tol: float, state, max_iter: int = 0, stream=None,
                     want_fields: bool = False, want_coeffs: bool = False, check_every: int = 0,
                     use_graph: int = 0, schedule: int = SCHED_GRID,
                     allow=(MOR_E_NOT_CONVERGED,)) -> SolveResult:
    """mor_solve_path_multi: macro_strains [B][steps][ncomp]; RVE b uses
    plans[plan_of[b]]; state: float32 CUDA tensor holding every RVE's
    [nstate][N] block (packed).  eff_stress comes back as [B][steps][6]."""
    eb = np.ascontiguousarray(macro_strains, dtype=np.float64)
    if eb.ndim != 3:
        raise ValueError("macro_strains must be [B][steps][ncomp]")
    B, steps, C = eb.shape
    po = np.ascontiguousarray(plan_of, dtype=np.int64)
    if po.shape != (B,) or po.min() < 0 or po.max() >= len(plans):
        raise ValueError("plan_of needs one index into plans per RVE")
    if C != plans[0].ncomp:
        raise ValueError(f"macro strains need {plans[0].ncomp} components")
    nst = 5 if plans[0].ndim == 2 else 7
    handles, n_pts, n_coef = _plan_arrays(plans)
    npts = _plan_sum(n_pts, po)
    _check_tensor(state, "state", "float32", nst * npts)
    ncoef = _plan_sum(n_coef, po) * C
    out, eff, its, res, strain, stress, coeffs = _outputs(B * steps, 6, B * steps, False, want_coeffs,
                                                          npts, C, ncoef)
    if want_fields:  # field outputs hold the last step of each RVE
        torch = _torch()
        strain = torch.empty(C * npts, dtype=torch.float32, device="cuda")
        stress = torch.empty(plans[0].nstress * npts, dtype=torch.float32, device="cuda")
        out.strain = strain.data_ptr()
        out.stress = stress.data_ptr()
    opts = _opts(max_iter, check_every, None, stream, PREC_FP32, TRANSFORM_AUTO, use_graph, schedule)
    st = _check(lib.mor_solve_path_multi(handles, len(plans), _np_ptr(po), _np_ptr(eb), B, steps, _phases(phases),
                                         float(tol), ct.byref(opts), ct.c_void_p(state.data_ptr()),
                                         ct.byref(out)), allow)
    return SolveResult(st, eff.reshape(B, steps, 6), its.reshape(B, steps), res.reshape(B, steps), strain, stress,
                       coeffs)


def compat(plan: Plan, plan_full: Plan, coeffs, macro_strain, phases, state=None, stream=None,
           want_fields: bool = True, want_coeffs: bool = False, precision: int = PREC_FP32,
           transform: int = TRANSFORM_AUTO) -> SolveResult:
    """mor_compat: one full-set pass from the reduced coefficients `coeffs`
    (complex64 [B][ncomp][plan.n_coeff]); plan_full holds every frequency of
    the same microstructure.  Fields and coefficients come back on plan_full."""
    eb = np.ascontiguousarray(np.atleast_2d(macro_strain), dtype=np.float64)
    B, C = eb.shape
    if C != plan.ncomp:
        raise ValueError(f"macro strain needs {plan.ncomp} components")
    _check_tensor(coeffs, "coeffs", "complex64", B * C * plan.n_coeff)
    _check_tensor(state, "state", "float32", B * (5 if plan.ndim == 2 else 7) * plan.N)
    S = plan.nstress
    out, eff, its, res, strain, stress, co = _outputs(B, S, B, want_fields, want_coeffs, B * plan.N, C,
                                                      B * C * plan_full.n_coeff)
    opts = _opts(1, 1, None, stream, precision, transform)
    sp = ct.c_void_p(state.data_ptr()) if state is not None else ct.c_void_p(None)
    st = _check(lib.mor_compat(plan.handle, plan_full.handle, ct.c_void_p(coeffs.data_ptr()), _np_ptr(eb), B,
                               _phases(phases), sp, ct.byref(opts), ct.byref(out)))
    if strain is not None:
        strain = strain.view(B, C, *plan.shape)
        stress = stress.view(B, S, *plan.shape)
    if co is not None:
        co = co.view(B, C, plan_full.n_coeff)
    return SolveResult(st, eff, its, res, strain, stress, co)


def stress_error(sigma, sigma_ref, eff, eff_ref, ndim: int, skip_rel: float = 1e-12, stream=None):
    """mor_stress_error: (E_bar [B], E [B]) of Sec. 5.  sigma/sigma_ref:
    float32 CUDA tensors [B][nstress][...grid]; eff/eff_ref: [B][nstress]."""
    S = 4 if ndim == 2 else 6
    B = sigma.shape[0]
    N = sigma.numel() // (B * S)
    _check_tensor(sigma, "sigma", "float32", B * S * N)
    _check_tensor(sigma_ref, "sigma_ref", "float32", B * S * N)
    a = np.ascontiguousarray(np.asarray(eff, dtype=np.float64)[:, :S])
    r = np.ascontiguousarray(np.asarray(eff_ref, dtype=np.float64)[:, :S])
    if a.shape != (B, S) or r.shape != (B, S):
        raise ValueError(f"eff and eff_ref must be [{B}][{S}]")
    Eb = np.zeros(B)
    E = np.zeros(B)
    _check(lib.mor_stress_error(ct.c_void_p(sigma.data_ptr()), ct.c_void_p(sigma_ref.data_ptr()), _np_ptr(a),
                                _np_ptr(r), B, N, ndim, float(skip_rel), _stream_ptr(stream), _np_ptr(Eb),
                                _np_ptr(E)))
    return Eb, E


def profile_enable(on: bool = True):
    _check(lib.mor_profile_enable(1 if on else 0))


def profile_reset():
    _check(lib.mor_profile_reset())


def profile_query(kernel: str):
    ms = ct.c_double()
    la = ct.c_int64()
    it = ct.c_int64()
    by = ct.c_double()
    _check(lib.mor_profile_query(kernel.encode(), ct.byref(ms), ct.byref(la), ct.byref(it), ct.byref(by)))
    return {"ms": ms.value, "launches": la.value, "items": it.value, "bytes": by.value}


def version() -> str:
    return lib.mor_version().decode()


# ---------------------------------------------------------------- warm-start network
MLP_FP32 = 0
MLP_BF16 = 1


class MLP:
    """The library's 3-layer perceptron (mor_mlp_*): FP32 parameters on the device."""

    def __init__(self, in_dim: int, hidden: int, out_dim: int, seed: int = 0):
        h = ct.c_void_p()
        _check(lib.mor_mlp_create(int(in_dim), int(hidden), int(out_dim), int(seed), ct.byref(h)))
        self._h = h
        self.in_dim, self.hidden, self.out_dim = int(in_dim), int(hidden), int(out_dim)
        n = ct.c_int64()
        _check(lib.mor_mlp_num_params(self._h, ct.byref(n)))
        self.num_params = n.value

    def _get(self, which):
        out = np.zeros(self.num_params, np.float32)
        _check(lib.mor_mlp_get_params(self._h, _np_ptr(out), self.num_params, which))
        return out

    def params(self):
        return self._get(0)

    def grads(self):
        return self._get(1)

    def adam_moments(self):
        return self._get(2), self._get(3)

    def set_params(self, flat, which: int = 0):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        _check(lib.mor_mlp_set_params(self._h, _np_ptr(a), self.num_params, which))

    def split(self, flat):
        """[W1, b1, W2, b2, W3, b3] views of a flat parameter vector."""
        i, h, o = self.in_dim, self.hidden, self.out_dim
        sizes = [(i, h), (h,), (h, h), (h,), (h, o), (o,)]
        out, k = [], 0
        for sh in sizes:
            n = int(np.prod(sh))
            out.append(flat[k:k + n].reshape(sh))
            k += n
        return out

    def forward(self, X, precision: int = MLP_FP32, stream=None):
        torch = _torch()
        if X.dim() != 2 or X.shape[1] != self.in_dim:
            raise ValueError(f"X must be [B][{self.in_dim}]")
        _check_tensor(X, "X", "float32", X.shape[0] * self.in_dim)
        B = X.shape[0]
        Y = torch.empty((B, self.out_dim), dtype=torch.float32, device=X.device)
        _check(lib.mor_mlp_forward(self._h, ct.c_void_p(X.data_ptr()), B, ct.c_void_p(Y.data_ptr()),
                                   precision, _stream_ptr(stream)))
        return Y

    def grad(self, X, T, stream=None) -> float:
        if X.dim() != 2 or X.shape[1] != self.in_dim or T.dim() != 2 or T.shape != (X.shape[0], self.out_dim):
            raise ValueError(f"X must be [B][{self.in_dim}] and T [B][{self.out_dim}]")
        _check_tensor(X, "X", "float32", X.numel())
        _check_tensor(T, "T", "float32", T.numel())
        loss = ct.c_double()
        _check(lib.mor_mlp_grad(self._h, ct.c_void_p(X.data_ptr()), ct.c_void_p(T.data_ptr()), X.shape[0],
                                ct.byref(loss), _stream_ptr(stream)))
        return loss.value

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(lib.mor_mlp_adam(self._h, float(lr), float(beta1), float(beta2), float(eps), _stream_ptr(stream)))

    def close(self):
        if getattr(self, "_h", None):
            lib.mor_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _plan_array(plans):
    return _plan_arrays(plans)[0]


def warm_features(plans, plan_of, nslots: int, stream=None):
    torch = _torch()
    po = np.ascontiguousarray(plan_of, dtype=np.int64)
    X = torch.empty((len(po), 4 * nslots + 1), dtype=torch.float32, device="cuda")
    _check(lib.mor_warm_features(_plan_array(plans), len(plans), _np_ptr(po), len(po), nslots,
                                 ct.c_void_p(X.data_ptr()), _stream_ptr(stream)))
    return X


def warm_targets(plans, plan_of, nslots: int, phases, coeffs, stream=None):
    torch = _torch()
    po = np.ascontiguousarray(plan_of, dtype=np.int64)
    _check_tensor(coeffs, "coeffs", "complex64", 9 * _plan_sum(_plan_arrays(plans)[2], po))
    T = torch.empty((len(po), 18 * nslots), dtype=torch.float32, device="cuda")
    _check(lib.mor_warm_targets(_plan_array(plans), len(plans), _np_ptr(po), len(po), nslots, _phases(phases),
                                ct.c_void_p(coeffs.data_ptr()), ct.c_void_p(T.data_ptr()), _stream_ptr(stream)))
    return T


def warm_apply(plans, plan_of, nslots: int, phases, Y, macro_strain, stream=None):
    torch = _torch()
    po = np.ascontiguousarray(plan_of, dtype=np.int64)
    eb = np.ascontiguousarray(macro_strain, dtype=np.float64)
    if eb.shape != (len(po), 3):
        raise ValueError("macro_strain must be [B][3]")
    _check_tensor(Y, "Y", "float32", len(po) * 18 * int(nslots))
    n = _plan_sum(_plan_arrays(plans)[2], po) * 3
    W = torch.empty(n, dtype=torch.complex64, device="cuda")
    _check(lib.mor_warm_apply(_plan_array(plans), len(plans), _np_ptr(po), len(po), nslots, _phases(phases),
                              ct.c_void_p(Y.data_ptr()), _np_ptr(eb), ct.c_void_p(W.data_ptr()),
                              _stream_ptr(stream)))
    return W


# ---------------------------------------------------------------- kernel variants / autotuner
KERNEL_ROW = 0
KERNEL_COL = 1


def tune_variants(ndim: int, length: int, kernel: int = KERNEL_ROW) -> int:
    n = ct.c_int32(0)
    _check(lib.mor_tune_variants(kernel, ndim, length, ct.byref(n)))
    return n.value


def tune_get(ndim: int, length: int, kernel: int = KERNEL_ROW) -> int:
    v = ct.c_int32(0)
    _check(lib.mor_tune_get(kernel, ndim, length, ct.byref(v)))
    return v.value


def tune_set(ndim: int, length: int, variant: int, kernel: int = KERNEL_ROW) -> None:
    _check(lib.mor_tune_set(kernel, ndim, length, variant))


def tune_subbatch(nbytes: int = -1, min_rves: int = -1):
    """Set the sub-batch limits of the batched solves (bytes of transform
    lines, 0 = one sub-batch per grid; fewest RVEs per sub-batch; -1 keeps a
    value); returns the previous (bytes, min_rves)."""
    pb, pm = ct.c_int64(), ct.c_int64()
    _check(lib.mor_tune_subbatch(int(nbytes), int(min_rves), ct.byref(pb), ct.byref(pm)))
    return pb.value, pm.value


def autotune(plans, plan_of, macro_strain, phases, tol: float, reps: int = 2, stream=None) -> None:
    po = np.ascontiguousarray(plan_of, dtype=np.int64)
    eb = np.ascontiguousarray(macro_strain, dtype=np.float64)
    _check(lib.mor_autotune(_plan_array(plans), len(plans), _np_ptr(po), _np_ptr(eb), len(po), _phases(phases),
                            float(tol), reps, _stream_ptr(stream)))
