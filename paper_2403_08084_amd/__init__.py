"""Python binding of the MI355X fully implicit Runge-Kutta stage solver (libirk.so).

This module only marshals arguments: every step of the solve runs in the HIP
kernels behind the C ABI declared in include/irk.h. PyTorch supplies device
memory (CUDA/HIP tensors) and the stream; nothing here computes on the CPU.
If libirk.so has not been built, using any entry point raises RuntimeError
(there is no fallback path).

Main objects
  Problem(N, kappa)                the Q1 grid and per-element diffusivity
  Stepper(problem, tableau, dt, ...)  a tableau, time step and solver options
  IrkSolve                         torch.autograd.Function: u_N(u_0, log kappa)

Stepper options (fields of irk_options; defaults from irk_options_default):
  precond       PC_GS_LOWER (block lower Gauss-Seidel), PC_JACOBI, PC_GS_UPPER, PC_RANA_LD, PC_MONOLITHIC
  splitting     SPLIT_AI (stage derivatives k) or SPLIT_IA (w = (A (x) I) k)
  stage_type    STAGE_COUPLED or STAGE_DIRK (stage-by-stage solves, lower-triangular A)
  mg_precision  F64, F32 or BF16 storage of the multigrid vectors (FGMRES stays FP64; with F32 / BF16 the
                flexible basis of preconditioned vectors is FP32 unless basis_f64=1, which gives the same bits)
  orth          ORTH_DCGS2 (one reduction per Arnoldi step), ORTH_CGS2, ORTH_CGS_SELECTIVE
  lookahead     LOOKAHEAD_ADAPTIVE (queue the next Arnoldi step before the host's convergence test
                while the residual history predicts it is needed), LOOKAHEAD_OFF, LOOKAHEAD_ALWAYS
  rtol, restart, max_it, mg_coarse_n, cheb_degree, cheb_lo, cheb_hi, power_its, initial_guess, use_graphs

Example (1024^2, Radau IIA(3), mixed precision, monolithic multigrid):
  prob = Problem(1024, kappa_dev)
  stp = Stepper(prob, tableaux.radau_iia(3), 1e-3, mg_precision=F32, precond=PC_MONOLITHIC)
  rc, stats = stp.advance(u_dev, 20)
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

from . import tableaux  # noqa: F401  (product-side tableau constructors)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libirk.so")

IRK_OK, IRK_EINVAL, IRK_ENOMEM, IRK_EHIP, IRK_ENOCONV, IRK_EBREAKDOWN = 0, -1, -2, -3, -4, -5
PC_JACOBI, PC_GS_LOWER, PC_RANA_LD, PC_GS_UPPER, PC_MONOLITHIC = 0, 1, 2, 3, 4
SPLIT_AI, SPLIT_IA = 0, 1
STAGE_COUPLED, STAGE_DIRK = 0, 1
F64, F32, BF16 = 0, 1, 2
ORTH_CGS2, ORTH_CGS_SELECTIVE, ORTH_DCGS2 = 0, 1, 2
GUESS_ZERO, GUESS_PREV = 0, 1
LOOKAHEAD_OFF, LOOKAHEAD_ADAPTIVE, LOOKAHEAD_ALWAYS = 0, 1, 2
KFAM_GRAM_SCHMIDT, KFAM_OPERATOR, KFAM_MG_FINE, KFAM_MG_COARSE, KFAM_COARSE_SOLVE, KFAM_REDUCE_FINISH, KFAM_OTHER = range(7)
KFAM_NAMES = ["gram_schmidt", "operator", "mg_fine", "mg_coarse", "coarse_solve", "reduce_finish", "other"]
KFAM_ALL = 100

_STATUS = {IRK_EINVAL: "EINVAL", IRK_ENOMEM: "ENOMEM", IRK_EHIP: "EHIP", IRK_ENOCONV: "ENOCONV",
           IRK_EBREAKDOWN: "EBREAKDOWN"}


class IrkError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"irk error {_STATUS.get(code, code)}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [
        ("precond", ctypes.c_int),
        ("rtol", ctypes.c_double),
        ("restart", ctypes.c_int),
        ("max_it", ctypes.c_int),
        ("mg_coarse_n", ctypes.c_int),
        ("cheb_degree", ctypes.c_int),
        ("cheb_lo", ctypes.c_double),
        ("cheb_hi", ctypes.c_double),
        ("power_its", ctypes.c_int),
        ("mg_precision", ctypes.c_int),
        ("orth", ctypes.c_int),
        ("initial_guess", ctypes.c_int),
        ("use_graphs", ctypes.c_int),
        ("splitting", ctypes.c_int),
        ("stage_type", ctypes.c_int),
        ("lookahead", ctypes.c_int),
        ("basis_f64", ctypes.c_int),
    ]


class _Tableau(ctypes.Structure):
    _fields_ = [
        ("s", ctypes.c_int),
        ("A", ctypes.POINTER(ctypes.c_double)),
        ("b", ctypes.POINTER(ctypes.c_double)),
        ("c", ctypes.POINTER(ctypes.c_double)),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("steps_done", ctypes.c_int),
        ("fgmres_its_total", ctypes.c_int),
        ("fgmres_its_max", ctypes.c_int),
        ("restarts_total", ctypes.c_int),
        ("solves", ctypes.c_int),
        ("forward_advances", ctypes.c_int),
        ("last_rel_resid", ctypes.c_double),
        ("failed_step", ctypes.c_int),
        ("arnoldi_discarded", ctypes.c_int),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None

SYMBOLS = [
    "irk_last_error", "irk_options_default", "irk_problem_create", "irk_problem_destroy", "irk_problem_set_kappa",
    "irk_apply_mass", "irk_apply_stiffness", "irk_apply_mass_noalloc", "irk_stepper_create", "irk_stepper_destroy",
    "irk_stepper_refresh", "irk_stage_rhs", "irk_apply_stage_operator", "irk_apply_preconditioner", "irk_vcycle",
    "irk_solve_stages", "irk_advance", "irk_adjoint", "irk_revolve_schedule", "irk_stepper_sizes", "irk_stepper_mu",
    "irk_stepper_mmg_mu", "irk_kernel_timer", "irk_kernel_timer_family", "irk_kernel_timer_read", "irk_device_copy",
]


def lib():
    """Load libirk.so (once). Raises RuntimeError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libirk.so not found at {LIB_PATH}: build it with `python -m paper_2403_08084_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
    L.irk_last_error.restype = ctypes.c_char_p
    L.irk_last_error.argtypes = []
    L.irk_options_default.restype = None
    L.irk_options_default.argtypes = [ctypes.POINTER(Options)]
    L.irk_problem_create.argtypes = [ctypes.POINTER(vp), ip, vp, vp]
    L.irk_problem_destroy.restype = None
    L.irk_problem_destroy.argtypes = [vp]
    L.irk_problem_set_kappa.argtypes = [vp, vp, vp]
    L.irk_apply_mass.argtypes = [vp, vp, vp, vp]
    L.irk_apply_stiffness.argtypes = [vp, vp, vp, vp]
    L.irk_apply_mass_noalloc.argtypes = [vp, vp, vp, vp]
    L.irk_stepper_create.argtypes = [ctypes.POINTER(vp), vp, ctypes.POINTER(_Tableau), ctypes.c_double,
                                     ctypes.POINTER(Options), vp]
    L.irk_stepper_destroy.restype = None
    L.irk_stepper_destroy.argtypes = [vp]
    L.irk_stepper_refresh.argtypes = [vp, vp]
    L.irk_stage_rhs.argtypes = [vp, vp, vp, vp, vp]
    L.irk_apply_stage_operator.argtypes = [vp, vp, vp, ip, vp]
    L.irk_apply_preconditioner.argtypes = [vp, vp, vp, ip, vp]
    L.irk_vcycle.argtypes = [vp, ip, vp, vp, vp]
    L.irk_solve_stages.argtypes = [vp, vp, vp, ip, ctypes.POINTER(Stats), vp]
    L.irk_advance.argtypes = [vp, vp, vp, ip, ctypes.POINTER(Stats), vp]
    L.irk_adjoint.argtypes = [vp, vp, ip, ip, vp, vp, vp, ctypes.POINTER(Stats), vp]
    L.irk_revolve_schedule.argtypes = [ip, ip, ctypes.POINTER(ctypes.c_int), ip, ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_int)]
    L.irk_stepper_sizes.argtypes = [vp, ctypes.POINTER(ip), ctypes.POINTER(ip), ctypes.POINTER(ip)]
    L.irk_stepper_mu.argtypes = [vp, ip, ip, dp]
    L.irk_stepper_mmg_mu.argtypes = [vp, ip, ip, dp, ctypes.POINTER(ip)]
    L.irk_kernel_timer.argtypes = [vp, ip, ip]
    L.irk_kernel_timer_read.argtypes = [vp, ctypes.POINTER(ip), dp, dp]
    L.irk_kernel_timer_family.argtypes = [vp, ip, ctypes.POINTER(ip), dp, dp, dp]
    L.irk_device_copy.argtypes = [vp, vp, ctypes.c_longlong, vp]
    for name in SYMBOLS:
        if name not in ("irk_last_error", "irk_options_default", "irk_problem_destroy", "irk_stepper_destroy"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != IRK_OK:
        raise IrkError(rc, lib().irk_last_error().decode())


def default_options(**overrides) -> Options:
    o = Options()
    lib().irk_options_default(ctypes.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _torch():
    import torch

    return torch


def _dev_ptr(t, numel=None, name="tensor"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device (HIP) tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} entries, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Problem:
    """Uniform N x N Q1 grid of the unit square with per-element kappa (device, N*N float64)."""

    def __init__(self, N: int, kappa, stream=None):
        self.N = int(N)
        self.n = (self.N - 1) ** 2
        self._h = ctypes.c_void_p()
        _check(lib().irk_problem_create(ctypes.byref(self._h), self.N, _dev_ptr(kappa, self.N * self.N, "kappa"),
                                        _stream(stream)))

    def close(self):
        if self._h:
            lib().irk_problem_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_kappa(self, kappa, stream=None):
        """Replace kappa (device, N*N float64); call refresh() on every Stepper of this problem afterwards."""
        _check(lib().irk_problem_set_kappa(self._h, _dev_ptr(kappa, self.N * self.N, "kappa"), _stream(stream)))

    def apply_mass(self, x, stream=None):
        y = _torch().empty_like(x)
        _check(lib().irk_apply_mass(self._h, _dev_ptr(x, self.n, "x"), _dev_ptr(y), _stream(stream)))
        return y

    def apply_mass_noalloc(self, x, y, stream=None):
        """y = M x into the caller's y without any device allocation by the library (N <= 1024)."""
        _check(lib().irk_apply_mass_noalloc(self._h, _dev_ptr(x, self.n, "x"), _dev_ptr(y, self.n, "y"),
                                            _stream(stream)))
        return y

    def apply_stiffness(self, x, stream=None):
        y = _torch().empty_like(x)
        _check(lib().irk_apply_stiffness(self._h, _dev_ptr(x, self.n, "x"), _dev_ptr(y), _stream(stream)))
        return y


class Stepper:
    """A Butcher tableau, time step and solver options on a Problem (see irk.h for the options)."""

    def __init__(self, problem: Problem, tableau, dt: float, stream=None, **options):
        import numpy as np

        A = np.ascontiguousarray(np.asarray(tableau["A"], dtype=np.float64))
        b = np.ascontiguousarray(np.asarray(tableau["b"], dtype=np.float64))
        c = np.ascontiguousarray(np.asarray(tableau.get("c", np.zeros_like(b)), dtype=np.float64))
        self.s = int(b.size)
        self.problem = problem
        self.N = problem.N
        self.n = problem.n
        self.dt = float(dt)
        self._keep = (A, b, c)
        tab = _Tableau(self.s, A.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                       b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                       c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        self.options = default_options(**options)
        self._h = ctypes.c_void_p()
        _check(lib().irk_stepper_create(ctypes.byref(self._h), problem._h, ctypes.byref(tab), self.dt,
                                        ctypes.byref(self.options), _stream(stream)))

    def close(self):
        if self._h:
            lib().irk_stepper_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def refresh(self, stream=None):
        """Rebuild the kappa-dependent multigrid state after Problem.set_kappa (buffers are reused)."""
        _check(lib().irk_stepper_refresh(self._h, _stream(stream)))

    @property
    def levels(self) -> int:
        L = ctypes.c_int()
        _check(lib().irk_stepper_sizes(self._h, None, None, ctypes.byref(L)))
        return L.value

    def mu(self, stage: int, level: int) -> float:
        v = ctypes.c_double()
        _check(lib().irk_stepper_mu(self._h, stage, level, ctypes.byref(v)))
        return v.value

    @property
    def mmg_levels(self) -> int:
        """Level count of the monolithic cycle (monolithic-multigrid steppers only)."""
        L = ctypes.c_int()
        _check(lib().irk_stepper_mmg_mu(self._h, 0, 0, None, ctypes.byref(L)))
        return L.value

    def mmg_mu(self, level: int, transpose: bool = False) -> float:
        v = ctypes.c_double()
        _check(lib().irk_stepper_mmg_mu(self._h, int(bool(transpose)), level, ctypes.byref(v), None))
        return v.value

    def kernel_timer(self, family: int = 0, enable: bool = True):
        """Enable/disable the HIP-event measurement hook for a kernel family (KFAM_*, or KFAM_ALL)."""
        _check(lib().irk_kernel_timer(self._h, int(family), int(bool(enable))))

    def kernel_timer_read(self):
        """(launches, total_ms, algorithmic_bytes) accumulated over the timed families since enabling."""
        n = ctypes.c_int()
        ms = ctypes.c_double()
        by = ctypes.c_double()
        _check(lib().irk_kernel_timer_read(self._h, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
        return n.value, ms.value, by.value

    def kernel_timer_family(self, family: int):
        """(launches, total_ms, bytes per-pass model, bytes fused minimum) of one family (or KFAM_ALL)."""
        n = ctypes.c_int()
        ms, by, bm = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib().irk_kernel_timer_family(self._h, int(family), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by),
                                             ctypes.byref(bm)))
        return n.value, ms.value, by.value, bm.value

    def stage_rhs(self, u, F=None, stream=None):
        f = _torch().empty(self.s * self.n, dtype=u.dtype, device=u.device)
        Fp = _dev_ptr(F, self.n, "F") if F is not None else None
        _check(lib().irk_stage_rhs(self._h, _dev_ptr(u, self.n, "u"), Fp, _dev_ptr(f), _stream(stream)))
        return f

    def apply_stage_operator(self, x, transpose=False, stream=None):
        y = _torch().empty_like(x)
        _check(lib().irk_apply_stage_operator(self._h, _dev_ptr(x, self.s * self.n, "x"), _dev_ptr(y),
                                              int(bool(transpose)), _stream(stream)))
        return y

    def apply_preconditioner(self, v, transpose=False, stream=None):
        z = _torch().empty_like(v)
        _check(lib().irk_apply_preconditioner(self._h, _dev_ptr(v, self.s * self.n, "v"), _dev_ptr(z),
                                              int(bool(transpose)), _stream(stream)))
        return z

    def vcycle(self, stage: int, t, stream=None):
        z = _torch().empty_like(t)
        _check(lib().irk_vcycle(self._h, int(stage), _dev_ptr(t, self.n, "t"), _dev_ptr(z), _stream(stream)))
        return z

    def solve_stages(self, f, transpose=False, stream=None):
        k = _torch().empty_like(f)
        st = Stats()
        _check(lib().irk_solve_stages(self._h, _dev_ptr(f, self.s * self.n, "f"), _dev_ptr(k), int(bool(transpose)),
                                      ctypes.byref(st), _stream(stream)))
        return k, st.as_dict()

    def advance(self, u, nsteps: int, F=None, stream=None, check=True):
        """Advance u (device, n float64) in place by nsteps steps; returns (status, stats dict)."""
        st = Stats()
        Fp = _dev_ptr(F, self.n, "F") if F is not None else None
        rc = lib().irk_advance(self._h, _dev_ptr(u, self.n, "u"), Fp, int(nsteps), ctypes.byref(st), _stream(stream))
        if check:
            _check(rc)
        return rc, st.as_dict()

    def adjoint(self, u0, nsteps: int, nsnap: int, lam_T, stream=None):
        """Returns (lambda_0, grad_log_kappa, stats dict)."""
        torch = _torch()
        lam0 = torch.empty_like(u0)
        grad = torch.empty(self.N * self.N, dtype=u0.dtype, device=u0.device)
        st = Stats()
        _check(lib().irk_adjoint(self._h, _dev_ptr(u0, self.n, "u0"), int(nsteps), int(nsnap),
                                 _dev_ptr(lam_T, self.n, "lambda_T"), _dev_ptr(lam0), _dev_ptr(grad),
                                 ctypes.byref(st), _stream(stream)))
        return lam0, grad, st.as_dict()


def device_copy(x, y, stream=None):
    """y = x (device float64 vectors of equal length): the library's plain streaming copy, the reference kernel for
    bandwidth ceilings and counter scaling."""
    n = int(x.numel())
    if int(y.numel()) != n:
        raise ValueError("x and y differ in length")
    _check(lib().irk_device_copy(_dev_ptr(x, n, "x"), _dev_ptr(y, n, "y"), n, _stream(stream)))


def revolve_schedule(nsteps: int, nsnap: int):
    """Binomial checkpointing schedule: (list of (kind, arg), forward advances). Host only."""
    count = ctypes.c_int()
    adv = ctypes.c_int()
    _check(lib().irk_revolve_schedule(nsteps, nsnap, None, 0, ctypes.byref(count), ctypes.byref(adv)))
    buf = (ctypes.c_int * (2 * count.value))()
    _check(lib().irk_revolve_schedule(nsteps, nsnap, buf, count.value, ctypes.byref(count), ctypes.byref(adv)))
    acts = [(buf[2 * i], buf[2 * i + 1]) for i in range(count.value)]
    return acts, adv.value


@dataclass
class SolveConfig:
    """Fixed settings of an IrkSolve call: N, tableau, dt, steps, snapshot count, solver options."""

    N: int
    tableau: dict
    dt: float
    nsteps: int
    nsnap: int = 8
    options: dict = None


def _solver_key(cfg: SolveConfig, device):
    import numpy as np

    tab = tuple(tuple(np.asarray(cfg.tableau[k], dtype=np.float64).ravel().tolist())
                for k in ("A", "b", "c") if k in cfg.tableau)
    opts = tuple(sorted((cfg.options or {}).items()))
    return (int(cfg.N), str(device), float(cfg.dt), tab, opts)


class _CachedSolver:
    """A Problem/Stepper pair and the kappa it currently holds (version counts the loads of kappa)."""

    def __init__(self, cfg: SolveConfig, kappa):
        self.problem = Problem(cfg.N, kappa)
        self.stepper = Stepper(self.problem, cfg.tableau, cfg.dt, **(cfg.options or {}))
        self.kappa = kappa
        self.version = 0

    def hold(self, kappa):
        """Load kappa (unless it is the one held) and refresh the stepper; returns the version holding it."""
        if kappa is not self.kappa and not _torch().equal(kappa, self.kappa):
            self.problem.set_kappa(kappa)
            self.stepper.refresh()
            self.version += 1
        self.kappa = kappa
        return self.version


class _SolverCache:
    """Solvers of IrkSolve, kept across calls with the same grid, tableau, dt, options and device: a call with
    a new kappa reloads it into the cached problem and refreshes the stepper (no new workspace, no set-up of
    the Krylov buffers). A backward pass whose kappa another call has replaced since its forward pass loads
    its own again. Entries dropped from the cache live on while a pending backward pass holds them."""

    def __init__(self, size: int = 2):
        self.size = size
        self.entries = {}  # key -> _CachedSolver; insertion order = age

    def get(self, cfg: SolveConfig, kappa) -> _CachedSolver:
        key = _solver_key(cfg, kappa.device)
        e = self.entries.pop(key, None)
        if e is None:
            while len(self.entries) >= self.size:
                self.entries.pop(next(iter(self.entries)))
            e = _CachedSolver(cfg, kappa)
        else:
            e.hold(kappa)
        self.entries[key] = e
        return e

    def clear(self):
        self.entries.clear()


_solver_cache = _SolverCache()


def _make_irk_solve():
    torch = _torch()

    class IrkSolve(torch.autograd.Function):
        """u_N = Phi(u_0, log kappa): nsteps implicit Runge-Kutta steps; backward = discrete adjoint.
        The Problem/Stepper of a configuration are cached across calls (see _SolverCache)."""

        @staticmethod
        def forward(ctx, u0, log_kappa, cfg: SolveConfig):
            kappa = torch.exp(log_kappa.detach()).contiguous()
            e = _solver_cache.get(cfg, kappa)
            u = u0.detach().clone().contiguous()
            e.stepper.advance(u, cfg.nsteps)
            ctx.solver = e
            ctx.cfg = cfg
            ctx.save_for_backward(u0.detach().clone(), kappa)
            return u

        @staticmethod
        def backward(ctx, grad_out):
            u0, kappa = ctx.saved_tensors
            cfg = ctx.cfg
            e = ctx.solver
            e.hold(kappa)
            lam0, grad, _ = e.stepper.adjoint(u0, cfg.nsteps, cfg.nsnap, grad_out.contiguous())
            return lam0, grad, None

    return IrkSolve


class _Lazy:
    _cls = None

    def __getattr__(self, item):
        if _Lazy._cls is None:
            _Lazy._cls = _make_irk_solve()
        return getattr(_Lazy._cls, item)


IrkSolve = _Lazy()
