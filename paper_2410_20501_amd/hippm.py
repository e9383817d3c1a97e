"""ctypes binding of libhippm.so (include/hippm.h): argument marshalling only.

Every function takes torch tensors that live on the GPU, checks dtype, shape
and contiguity, and passes raw device pointers and the current torch stream to
the C entry point of the same name. No arithmetic of the method happens here.
"""
from __future__ import annotations

import ctypes
import os
import warnings
from ctypes import POINTER, byref, c_char_p, c_double, c_float, c_int, c_int64, c_void_p

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhippm.so")

# enums (mirror include/hippm.h)
PM_OK, PM_WARN_NOT_CONVERGED, PM_WARN_FLOOR = 0, 1, 2
PM_ERR_ARG, PM_ERR_SHAPE, PM_ERR_NOMEM, PM_ERR_HIP, PM_ERR_NONFINITE = -1, -2, -3, -4, -5
PM_NGP, PM_CIC, PM_TSC = 1, 2, 3
PM_DEPOSIT_ATOMIC, PM_DEPOSIT_SORTED = 0, 1
PM_POS_BOX, PM_POS_CELLOFF = 0, 1
PM_RESTRICT_FW, PM_RESTRICT_AVG = 0, 1
PM_CYCLE_V, PM_CYCLE_W, PM_CYCLE_F = 0, 1, 2
PM_SOLVER_MG, PM_SOLVER_FFT, PM_SOLVER_FFT_7PT, PM_SOLVER_FULL_FFT = 0, 1, 2, 3
PM_FFT_GREEN, PM_FFT_7PT, PM_FFT_FULL = 0, 1, 2
PM_GRAVITY_NEWTON, PM_GRAVITY_MU, PM_GRAVITY_QUMOND, PM_GRAVITY_FR = 0, 1, 2, 3
PM_NU_SIMPLE, PM_NU_N, PM_NU_BETA, PM_NU_GAMMA, PM_NU_DELTA = 0, 1, 2, 3, 4
PM_GUESS_JACOBI, PM_GUESS_WARM, PM_GUESS_WARM_RESCALED, PM_GUESS_EXTRAPOLATED = 0, 1, 2, 3
PM_CHAIN_FIRST, PM_CHAIN_NEXT = 0, 1
PM_ADJ_CLOSING_MERGED = 1
PM_CREATE_REFERENCE_KERNELS, PM_CREATE_CHECK_FINITE = 1, 2
PM_KERNEL_NONE, PM_KERNEL_DEPOSIT, PM_KERNEL_SMOOTH, PM_KERNEL_INTERP, PM_KERNEL_FR_SWEEP = 0, 1, 2, 3, 4

MAS = {"ngp": PM_NGP, "cic": PM_CIC, "tsc": PM_TSC}
SOLVER = {"mg": PM_SOLVER_MG, "fft": PM_SOLVER_FFT, "fft_7pt": PM_SOLVER_FFT_7PT,
          "full_fft": PM_SOLVER_FULL_FFT}
FFT_KERNEL = {"green": PM_FFT_GREEN, "7pt": PM_FFT_7PT, "full": PM_FFT_FULL}
GRAVITY = {"newton": PM_GRAVITY_NEWTON, "mu": PM_GRAVITY_MU, "qumond": PM_GRAVITY_QUMOND,
           "fr": PM_GRAVITY_FR}
NU_FAMILY = {"simple": PM_NU_SIMPLE, "n": PM_NU_N, "beta": PM_NU_BETA, "gamma": PM_NU_GAMMA,
             "delta": PM_NU_DELTA}
ORDER = {"atomic": PM_DEPOSIT_ATOMIC, "sorted": PM_DEPOSIT_SORTED}


class PMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hippm error {code}: {msg}")
        self.code = code


class PMWarning(UserWarning):
    pass


class MGParams(ctypes.Structure):
    _fields_ = [("pre", c_int), ("post", c_int), ("omega", c_float), ("tol", c_float),
                ("max_cycles", c_int), ("restrict_kind", c_int), ("guess", c_int),
                ("fixed_cycles", c_int), ("alpha", c_float), ("cycle", c_int)]


class MGStats(ctypes.Structure):
    _fields_ = [("cycles", c_int), ("status", c_int), ("relres", c_double * 64)]

    def history(self):
        return [self.relres[i] for i in range(self.cycles + 1)]


class StepParams(ctypes.Structure):
    _fields_ = [("mas", c_int), ("order", c_int), ("solver", c_int), ("fft_deconv", c_int),
                ("omega_m", c_double), ("mg", MGParams), ("timing", c_int),
                ("omega_l", c_double), ("gravity", c_int), ("mond_family", c_int),
                ("mu0", c_double), ("mond_g0", c_double), ("mond_g0_exp", c_double),
                ("mond_param", c_double), ("fr_f0", c_double), ("fr_c2", c_double),
                ("fr_n", c_int), ("fr_cycles", c_int), ("fr_cycle", c_int), ("fr_pre", c_int),
                ("fr_post", c_int), ("fr_coarse_sweeps", c_int)]


class StepStats(ctypes.Structure):
    _fields_ = [("mg", MGStats), ("ms_drift", c_float), ("ms_deposit", c_float),
                ("ms_solve", c_float), ("ms_gradient", c_float), ("ms_interp", c_float)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python paper_2410_20501_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    sig = {
        "pm_default_step_params": (None, [POINTER(StepParams)]),
        "pm_supercomoving_time": (c_double, [c_double, c_double, c_double, c_double]),
        "pm_create": (c_int, [POINTER(c_void_p), c_int, c_int64, c_int]),
        "pm_destroy": (None, [P]),
        "pm_last_error": (c_char_p, [P]),
        "pm_deposit": (c_int, [P, P, P, c_int64, c_int, c_int, c_int, P, P]),
        "pm_solve_mg": (c_int, [P, P, c_float, P, POINTER(MGParams), POINTER(MGStats), P]),
        "pm_solve_fft": (c_int, [P, P, c_float, c_int, P, P]),
        "pm_solve_fft_kernel": (c_int, [P, P, c_float, c_int, c_int, P, P]),
        "pm_solve_fft_noalloc": (c_int, [P, c_int, c_float, c_int, P, P]),
        "pm_solve_fr": (c_int, [P, P, c_double, POINTER(StepParams), P, POINTER(c_double), P]),
        "pm_gradient": (c_int, [P, P, c_int, P, P]),
        "pm_interp": (c_int, [P, P, P, c_int64, c_int, c_int, P, P, P]),
        "pm_accel": (c_int, [P, P, P, c_int64, c_int, c_double, POINTER(StepParams), P, P,
                             POINTER(StepStats), P]),
        "pm_kernel_timer": (c_int, [P, c_int, c_int]),
        "pm_kernel_timer_read": (c_int, [P, POINTER(c_double), POINTER(c_int64), POINTER(c_double)]),
        "pm_reorder": (c_int, [P, P, P, P, P, P, c_int64, c_int, P]),
        "pm_kdk": (c_int, [P, P, P, P, c_int64, c_int, c_double, c_double, POINTER(StepParams),
                           P, P, POINTER(StepStats), P]),
        "pm_kdk_chain": (c_int, [P, P, P, P, c_int64, c_int, c_double, c_double, c_double, c_int,
                                 POINTER(StepParams), P, P, POINTER(StepStats), P]),
        "pm_deposit_vjp": (c_int, [P, P, P, c_int64, c_int, c_int, P, P, P]),
        "pm_interp_vjp": (c_int, [P, P, P, c_int64, c_int, c_int, P, P, P, P, P]),
        "pm_gradient_vjp": (c_int, [P, P, c_int, P, P]),
        "pm_accel_vjp": (c_int, [P, P, P, c_int64, c_int, c_double, POINTER(StepParams), P, P,
                                 c_float, P, POINTER(MGStats), P]),
        "pm_kdk_adjoint": (c_int, [P, P, P, P, P, P, P, c_int64, c_int, c_double, c_double,
                                   c_double, POINTER(StepParams), c_int, P, P,
                                   POINTER(StepStats), P]),
        "pm_density_loss": (c_int, [P, P, P, c_int64, c_int, c_int, c_int, P,
                                    POINTER(c_double), P, P]),
        "pm_ic_state": (c_int, [P, P, P, c_int64, c_double, P, P, P, P]),
        "pm_ic_vjp": (c_int, [P, P, P, c_int64, c_double, P, P]),
        "pm_ic_lpt": (c_int, [P, P, c_int, POINTER(c_double), POINTER(c_double), c_int, c_int,
                              c_double, P, P, P, P]),
        "pm_power_spectrum": (c_int, [P, P, c_int, c_int, POINTER(c_double), POINTER(c_double),
                                      POINTER(c_int64), P]),
        "pm_batch_create": (c_int, [POINTER(c_void_p), c_int, POINTER(c_int), POINTER(c_int64),
                                    c_int]),
        "pm_batch_destroy": (None, [P]),
        "pm_batch_last_error": (c_char_p, [P]),
        "pm_batch_layout": (c_int, [P, POINTER(c_int64), POINTER(c_int64)]),
        "pm_batch_accel": (c_int, [P, P, P, P, c_double, POINTER(StepParams), POINTER(c_double),
                                   P]),
        "pm_batch_kdk": (c_int, [P, P, P, P, P, c_int, POINTER(c_double), POINTER(StepParams),
                                 c_int, P]),
        "pm_graph_capture_step": (c_int, [P, P, P, P, P, POINTER(StepParams), P]),
        "pm_tune": (c_int, [P, P, P, POINTER(StepParams), POINTER(c_int), P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib, sorted(sig)


_lib, EXPORTED = _load()


def default_step_params(**kw) -> StepParams:
    p = StepParams()
    _lib.pm_default_step_params(byref(p))
    for k, v in kw.items():
        if k == "mas":
            v = MAS.get(v, v)
        elif k == "order":
            v = ORDER.get(v, v)
        elif k == "solver":
            v = SOLVER.get(v, v)
        elif k == "gravity":
            v = GRAVITY.get(v, v)
        elif k == "mond_family":
            v = NU_FAMILY.get(v, v)
        elif k == "guess":
            v = {"jacobi": PM_GUESS_JACOBI, "warm": PM_GUESS_WARM,
                 "warm_rescaled": PM_GUESS_WARM_RESCALED,
                 "extrapolated": PM_GUESS_EXTRAPOLATED}.get(v, v)
        elif k == "restrict_kind":
            v = {"fw": PM_RESTRICT_FW, "avg": PM_RESTRICT_AVG}.get(v, v)
        elif k in ("cycle", "fr_cycle"):
            v = {"V": PM_CYCLE_V, "W": PM_CYCLE_W, "F": PM_CYCLE_F}.get(v, v)
        if hasattr(p.mg, k) and k not in ("mas",):
            setattr(p.mg, k, v)
        else:
            setattr(p, k, v)
    return p


def pm_supercomoving_time(omega_m, omega_l, a0, a1):
    """Supercomoving time between a0 and a1 for the background (host function)."""
    return _lib.pm_supercomoving_time(float(omega_m), float(omega_l), float(a0), float(a1))


def _stream():
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype=torch.float32, shape=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return c_void_p(t.data_ptr())


class Context:
    """Owner of a pm_ctx (scratch for an n^3 grid and up to np_max particles)."""

    def __init__(self, n: int, np_max: int = 0, flags: int = 0):
        h = c_void_p()
        st = _lib.pm_create(byref(h), int(n), int(np_max), int(flags))
        if st != PM_OK:
            raise PMError(st, f"pm_create(n={n}, np_max={np_max}) failed")
        self._h = h
        self.n = int(n)

    def close(self):
        if getattr(self, "_h", None):
            _lib.pm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        if not self._h:
            raise PMError(PM_ERR_ARG, "context closed")
        return self._h

    def _check(self, st, what):
        if st < 0:
            raise PMError(st, f"{what}: {_lib.pm_last_error(self._h).decode()}")
        if st > 0:
            warnings.warn(f"{what}: {_lib.pm_last_error(self._h).decode()}", PMWarning, stacklevel=3)
        return st


def pm_create(n, np_max=0, flags=0) -> Context:
    return Context(n, np_max, flags)


def pm_destroy(ctx: Context):
    ctx.close()


def _particles(pos, cell):
    np_ = pos.shape[0]
    if pos.dim() != 2 or pos.shape[1] != 3:
        raise ValueError("positions must be [np, 3]")
    kind = PM_POS_BOX if cell is None else PM_POS_CELLOFF
    return np_, kind, _ptr(pos, shape=(np_, 3), name="pos"), _ptr(cell, torch.int32, (np_,), "cell")


def pm_deposit(ctx: Context, pos, rho, cell=None, mas="tsc", order="atomic"):
    n = ctx.n
    np_, kind, pp, cp = _particles(pos, cell)
    st = _lib.pm_deposit(ctx.handle, pp, cp, np_, kind, MAS.get(mas, mas), ORDER.get(order, order),
                         _ptr(rho, shape=(n, n, n), name="rho"), _stream())
    return ctx._check(st, "pm_deposit")


def pm_solve_mg(ctx: Context, rho, coef, phi, params: MGParams | None = None, **kw):
    n = ctx.n
    if params is None:
        params = default_step_params(**kw).mg
    stats = MGStats()
    st = _lib.pm_solve_mg(ctx.handle, _ptr(rho, shape=(n, n, n), name="rho"), float(coef),
                          _ptr(phi, shape=(n, n, n), name="phi"), byref(params), byref(stats),
                          _stream())
    ctx._check(st, "pm_solve_mg")
    return stats


def pm_solve_fft(ctx: Context, rho, coef, phi, deconv=3):
    n = ctx.n
    st = _lib.pm_solve_fft(ctx.handle, _ptr(rho, shape=(n, n, n), name="rho"), float(coef),
                           int(deconv), _ptr(phi, shape=(n, n, n), name="phi"), _stream())
    return ctx._check(st, "pm_solve_fft")


def pm_solve_fft_kernel(ctx: Context, rho, coef, out, kernel="green", deconv=3):
    """kernel "green" / "7pt": out = phi [n, n, n]; "full": out = g [n, n, n, 3]."""
    n = ctx.n
    kid = FFT_KERNEL.get(kernel, kernel)
    shape = (n, n, n, 3) if kid == PM_FFT_FULL else (n, n, n)
    st = _lib.pm_solve_fft_kernel(ctx.handle, _ptr(rho, shape=(n, n, n), name="rho"), float(coef),
                                  int(kid), int(deconv), _ptr(out, shape=shape, name="out"),
                                  _stream())
    return ctx._check(st, "pm_solve_fft_kernel")


def pm_solve_fr(ctx: Context, rho, a, params: StepParams, u, relres=False):
    """f(R) scalaron u (float64 [n, n, n], in: guess, out: result) by params.fr_cycles FAS
    cycles on the density rho. With relres=True returns the relative residual before and
    after the cycles (host synchronisation), else None."""
    n = ctx.n
    rr = (c_double * 2)()
    st = _lib.pm_solve_fr(ctx.handle, _ptr(rho, shape=(n, n, n), name="rho"), float(a),
                          byref(params), _ptr(u, dtype=torch.float64, shape=(n, n, n), name="u"),
                          rr if relres else None, _stream())
    ctx._check(st, "pm_solve_fr")
    return (rr[0], rr[1]) if relres else None


def pm_solve_fft_noalloc(rho, coef, phi, deconv=3):
    """pm_solve_fft without a context and without allocating (grids up to 128^3, the
    library's static scratch; calls that overlap on one GPU race on it)."""
    if rho.dim() != 3 or len(set(rho.shape)) != 1:
        raise ValueError("rho must be [n, n, n]")
    n = rho.shape[0]
    st = _lib.pm_solve_fft_noalloc(_ptr(rho, shape=(n, n, n), name="rho"), int(n), float(coef),
                                   int(deconv), _ptr(phi, shape=(n, n, n), name="phi"), _stream())
    if st < 0:
        raise PMError(st, f"pm_solve_fft_noalloc(n={n}) failed")
    return st


def pm_gradient(ctx: Context, phi, g, points=5):
    n = ctx.n
    st = _lib.pm_gradient(ctx.handle, _ptr(phi, shape=(n, n, n), name="phi"), int(points),
                          _ptr(g, shape=(n, n, n, 3), name="g"), _stream())
    return ctx._check(st, "pm_gradient")


def pm_interp(ctx: Context, pos, g, acc, cell=None, mas="tsc"):
    n = ctx.n
    np_, kind, pp, cp = _particles(pos, cell)
    st = _lib.pm_interp(ctx.handle, pp, cp, np_, kind, MAS.get(mas, mas),
                        _ptr(g, shape=(n, n, n, 3), name="g"), _ptr(acc, shape=(np_, 3), name="acc"),
                        _stream())
    return ctx._check(st, "pm_interp")


def pm_accel(ctx: Context, pos, a, phi, acc, cell=None, params: StepParams | None = None):
    n = ctx.n
    np_, kind, pp, cp = _particles(pos, cell)
    params = params or default_step_params()
    stats = StepStats()
    st = _lib.pm_accel(ctx.handle, pp, cp, np_, kind, float(a), byref(params),
                       _ptr(phi, shape=(n, n, n), name="phi"), _ptr(acc, shape=(np_, 3), name="acc"),
                       byref(stats), _stream())
    ctx._check(st, "pm_accel")
    return stats


def pm_kernel_timer(ctx: Context, kernel, capacity=4096):
    kid = {"none": PM_KERNEL_NONE, "deposit": PM_KERNEL_DEPOSIT, "smooth": PM_KERNEL_SMOOTH,
           "interp": PM_KERNEL_INTERP, "fr_sweep": PM_KERNEL_FR_SWEEP}.get(kernel, kernel)
    return ctx._check(_lib.pm_kernel_timer(ctx.handle, int(kid), int(capacity)), "pm_kernel_timer")


def pm_kernel_timer_read(ctx: Context):
    ms, n, b = c_double(), c_int64(), c_double()
    ctx._check(_lib.pm_kernel_timer_read(ctx.handle, byref(ms), byref(n), byref(b)),
               "pm_kernel_timer_read")
    return ms.value, n.value, b.value


def pm_reorder(ctx: Context, pos, vel=None, acc=None, ids=None, cell=None):
    np_, kind, pp, cp = _particles(pos, cell)
    st = _lib.pm_reorder(ctx.handle, pp, cp, _ptr(vel, shape=(np_, 3), name="vel"),
                         _ptr(acc, shape=(np_, 3), name="acc"),
                         _ptr(ids, torch.int64, (np_,), "ids"), np_, kind, _stream())
    return ctx._check(st, "pm_reorder")


def pm_kdk(ctx: Context, pos, vel, a0, a1, phi, acc, cell=None, params: StepParams | None = None):
    n = ctx.n
    np_, kind, pp, cp = _particles(pos, cell)
    params = params or default_step_params()
    stats = StepStats()
    st = _lib.pm_kdk(ctx.handle, pp, cp, _ptr(vel, shape=(np_, 3), name="vel"), np_, kind,
                     float(a0), float(a1), byref(params), _ptr(phi, shape=(n, n, n), name="phi"),
                     _ptr(acc, shape=(np_, 3), name="acc"), byref(stats), _stream())
    ctx._check(st, "pm_kdk")
    return stats


def pm_kdk_chain(ctx: Context, pos, vel, a0, a1, a2, stage, phi, acc, cell=None,
                 params: StepParams | None = None):
    """One step a0 -> a1 of a chain of KDK steps (a2 <= a1: last step); stage is
    PM_CHAIN_FIRST or PM_CHAIN_NEXT (include/hippm.h)."""
    n = ctx.n
    np_, kind, pp, cp = _particles(pos, cell)
    params = params or default_step_params()
    stats = StepStats()
    st = _lib.pm_kdk_chain(ctx.handle, pp, cp, _ptr(vel, shape=(np_, 3), name="vel"), np_, kind,
                           float(a0), float(a1), float(a2), int(stage), byref(params),
                           _ptr(phi, shape=(n, n, n), name="phi"),
                           _ptr(acc, shape=(np_, 3), name="acc"), byref(stats), _stream())
    ctx._check(st, "pm_kdk_chain")
    return stats


# ------------------------------------------------------------------ reverse mode

def pm_deposit_vjp(ctx: Context, pos, rho_bar, pos_bar, cell=None, mas="tsc"):
    """pos_bar += (d rho / d x)^T rho_bar (box-unit positions)."""
    n = ctx.n
    np_, kind, pp, cp = _particles(pos, cell)
    st = _lib.pm_deposit_vjp(ctx.handle, pp, cp, np_, kind, MAS.get(mas, mas),
                             _ptr(rho_bar, shape=(n, n, n), name="rho_bar"),
                             _ptr(pos_bar, shape=(np_, 3), name="pos_bar"), _stream())
    return ctx._check(st, "pm_deposit_vjp")


def pm_interp_vjp(ctx: Context, pos, lam, g=None, g_bar=None, pos_bar=None, cell=None, mas="tsc"):
    """g_bar += interp^T lam; pos_bar += (d interp / d x)^T lam at the field g."""
    n = ctx.n
    np_, kind, pp, cp = _particles(pos, cell)
    st = _lib.pm_interp_vjp(ctx.handle, pp, cp, np_, kind, MAS.get(mas, mas),
                            _ptr(g, shape=(n, n, n, 3), name="g"),
                            _ptr(lam, shape=(np_, 3), name="lam"),
                            _ptr(g_bar, shape=(n, n, n, 3), name="g_bar"),
                            _ptr(pos_bar, shape=(np_, 3), name="pos_bar"), _stream())
    return ctx._check(st, "pm_interp_vjp")


def pm_gradient_vjp(ctx: Context, g_bar, phi_bar, points=5):
    """phi_bar += sum_d D_d g_bar_d."""
    n = ctx.n
    st = _lib.pm_gradient_vjp(ctx.handle, _ptr(g_bar, shape=(n, n, n, 3), name="g_bar"),
                              int(points), _ptr(phi_bar, shape=(n, n, n), name="phi_bar"),
                              _stream())
    return ctx._check(st, "pm_gradient_vjp")


def pm_accel_vjp(ctx: Context, pos, a, phi, lam, pos_bar, scale=1.0, cell=None,
                 params: StepParams | None = None):
    """pos_bar += scale J(x)^T lam, J = d accel / d x at scale factor a; phi = potential of x."""
    n = ctx.n
    np_, kind, pp, cp = _particles(pos, cell)
    params = params or default_step_params()
    stats = MGStats()
    st = _lib.pm_accel_vjp(ctx.handle, pp, cp, np_, kind, float(a), byref(params),
                           _ptr(phi, shape=(n, n, n), name="phi"),
                           _ptr(lam, shape=(np_, 3), name="lam"), float(scale),
                           _ptr(pos_bar, shape=(np_, 3), name="pos_bar"), byref(stats), _stream())
    ctx._check(st, "pm_accel_vjp")
    return stats


def pm_kdk_adjoint(ctx: Context, pos0, phi0, pos1, phi1, a0, a1, pos_bar, vel_bar, a_prev=0.0,
                   closing_merged=False, cell0=None, cell1=None,
                   params: StepParams | None = None):
    """Reverse one KDK step a0 -> a1 in place on (pos_bar, vel_bar). a_prev > 0 merges the
    closing term of the step a_prev -> a0 into this step's opening term; closing_merged
    skips this step's closing term (pos1/phi1 may then be None)."""
    n = ctx.n
    np_, kind, p0, c0 = _particles(pos0, cell0)
    if closing_merged:
        p1 = c1 = None
    else:
        _, kind1, p1, c1 = _particles(pos1, cell1)
        if kind1 != kind or pos1.shape[0] != np_:
            raise ValueError("pos0 and pos1 must have the same form and count")
    params = params or default_step_params()
    stats = StepStats()
    st = _lib.pm_kdk_adjoint(ctx.handle, p0, c0, _ptr(phi0, shape=(n, n, n), name="phi0"),
                             p1, c1, _ptr(phi1, shape=(n, n, n), name="phi1"), np_, kind,
                             float(a_prev), float(a0), float(a1), byref(params),
                             PM_ADJ_CLOSING_MERGED if closing_merged else 0,
                             _ptr(pos_bar, shape=(np_, 3), name="pos_bar"),
                             _ptr(vel_bar, shape=(np_, 3), name="vel_bar"), byref(stats), _stream())
    ctx._check(st, "pm_kdk_adjoint")
    return stats


def pm_density_loss(ctx: Context, pos, w, pos_bar=None, cell=None, mas="tsc", order="sorted",
                    want_loss=True):
    """L = sum_c w (rho - 1)^2 (returned as a float when want_loss); pos_bar += dL/dx."""
    n = ctx.n
    np_, kind, pp, cp = _particles(pos, cell)
    loss = c_double(0.0)
    st = _lib.pm_density_loss(ctx.handle, pp, cp, np_, kind, MAS.get(mas, mas),
                              ORDER.get(order, order), _ptr(w, shape=(n, n, n), name="w"),
                              byref(loss) if want_loss else None,
                              _ptr(pos_bar, shape=(np_, 3), name="pos_bar"), _stream())
    ctx._check(st, "pm_density_loss")
    return loss.value if want_loss else None


def pm_ic_state(ctx: Context, q, psi, a0, pos, vel, cell=None):
    """pos = wrap(q + psi), vel = a0^(1/2) psi (cell-offset form when cell is given)."""
    np_ = q.shape[0]
    st = _lib.pm_ic_state(ctx.handle, _ptr(q, shape=(np_, 3), name="q"),
                          _ptr(psi, shape=(np_, 3), name="psi"), np_, float(a0),
                          _ptr(pos, shape=(np_, 3), name="pos"),
                          _ptr(cell, torch.int32, (np_,), "cell"),
                          _ptr(vel, shape=(np_, 3), name="vel"), _stream())
    return ctx._check(st, "pm_ic_state")


def pm_ic_vjp(ctx: Context, pos_bar, vel_bar, a0, psi_bar):
    """psi_bar = pos_bar + a0^(1/2) vel_bar."""
    np_ = pos_bar.shape[0]
    st = _lib.pm_ic_vjp(ctx.handle, _ptr(pos_bar, shape=(np_, 3), name="pos_bar"),
                        _ptr(vel_bar, shape=(np_, 3), name="vel_bar"), np_, float(a0),
                        _ptr(psi_bar, shape=(np_, 3), name="psi_bar"), _stream())
    return ctx._check(st, "pm_ic_vjp")


def pm_ic_lpt(ctx: Context, noise, k_tab, p_tab, a0, pos, vel, cell=None, order=2, dealias=True):
    """Lagrangian-perturbation-theory initial conditions of the n^3 lattice (order 1..3)
    from a white-noise grid [n, n, n] and a P(k) table (host sequences, a = 1)."""
    n = ctx.n
    np_ = n ** 3
    kt = (c_double * len(k_tab))(*[float(x) for x in k_tab])
    pt = (c_double * len(p_tab))(*[float(x) for x in p_tab])
    if len(k_tab) != len(p_tab):
        raise ValueError("k_tab and p_tab must have the same length")
    st = _lib.pm_ic_lpt(ctx.handle, _ptr(noise, shape=(n, n, n), name="noise"), len(k_tab), kt,
                        pt, int(order), 1 if dealias else 0, float(a0),
                        _ptr(pos, shape=(np_, 3), name="pos"), _ptr(cell, torch.int32, (np_,), "cell"),
                        _ptr(vel, shape=(np_, 3), name="vel"), _stream())
    return ctx._check(st, "pm_ic_lpt")


def pm_power_spectrum(ctx: Context, rho, deconv=3, nbins=None):
    """(P, mean k, modes) per shell rint(|m|) = 1 .. nbins of delta = rho / mean - 1."""
    n = ctx.n
    nbins = n // 2 if nbins is None else int(nbins)
    pk = (c_double * nbins)()
    km = (c_double * nbins)()
    nm = (c_int64 * nbins)()
    st = _lib.pm_power_spectrum(ctx.handle, _ptr(rho, shape=(n, n, n), name="rho"), int(deconv),
                                nbins, pk, km, nm, _stream())
    ctx._check(st, "pm_power_spectrum")
    return list(pk), list(km), list(nm)


# ------------------------------------------------------------------ batched ensembles

class Batch:
    """Owner of a pm_batch: boxes of grid sizes n[b] with np[b] particles each.

    Attributes p_off / c_off (lists of nboxes + 1) give the packing of the particle
    arrays ([sum np, 3]) and of the potential arena ([sum n^3]).
    """

    def __init__(self, n, np_, flags=0):
        nb = len(n)
        if len(np_) != nb:
            raise ValueError("n and np must have the same length")
        h = c_void_p()
        n_arr = (c_int * nb)(*[int(x) for x in n])
        np_arr = (c_int64 * nb)(*[int(x) for x in np_])
        st = _lib.pm_batch_create(byref(h), nb, n_arr, np_arr, int(flags))
        if st != PM_OK:
            raise PMError(st, f"pm_batch_create({nb} boxes) failed")
        self._h = h
        self.n = [int(x) for x in n]
        self.np = [int(x) for x in np_]
        po = (c_int64 * (nb + 1))()
        co = (c_int64 * (nb + 1))()
        _lib.pm_batch_layout(h, po, co)
        self.p_off = list(po)
        self.c_off = list(co)
        self.np_total = self.p_off[-1]
        self.ncell_total = self.c_off[-1]

    def close(self):
        if getattr(self, "_h", None):
            _lib.pm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        if not self._h:
            raise PMError(PM_ERR_ARG, "batch closed")
        return self._h

    def _check(self, st, what):
        if st < 0:
            raise PMError(st, f"{what}: {_lib.pm_batch_last_error(self._h).decode()}")
        return st

    def _parts(self, *ts):
        return [_ptr(t, shape=(self.np_total, 3), name="particle array") for t in ts]

    def _phi(self, phi):
        return _ptr(phi, shape=(self.ncell_total,), name="phi")


def pm_batch_create(n, np_, flags=0) -> Batch:
    return Batch(n, np_, flags)


def pm_batch_accel(batch: Batch, pos, acc, phi, a, params: StepParams, want_relres=False):
    pp, ap = batch._parts(pos, acc)
    rel = (c_double * len(batch.n))() if want_relres else None
    st = _lib.pm_batch_accel(batch.handle, pp, ap, batch._phi(phi), float(a), byref(params), rel,
                             _stream())
    batch._check(st, "pm_batch_accel")
    return list(rel) if want_relres else None


def pm_batch_kdk(batch: Batch, pos, vel, acc, phi, a_list, params: StepParams, use_graph=False):
    pp, vp, ap = batch._parts(pos, vel, acc)
    nsteps = len(a_list) - 1
    a_arr = (c_double * len(a_list))(*[float(x) for x in a_list])
    st = _lib.pm_batch_kdk(batch.handle, pp, vp, ap, batch._phi(phi), nsteps, a_arr, byref(params),
                           1 if use_graph else 0, _stream())
    return batch._check(st, "pm_batch_kdk")


def pm_graph_capture_step(batch: Batch, pos, vel, acc, phi, params: StepParams):
    pp, vp, ap = batch._parts(pos, vel, acc)
    st = _lib.pm_graph_capture_step(batch.handle, pp, vp, ap, batch._phi(phi), byref(params),
                                    _stream())
    return batch._check(st, "pm_graph_capture_step")


def pm_tune(batch: Batch, pos, phi, params: StepParams):
    (pp,) = batch._parts(pos)
    choice = (c_int * 2)()
    st = _lib.pm_tune(batch.handle, pp, batch._phi(phi), byref(params), choice, _stream())
    batch._check(st, "pm_tune")
    return {"smooth_rows": choice[0], "gradient_rows": choice[1]}
