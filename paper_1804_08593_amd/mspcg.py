"""Thin ctypes binding of libmspcg.so (include/mspcg.h).

Argument marshalling only: every step of the solver runs in the HIP library.
PyTorch supplies device memory (complex128 CUDA tensors) and the current
stream.  The library must be built (paper_1804_08593_amd.build); there is no
CPU fallback, and loading fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmspcg.so")

OK, EINVAL, ENOMEM, EHIP, ENOGAUGE, ENOCONV, EBREAKDOWN, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
ESCRATCH = -8
EINTERNAL = -9
NOALLOC_SCRATCH_BYTES = 128 << 20
OP_D, OP_DDAG, OP_HOP, OP_HOPDAG, OP_MHAT, OP_MHATDAG, OP_A, OP_M5INV, OP_PREPARE, OP_KBLOCK = range(10)
FP64, FP32, FP16 = 0, 1, 2
SOLVER_CG, SOLVER_MIXED_CG, SOLVER_MSPCG, SOLVER_MULTISPLIT = 0, 1, 2, 3
FORM_DOMAIN, FORM_SPLIT = 0, 1
KC_HOP64, KC_HOP32, KC_HOPDOM, KC_FIVED, KC_BLAS, KC_HOPCG, KC_HOPDOMCG = range(7)
KC_NAMES = ("hop64", "hop32", "hopdom", "fived", "blas", "hopcg", "hopdomcg")
KC_COUNT = 7
EXPORTS = ("mspcg_create", "mspcg_destroy", "mspcg_strerror", "mspcg_version",
           "mspcg_load_gauge", "mspcg_apply", "mspcg_set_blocking", "mspcg_precond",
           "mspcg_solve", "mspcg_solve_batch", "mspcg_force", "mspcg_get_tuning",
           "mspcg_set_tuning", "mspcg_autotune", "mspcg_tune_blocking",
           "mspcg_get_warnings", "mspcg_gauge_generation", "mspcg_pseudofermion_action",
           "mspcg_apply_noalloc")
WARN_M5_RANGE = 1


class MspcgError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


class Action(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int * 4), ("Ls", ctypes.c_int), ("M5", ctypes.c_double),
                ("mf", ctypes.c_double), ("b", ctypes.c_double), ("c", ctypes.c_double),
                ("antiperiodic_t", ctypes.c_int)]


class Blocking(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int * 4), ("pad", ctypes.c_int), ("form", ctypes.c_int)]


class Tuning(ctypes.Structure):
    _fields_ = [("xcd_remap", ctypes.c_int), ("tile", (ctypes.c_int * 4) * 3)]

    def as_dict(self):
        return {"xcd_remap": self.xcd_remap,
                "tile": {n: list(self.tile[i]) for i, n in enumerate(("fp64", "fp32", "fp16"))}}


class SolveParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int), ("solver", ctypes.c_int),
                ("use_x0", ctypes.c_int), ("blocking", Blocking), ("inner_iters", ctypes.c_int),
                ("inner_prec", ctypes.c_int), ("check_every", ctypes.c_int),
                ("delta", ctypes.c_double), ("timing", ctypes.c_int),
                ("rhs_normal", ctypes.c_int), ("batch_kernels", ctypes.c_int)]


class SolveStats(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int), ("inner_iters_total", ctypes.c_int),
                ("restarts", ctypes.c_int), ("converged", ctypes.c_int),
                ("true_rel_resid", ctypes.c_double), ("seconds", ctypes.c_double),
                ("resid_history", ctypes.POINTER(ctypes.c_double)),
                ("resid_history_cap", ctypes.c_int), ("resid_history_len", ctypes.c_int),
                ("kernel_ms", ctypes.c_double * KC_COUNT),
                ("kernel_launches", ctypes.c_long * KC_COUNT),
                ("kernel_bytes", ctypes.c_double * KC_COUNT),
                ("cg_coef", ctypes.POINTER(ctypes.c_double)),
                ("cg_coef_cap", ctypes.c_int), ("cg_coef_len", ctypes.c_int),
                ("batch_persistent", ctypes.c_int)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libmspcg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with "
                              "`python -m paper_1804_08593_amd.build` (no CPU fallback exists)")
        try:  # share torch's HIP runtime (same soname) when torch is present
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(path)
        P, I = ctypes.c_void_p, ctypes.c_int
        lib.mspcg_create.argtypes = [ctypes.POINTER(Action), I, ctypes.POINTER(P)]
        lib.mspcg_destroy.argtypes = [P]
        lib.mspcg_destroy.restype = None
        lib.mspcg_strerror.argtypes = [I]
        lib.mspcg_strerror.restype = ctypes.c_char_p
        lib.mspcg_version.restype = I
        lib.mspcg_load_gauge.argtypes = [P, P, P]
        lib.mspcg_apply.argtypes = [P, I, I, P, P, P]
        lib.mspcg_apply_noalloc.argtypes = [P, I, I, P, P, P]
        lib.mspcg_set_blocking.argtypes = [P, ctypes.POINTER(Blocking)]
        lib.mspcg_precond.argtypes = [P, I, I, P, P, P]
        lib.mspcg_solve.argtypes = [P, P, P, ctypes.POINTER(SolveParams),
                                    ctypes.POINTER(SolveStats), P]
        lib.mspcg_solve_batch.argtypes = [ctypes.POINTER(P), I, ctypes.POINTER(P),
                                          ctypes.POINTER(P), ctypes.POINTER(SolveParams),
                                          ctypes.POINTER(SolveStats), P]
        lib.mspcg_force.argtypes = [P, P, P, P, P, P]
        lib.mspcg_get_warnings.argtypes = [P, ctypes.POINTER(I)]
        lib.mspcg_gauge_generation.argtypes = [P, ctypes.POINTER(ctypes.c_ulonglong)]
        lib.mspcg_pseudofermion_action.argtypes = [P, P, P, P, ctypes.POINTER(SolveParams),
                                                   ctypes.POINTER(ctypes.c_double),
                                                   ctypes.POINTER(SolveStats), P]
        lib.mspcg_get_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
        lib.mspcg_set_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
        lib.mspcg_autotune.argtypes = [P, ctypes.POINTER(Blocking), ctypes.c_char_p, P]
        lib.mspcg_tune_blocking.argtypes = [P, ctypes.POINTER(SolveParams), I,
                                            ctypes.POINTER(Blocking), P]
        _lib = lib
    return _lib


def strerror(code: int) -> str:
    return load().mspcg_strerror(int(code)).decode()


def _check(code: int, where: str, allow=()):
    if code != OK and code not in allow:
        raise MspcgError(code, where)
    return code


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t, numel=None, device=None):
    """Device pointer of a field, after the checks the C ABI cannot make on a
    bare pointer: complex128, on a HIP device, contiguous and, when given, the
    element count and device index the context expects."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.complex128:
        raise TypeError("fields are complex128 tensors on a HIP device")
    if not t.is_contiguous():
        raise ValueError("fields must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"field has {t.numel()} elements where the context expects {numel}")
    if device is not None and t.device.index != device:
        raise ValueError(f"field is on device {t.device.index}, the context on device {device}")
    return ctypes.c_void_p(t.data_ptr())


def make_params(tol=1e-10, maxiter=10000, solver=SOLVER_CG, use_x0=False, block=(0, 0, 0, 0),
                pad=2, inner_iters=6, inner_prec=FP16, check_every=0, delta=0.1,
                timing=False, rhs_normal=False, form=FORM_DOMAIN, batch_kernels=0) -> SolveParams:
    p = SolveParams()
    p.tol, p.maxiter, p.solver, p.use_x0 = float(tol), int(maxiter), int(solver), int(use_x0)
    for i in range(4):
        p.blocking.block[i] = int(block[i])
    p.blocking.pad = int(pad)
    p.blocking.form = int(form)
    p.inner_iters, p.inner_prec = int(inner_iters), int(inner_prec)
    p.check_every, p.delta, p.timing = int(check_every), float(delta), int(timing)
    p.rhs_normal = int(bool(rhs_normal))
    p.batch_kernels = int(batch_kernels)
    return p


class Context:
    """One action on one device (mspcg_ctx)."""

    def __init__(self, dims, Ls, M5, mf, b=1.0, c=0.0, antiperiodic_t=True, device=0):
        lib = load()
        a = Action()
        for i in range(4):
            a.dims[i] = int(dims[i])
        a.Ls, a.M5, a.mf, a.b, a.c = int(Ls), float(M5), float(mf), float(b), float(c)
        a.antiperiodic_t = int(bool(antiperiodic_t))
        h = ctypes.c_void_p()
        _check(lib.mspcg_create(ctypes.byref(a), int(device), ctypes.byref(h)), "mspcg_create")
        self._h = h
        self.dims = tuple(int(x) for x in dims)
        self.Ls = int(Ls)
        self.device = int(device)
        w = ctypes.c_int()
        _check(lib.mspcg_get_warnings(h, ctypes.byref(w)), "mspcg_get_warnings")
        self.warnings = w.value
        if w.value & WARN_M5_RANGE:
            import warnings
            warnings.warn(f"M5 = {M5} lies outside (0, 2): the operator has no wall-bound "
                          "light mode", RuntimeWarning, stacklevel=2)

    @property
    def gauge_generation(self) -> int:
        g = ctypes.c_ulonglong()
        _check(load().mspcg_gauge_generation(self._h, ctypes.byref(g)), "mspcg_gauge_generation")
        return g.value

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().mspcg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def fshape(self):
        Lx, Ly, Lz, Lt = self.dims
        return (self.Ls, Lt, Lz, Ly, Lx, 4, 3)

    @property
    def gshape(self):
        Lx, Ly, Lz, Lt = self.dims
        return (4, Lt, Lz, Ly, Lx, 3, 3)

    def _f(self, t):
        """Pointer of a fermion field of this context (checked)."""
        return _ptr(t, int(np.prod(self.fshape)), self.device)

    def _g(self, t):
        """Pointer of a link field of this context (checked)."""
        return _ptr(t, int(np.prod(self.gshape)), self.device)

    def load_gauge(self, U, stream=None):
        _check(load().mspcg_load_gauge(self._h, self._g(U), _stream(stream)), "mspcg_load_gauge")

    def apply(self, op, inp, out, prec=FP64, stream=None):
        _check(load().mspcg_apply(self._h, int(op), int(prec), self._f(inp), self._f(out),
                                  _stream(stream)), "mspcg_apply")
        return out

    def apply_noalloc(self, op, inp, out, prec=FP64, stream=None):
        """mspcg_apply without device allocation (fixed per-GPU scratch)."""
        _check(load().mspcg_apply_noalloc(self._h, int(op), int(prec), self._f(inp), self._f(out),
                                          _stream(stream)), "mspcg_apply_noalloc")
        return out

    def set_blocking(self, block, pad=2, form=FORM_DOMAIN):
        b = Blocking()
        for i in range(4):
            b.block[i] = int(block[i])
        b.pad = int(pad)
        b.form = int(form)
        _check(load().mspcg_set_blocking(self._h, ctypes.byref(b)), "mspcg_set_blocking")

    def precond(self, r, z, inner_iters, prec=FP16, stream=None):
        _check(load().mspcg_precond(self._h, int(inner_iters), int(prec), self._f(r), self._f(z),
                                    _stream(stream)), "mspcg_precond")
        return z

    def solve(self, b, x, params: SolveParams, history=0, stream=None, allow_noconv=False,
              coef=0):
        """history / coef: iterations of residual history / (P)CG coefficients to return."""
        st = SolveStats()
        hist = cf = None
        if history:
            hist = (ctypes.c_double * int(history))()
            st.resid_history = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
            st.resid_history_cap = int(history)
        if coef:
            cf = (ctypes.c_double * (2 * int(coef)))()
            st.cg_coef = ctypes.cast(cf, ctypes.POINTER(ctypes.c_double))
            st.cg_coef_cap = int(coef)
        rc = load().mspcg_solve(self._h, self._f(b), self._f(x), ctypes.byref(params),
                                ctypes.byref(st), _stream(stream))
        _check(rc, "mspcg_solve", allow=(ENOCONV,) if allow_noconv else ())
        return stats_dict(st, hist, rc, cf)

    def pseudofermion_action(self, phi, X, dphi=None, params: SolveParams = None, stream=None,
                             allow_noconv=False):
        """S = phi^+ A^-1 phi; X receives A^-1 phi, dphi (optional) 2 X."""
        p = params if params is not None else make_params(tol=1e-12, maxiter=20000)
        S = ctypes.c_double()
        st = SolveStats()
        rc = load().mspcg_pseudofermion_action(self._h, self._f(phi), self._f(X),
                                               self._f(dphi) if dphi is not None else None,
                                               ctypes.byref(p), ctypes.byref(S),
                                               ctypes.byref(st), _stream(stream))
        _check(rc, "mspcg_pseudofermion_action", allow=(ENOCONV,) if allow_noconv else ())
        return S.value, stats_dict(st, None, rc)

    def get_tuning(self) -> Tuning:
        t = Tuning()
        _check(load().mspcg_get_tuning(self._h, ctypes.byref(t)), "mspcg_get_tuning")
        return t

    def set_tuning(self, xcd_remap=1, fp64=(0, 0, 0, 0), fp32=(0, 0, 0, 0), fp16=(0, 0, 0, 0)):
        t = Tuning()
        t.xcd_remap = int(xcd_remap)
        for i, tl in enumerate((fp64, fp32, fp16)):
            for m in range(4):
                t.tile[i][m] = int(tl[m])
        _check(load().mspcg_set_tuning(self._h, ctypes.byref(t)), "mspcg_set_tuning")

    def autotune(self, block=None, pad=2, cache_path=None, stream=None) -> dict:
        b = None
        if block is not None:
            b = Blocking()
            for i in range(4):
                b.block[i] = int(block[i])
            b.pad = int(pad)
        _check(load().mspcg_autotune(self._h, ctypes.byref(b) if b is not None else None,
                                     cache_path.encode() if cache_path else None,
                                     _stream(stream)), "mspcg_autotune")
        return self.get_tuning().as_dict()

    def tune_blocking(self, params: "SolveParams" = None, probe_iters=8, stream=None):
        """Pick the MSPCG block shape: fastest residual reduction per second over
        probe_iters outer iterations, or (probe_iters = 0) shortest time to
        solve each candidate to params' tolerance."""
        p = params if params is not None else make_params(solver=SOLVER_MSPCG)
        b = Blocking()
        _check(load().mspcg_tune_blocking(self._h, ctypes.byref(p), int(probe_iters),
                                          ctypes.byref(b), _stream(stream)), "mspcg_tune_blocking")
        return tuple(b.block), b.pad

    def force(self, X, Y, F=None, G=None, stream=None):
        """F: traceless Hermitian force per link; G: gradient w.r.t. the complex link."""
        _check(load().mspcg_force(self._h, self._f(X), self._f(Y),
                                  self._g(F) if F is not None else None,
                                  self._g(G) if G is not None else None, _stream(stream)),
               "mspcg_force")
        return F, G


def stats_dict(st: SolveStats, hist=None, rc=OK, coef=None) -> dict:
    d = {
        "rc": rc,
        "outer_iters": st.outer_iters,
        "inner_iters_total": st.inner_iters_total,
        "restarts": st.restarts,
        "converged": bool(st.converged),
        "true_rel_resid": st.true_rel_resid,
        "seconds": st.seconds,
        "batch_persistent": bool(st.batch_persistent),
        "kernel_ms": {KC_NAMES[i]: st.kernel_ms[i] for i in range(KC_COUNT)},
        "kernel_launches": {KC_NAMES[i]: int(st.kernel_launches[i]) for i in range(KC_COUNT)},
        "kernel_bytes": {KC_NAMES[i]: st.kernel_bytes[i] for i in range(KC_COUNT)},
    }
    if hist is not None:
        d["history"] = np.array(hist[:st.resid_history_len])
    if coef is not None:
        d["cg_coef"] = np.array(coef[:2 * st.cg_coef_len]).reshape(-1, 2)
    return d


def solve_batch(ctxs, bs, xs, params: SolveParams, history=0, stream=None, allow_noconv=False):
    """Solve n independent systems together (hipGraph-replayed outer iterations)."""
    n = len(ctxs)
    if len(bs) != n or len(xs) != n:
        raise ValueError("one right-hand side and one solution per context")
    H = (ctypes.c_void_p * n)(*[c.handle for c in ctxs])
    B = (ctypes.c_void_p * n)(*[c._f(b) for c, b in zip(ctxs, bs)])
    X = (ctypes.c_void_p * n)(*[c._f(x) for c, x in zip(ctxs, xs)])
    sts = (SolveStats * n)()
    hists = []
    for i in range(n):
        h = None
        if history:
            h = (ctypes.c_double * int(history))()
            sts[i].resid_history = ctypes.cast(h, ctypes.POINTER(ctypes.c_double))
            sts[i].resid_history_cap = int(history)
        hists.append(h)
    rc = load().mspcg_solve_batch(H, n, B, X, ctypes.byref(params), sts, _stream(stream))
    _check(rc, "mspcg_solve_batch", allow=(ENOCONV,) if allow_noconv else ())
    return [stats_dict(sts[i], hists[i], rc) for i in range(n)]
