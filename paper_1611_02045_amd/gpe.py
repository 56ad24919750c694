"""Thin Python binding of libgpe (the C ABI declared in include/gpe.h).

Argument marshalling only: every computation runs in the HIP kernels of libgpe.so.  PyTorch is
used for device memory (tensors) and streams; fields are passed as raw device pointers.
The binding refuses to run without the built library (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgpe.so")

F64, F32 = 0, 1
PRECONDS = {"none": 0, "kinetic": 1, "potential": 2, "combined": 3, "c1": 4, "c2": 5}
STATUS = {0: "ok", 1: "not_converged", -1: "einval", -2: "eunsupported", -3: "ehip", -4: "enonfinite",
          -5: "elinesearch"}


class GpeError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"libgpe error {status} ({STATUS.get(status, '?')}): {message}")
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("L", ctypes.c_double * 3),
                ("beta", ctypes.c_double), ("omega", ctypes.c_double)]


class PcgOpts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("precond", ctypes.c_int32), ("tol_res_inf", ctypes.c_double),
                ("tol_energy", ctypes.c_double), ("max_iter", ctypes.c_int64), ("precision", ctypes.c_int32),
                ("beta_rule", ctypes.c_int32), ("switch_res", ctypes.c_double), ("theta_default", ctypes.c_double),
                ("max_halvings", ctypes.c_int32), ("refresh_every", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("record_history", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("line_search", ctypes.c_int32)]


class PcgReport(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("switched", ctypes.c_int32), ("iters", ctypes.c_int64),
                ("iters_fp32", ctypes.c_int64), ("restarts", ctypes.c_int64), ("halvings", ctypes.c_int64),
                ("E", ctypes.c_double), ("lam", ctypes.c_double), ("res_inf", ctypes.c_double),
                ("dE", ctypes.c_double), ("dphi_inf", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self) -> dict:
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["status_name"] = STATUS.get(self.status, str(self.status))
        return d


# C entry points: name -> (restype, argtypes)
_VP, _I, _D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
SIGNATURES = {
    "gpe_plan_create": (_I, [ctypes.POINTER(Problem), _I, ctypes.POINTER(_VP)]),
    "gpe_plan_destroy": (_I, [_VP]),
    "gpe_energy": (_I, [_VP, _VP, _VP, ctypes.POINTER(_D), ctypes.POINTER(_D), _VP]),
    "gpe_apply_H": (_I, [_VP, _VP, _VP, _VP, _VP]),
    "gpe_apply_H_batched": (_I, [_VP, _I, _VP, _VP, _VP, _VP]),
    "gpe_apply_H_batched_noalloc": (_I, [_VP, _I, _VP, _VP, _VP, _VP]),
    "gpe_set_apply_kernel": (_I, [_I]),
    "gpe_apply_kernel_for": (_I, [_VP, _I, ctypes.POINTER(_I)]),
    "gpe_precond": (_I, [_VP, _I, _VP, _VP, _D, _VP, _VP, _VP]),
    "gpe_pcg_opts_default": (None, [ctypes.POINTER(PcgOpts)]),
    "gpe_pcg_solve": (_I, [_VP, _VP, _VP, ctypes.POINTER(PcgOpts), ctypes.POINTER(PcgReport), _VP]),
    "gpe_pcg_history": (_I, [_VP, ctypes.POINTER(_D), _I]),
    "gpe_pcg_solve_batched": (_I, [_I, ctypes.POINTER(Problem), _I, ctypes.POINTER(_VP), ctypes.POINTER(_VP),
                                   ctypes.POINTER(PcgOpts), ctypes.POINTER(PcgReport), _VP]),
    "gpe_prolong": (_I, [_VP, _VP, _VP, _VP]),
    "gpe_autotune": (_I, [_VP, _I, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_D), _VP]),
    "gpe_be_solve": (_I, [_VP, _VP, _VP, _D, _I, ctypes.POINTER(PcgOpts), _D, ctypes.POINTER(ctypes.c_int64),
                          ctypes.POINTER(PcgReport), _VP]),
    "gpe_pcg_solve_nested": (_I, [_I, _I, ctypes.POINTER(Problem), _I, ctypes.POINTER(_VP), ctypes.POINTER(_VP),
                                  ctypes.POINTER(_VP), ctypes.POINTER(PcgOpts), _D, ctypes.POINTER(PcgReport), _VP]),
    "gpe_energy_grad": (_I, [_VP, _VP, _VP, _VP, _VP, ctypes.POINTER(_D), ctypes.POINTER(_D), _VP]),
    "gpe_adjoint_solve": (_I, [_VP, _VP, _VP, _VP, _VP, ctypes.POINTER(PcgOpts), ctypes.POINTER(PcgReport), _VP]),
    "gpe_adjoint_param_grads": (_I, [_VP, _VP, _VP, _VP, ctypes.POINTER(_D), ctypes.POINTER(_D), _VP]),
    "gpe_pcg_profile": (_I, [_VP, _VP, _VP, ctypes.POINTER(PcgOpts), _I, _I, ctypes.POINTER(_D),
                             ctypes.POINTER(_D), ctypes.c_char_p, _VP]),
    "gpe_pcg_profile_batched": (_I, [_I, ctypes.POINTER(Problem), _I, ctypes.POINTER(_VP), ctypes.POINTER(_VP),
                                     ctypes.POINTER(PcgOpts), _I, _I, ctypes.POINTER(_D), ctypes.POINTER(_D),
                                     ctypes.c_char_p, _VP]),
    "gpe_last_error": (ctypes.c_char_p, []),
    "gpe_version": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libgpe.so (built in-tree); raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1611_02045_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status < 0:
        raise GpeError(status, lib().gpe_last_error().decode())
    return status


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


APPLY_KERNELS = {0: "auto", 1: "passes", 2: "plane"}


def set_apply_kernel(kind: str) -> None:
    """gpe_set_apply_kernel: "auto" (default), "passes" or "plane" for every H apply of the
    process from the next launch on."""
    codes = {v: k for k, v in APPLY_KERNELS.items()}
    if kind not in codes:
        raise ValueError(f"unknown apply kernel {kind!r}")
    _check(lib().gpe_set_apply_kernel(codes[kind]))


def make_problem(dim: int, n, L, beta: float, omega: float) -> Problem:
    p = Problem()
    p.dim = dim
    n = list(n) + [1] * (3 - len(n))
    L = list(L) + [1.0] * (3 - len(L))
    for a in range(3):
        p.n[a] = int(n[a])
        p.L[a] = float(L[a])
    p.beta = float(beta)
    p.omega = float(omega)
    return p


def default_opts(**kw) -> PcgOpts:
    """gpe_pcg_opts_t with the library's defaults, overridden by keyword: any field of PcgOpts, plus
    the aliases tol / tol_res (tol_res_inf) and names for the enumerations: precond ("none",
    "kinetic", "potential", "combined", "c1", "c2"), method ("pg", "pcg"), precision ("fp64",
    "mixed"), beta_rule ("pr", "fr"), line_search ("heuristic", "armijo", "full", "wolfe")."""
    o = PcgOpts()
    lib().gpe_pcg_opts_default(ctypes.byref(o))
    alias = {"tol": "tol_res_inf", "tol_res": "tol_res_inf"}
    for k, v in kw.items():
        k = alias.get(k, k)
        if k == "precond" and isinstance(v, str):
            v = PRECONDS[v]
        if k == "method" and isinstance(v, str):
            v = {"pg": 0, "pcg": 1}[v]
        if k == "precision" and isinstance(v, str):
            v = {"fp64": 0, "mixed": 1}[v]
        if k == "beta_rule" and isinstance(v, str):
            v = {"pr": 0, "fr": 1}[v]
        if k == "line_search" and isinstance(v, str):
            v = {"heuristic": 0, "armijo": 1, "full": 2, "wolfe": 3}[v]
        if not hasattr(o, k):
            raise TypeError(f"unknown solver option {k!r}")
        setattr(o, k, v)
    return o


class Plan:
    """A libgpe plan for one problem: grid (dim, n, L), beta, omega and storage dtype."""

    def __init__(self, dim: int, n, L, beta: float, omega: float, dtype: str = "f64"):
        self.dim = dim
        self.n = tuple(int(v) for v in n)[:dim]
        self.L = tuple(float(v) for v in L)[:dim]
        self.beta = float(beta)
        self.omega = float(omega)
        self.dtype = dtype
        self.shape = tuple(reversed(self.n))
        self.real_dtype = torch.float64 if dtype == "f64" else torch.float32
        self.complex_dtype = torch.complex128 if dtype == "f64" else torch.complex64
        self._prob = make_problem(dim, self.n, self.L, beta, omega)
        h = ctypes.c_void_p()
        _check(lib().gpe_plan_create(ctypes.byref(self._prob), F64 if dtype == "f64" else F32, ctypes.byref(h)))
        self._h = h

    @classmethod
    def from_problem(cls, prob, dtype: str = "f64"):
        return cls(prob.dim, prob.n, prob.L, prob.beta, prob.omega, dtype)

    def close(self):
        if getattr(self, "_h", None):
            lib().gpe_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- argument checks -------------------------------------------------------------------
    def _field(self, t: torch.Tensor, name: str, complex_: bool = True, batch: int | None = None):
        want = self.complex_dtype if complex_ else self.real_dtype
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA (HIP) tensor")
        if t.dtype != want:
            raise TypeError(f"{name} must have dtype {want}, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        shape = self.shape if batch is None else (batch,) + self.shape
        if tuple(t.shape) != shape:
            raise ValueError(f"{name} must have shape {shape}, got {tuple(t.shape)}")
        return ctypes.c_void_p(t.data_ptr())

    # -- operators ---------------------------------------------------------------------------
    def energy(self, phi, V, parts: bool = False, stream=None):
        E = ctypes.c_double()
        P = (ctypes.c_double * 4)()
        _check(lib().gpe_energy(self._h, self._field(phi, "phi"), self._field(V, "V", False), ctypes.byref(E), P,
                                _stream(stream)))
        if parts:
            return E.value, {"kinetic": P[0], "potential": P[1], "interaction": P[2], "rotation": P[3]}
        return E.value

    def apply_H(self, phi, V, out=None, stream=None):
        if out is None:
            out = torch.empty_like(phi)
        _check(lib().gpe_apply_H(self._h, self._field(phi, "phi"), self._field(V, "V", False),
                                 self._field(out, "out"), _stream(stream)))
        return out

    def apply_H_batched(self, phi, V, out=None, stream=None):
        count = int(phi.shape[0])
        if out is None:
            out = torch.empty_like(phi)
        _check(lib().gpe_apply_H_batched(self._h, count, self._field(phi, "phi", batch=count),
                                         self._field(V, "V", False), self._field(out, "out", batch=count),
                                         _stream(stream)))
        return out

    def apply_H_batched_noalloc(self, phi, V, out, stream=None):
        """gpe_apply_H_batched_noalloc: the batched apply with its intermediate in the library's
        static device scratch (no allocation; `out` must be given)."""
        count = int(phi.shape[0])
        _check(lib().gpe_apply_H_batched_noalloc(self._h, count, self._field(phi, "phi", batch=count),
                                                 self._field(V, "V", False), self._field(out, "out", batch=count),
                                                 _stream(stream)))
        return out

    def apply_kernel_for(self, count: int = 1) -> str:
        """gpe_apply_kernel_for: "plane" or "passes", the kernel an apply of `count` fields runs."""
        k = _I()
        _check(lib().gpe_apply_kernel_for(self._h, int(count), ctypes.byref(k)))
        return APPLY_KERNELS[k.value]

    def autotune(self, count: int = 1, stream=None):
        """Measure and record the fastest lines per workgroup of each axis's pass for batches of
        `count` fields: returns ([tile per axis], [microseconds per pass])."""
        t = (ctypes.c_int * 3)()
        u = (ctypes.c_double * 3)()
        _check(lib().gpe_autotune(self._h, int(count), t, u, _stream(stream)))
        return list(t)[: len(self.shape)], list(u)[: len(self.shape)]

    def prolong(self, phi, out=None, stream=None):
        """phi interpolated onto the grid with twice the points per axis (same box)."""
        fine = tuple(2 * m for m in self.shape)
        if out is None:
            out = torch.empty(fine, dtype=self.complex_dtype, device=phi.device)
        if (not isinstance(out, torch.Tensor) or not out.is_cuda or out.dtype != self.complex_dtype
                or not out.is_contiguous() or tuple(out.shape) != fine):
            raise ValueError(f"out must be a contiguous {self.complex_dtype} device tensor of shape {fine}")
        _check(lib().gpe_prolong(self._h, self._field(phi, "phi"), ctypes.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def precond(self, kind: str, phi, V, r, alpha: float | None = None, out=None, stream=None):
        if out is None:
            out = torch.empty_like(r)
        a = math.nan if alpha is None else float(alpha)
        _check(lib().gpe_precond(self._h, PRECONDS[kind], self._field(phi, "phi"), self._field(V, "V", False), a,
                                 self._field(r, "r"), self._field(out, "out"), _stream(stream)))
        return out

    def energy_grad(self, phi, V, want_V: bool = True, stream=None):
        gphi = torch.empty_like(phi)
        gV = torch.empty(self.shape, dtype=self.real_dtype, device=phi.device) if want_V else None
        db = ctypes.c_double()
        do = ctypes.c_double()
        _check(lib().gpe_energy_grad(self._h, self._field(phi, "phi"), self._field(V, "V", False),
                                     self._field(gphi, "grad_phi"),
                                     self._field(gV, "grad_V", False) if gV is not None else None,
                                     ctypes.byref(db), ctypes.byref(do), _stream(stream)))
        return gphi, gV, db.value, do.value

    # -- solver ---------------------------------------------------------------------------------
    def pcg_solve(self, V, phi, stream=None, **opts):
        """Solve in place (phi is overwritten by the final iterate); returns the report dict.  opts: see
        default_opts."""
        o = default_opts(**opts)
        rep = PcgReport()
        st = lib().gpe_pcg_solve(self._h, self._field(V, "V", False), self._field(phi, "phi"), ctypes.byref(o),
                                 ctypes.byref(rep), _stream(stream))
        _check(st)
        return rep.as_dict()

    def be_solve(self, V, phi, dt: float, lambda_term: bool = True, inner_tol: float = 1e-10, stream=None, **opts):
        """Backward Euler ground-state iteration (phi updated in place); the report carries
        `inner_iters`, the total of inner CG iterations."""
        o = default_opts(**opts)
        rep = PcgReport()
        inner = ctypes.c_int64(0)
        st = lib().gpe_be_solve(self._h, self._field(V, "V", False), self._field(phi, "phi"), float(dt),
                                int(bool(lambda_term)), ctypes.byref(o), float(inner_tol), ctypes.byref(inner),
                                ctypes.byref(rep), _stream(stream))
        _check(st)
        d = rep.as_dict()
        d["inner_iters"] = inner.value
        return d

    def history(self, cap: int = 100000):
        buf = (ctypes.c_double * (8 * cap))()
        n = _check(lib().gpe_pcg_history(self._h, buf, cap))
        keys = ("n", "E", "lam", "res", "theta", "beta", "halvings", "restarted")
        return [dict(zip(keys, buf[8 * i: 8 * i + 8])) for i in range(n)]

    def profile(self, V, phi, iters: int = 20, stream=None, **opts):
        """Per-kernel event timings of `iters` solver iterations: list of (name, avg_ms, bytes)."""
        o = default_opts(**opts)
        cap = 16
        ms = (ctypes.c_double * cap)()
        by = (ctypes.c_double * cap)()
        names = ctypes.create_string_buffer(32 * cap)
        n = _check(lib().gpe_pcg_profile(self._h, self._field(V, "V", False), self._field(phi, "phi"),
                                         ctypes.byref(o), int(iters), cap, ms, by, names, _stream(stream)))
        raw = names.raw
        return [(raw[32 * k: 32 * k + 32].split(b"\0", 1)[0].decode(), ms[k], by[k]) for k in range(n)]

    def adjoint_solve(self, phi_star, V, rhs, stream=None, **opts):
        """mu with A mu = Pi rhs on {phi*, i phi*}^perp (relative residual tolerance `tol`)."""
        opts.setdefault("tol", 1e-10)
        opts.setdefault("max_iter", 5000)
        o = default_opts(**opts)
        rep = PcgReport()
        mu = torch.empty_like(rhs)
        _check(lib().gpe_adjoint_solve(self._h, self._field(phi_star, "phi_star"), self._field(V, "V", False),
                                       self._field(rhs, "rhs"), self._field(mu, "mu"), ctypes.byref(o),
                                       ctypes.byref(rep), _stream(stream)))
        return mu, rep.as_dict()

    def adjoint_param_grads(self, phi_star, mu, stream=None):
        """(grad_V field, dl/dbeta, dl/domega) of the adjoint part -Re<mu, (d_theta H) phi*>."""
        gV = torch.empty(self.shape, dtype=self.real_dtype, device=phi_star.device)
        db = ctypes.c_double()
        do = ctypes.c_double()
        _check(lib().gpe_adjoint_param_grads(self._h, self._field(phi_star, "phi_star"), self._field(mu, "mu"),
                                             self._field(gV, "grad_V", False), ctypes.byref(db), ctypes.byref(do),
                                             _stream(stream)))
        return gV, db.value, do.value


def _batch_args(problems, Vs, phis, dtype):
    count = len(problems)
    P = (Problem * count)(*[make_problem(p.dim, p.n, p.L, p.beta, p.omega) for p in problems])
    want_c = torch.complex128 if dtype == "f64" else torch.complex64
    want_r = torch.float64 if dtype == "f64" else torch.float32
    for V, phi, p in zip(Vs, phis, problems):
        shape = tuple(reversed(tuple(p.n)[:p.dim]))
        if not (V.is_cuda and phi.is_cuda and V.is_contiguous() and phi.is_contiguous()):
            raise ValueError("fields must be contiguous device tensors")
        if V.dtype != want_r or phi.dtype != want_c or tuple(V.shape) != shape or tuple(phi.shape) != shape:
            raise ValueError("field dtype/shape does not match its problem")
    vp = (ctypes.c_void_p * count)(*[V.data_ptr() for V in Vs])
    pp = (ctypes.c_void_p * count)(*[phi.data_ptr() for phi in phis])
    return count, P, vp, pp


def pcg_profile_batched(problems, Vs, phis, dtype: str = "f64", iters: int = 20, stream=None, **opts):
    """Per-kernel timings of `iters` iterations of the instances solved together: (name, avg_ms, bytes)."""
    count, P, vp, pp = _batch_args(problems, Vs, phis, dtype)
    o = default_opts(**opts)
    cap = 16
    ms = (ctypes.c_double * cap)()
    by = (ctypes.c_double * cap)()
    names = ctypes.create_string_buffer(32 * cap)
    n = _check(lib().gpe_pcg_profile_batched(count, P, F64 if dtype == "f64" else F32, vp, pp, ctypes.byref(o),
                                             int(iters), cap, ms, by, names, _stream(stream)))
    raw = names.raw
    return [(raw[32 * k: 32 * k + 32].split(b"\0", 1)[0].decode(), ms[k], by[k]) for k in range(n)]


def pcg_solve_batched(problems, Vs, phis, dtype: str = "f64", stream=None, **opts):
    """Independent solves of several problems in one iteration loop (fields updated in place)."""
    count, P, vp, pp = _batch_args(problems, Vs, phis, dtype)
    o = default_opts(**opts)
    reps = (PcgReport * count)()
    st = lib().gpe_pcg_solve_batched(count, P, F64 if dtype == "f64" else F32, vp, pp, ctypes.byref(o), reps,
                                     _stream(stream))
    _check(st)
    return st, [r.as_dict() for r in reps]


def pcg_solve_nested(problems, Vs_per_level, phis, dtype: str = "f64", tol_coarse: float = 1e-6, stream=None,
                     **opts):
    """Ground states on nested grids: problems[i] is instance i on the coarsest grid, Vs_per_level[l][i]
    its potential on level l (n << l points per axis), phis[i] its start on the coarsest grid.
    Returns (status, finest-level fields, reports[l][i])."""
    count, levels = len(problems), len(Vs_per_level)
    P = (Problem * count)(*[make_problem(p.dim, p.n, p.L, p.beta, p.omega) for p in problems])
    want_c = torch.complex128 if dtype == "f64" else torch.complex64
    want_r = torch.float64 if dtype == "f64" else torch.float32
    Vflat = []
    for lvl, Vl in enumerate(Vs_per_level):
        if len(Vl) != count:
            raise ValueError("one potential per instance and level")
        for V, p in zip(Vl, problems):
            shape = tuple(reversed([m << lvl for m in tuple(p.n)[:p.dim]]))
            if not (V.is_cuda and V.is_contiguous() and V.dtype == want_r and tuple(V.shape) == shape):
                raise ValueError(f"level-{lvl} potential must be a contiguous {want_r} device tensor of shape {shape}")
            Vflat.append(V)
    outs = []
    for phi, p in zip(phis, problems):
        shape = tuple(reversed(tuple(p.n)[:p.dim]))
        if not (phi.is_cuda and phi.is_contiguous() and phi.dtype == want_c and tuple(phi.shape) == shape):
            raise ValueError(f"start must be a contiguous {want_c} device tensor of shape {shape}")
        fine = tuple(m << (levels - 1) for m in shape)
        outs.append(torch.empty(fine, dtype=want_c, device=phi.device))
    vp = (ctypes.c_void_p * len(Vflat))(*[V.data_ptr() for V in Vflat])
    pin = (ctypes.c_void_p * count)(*[phi.data_ptr() for phi in phis])
    pout = (ctypes.c_void_p * count)(*[o.data_ptr() for o in outs])
    o = default_opts(**opts)
    reps = (PcgReport * (levels * count))()
    st = lib().gpe_pcg_solve_nested(count, levels, P, F64 if dtype == "f64" else F32, vp, pin, pout,
                                    ctypes.byref(o), float(tol_coarse), reps, _stream(stream))
    _check(st)
    return st, outs, [[reps[lvl * count + i].as_dict() for i in range(count)] for lvl in range(levels)]
