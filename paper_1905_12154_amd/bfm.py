"""Python binding of ``libbfm.so`` (the C ABI declared in ``include/bfm.h``).

Argument marshalling only: every step of the computation runs in the HIP
library.  Tensors are PyTorch CUDA (ROCm) tensors, contiguous, of the plan's
dtype (float32 or float64); work is enqueued on the current PyTorch stream.
If the library is not built this module raises instead of computing anything
another way.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libbfm.so")

BFM_OK, BFM_EINVAL, BFM_EDEVICE, BFM_ENUMERIC, BFM_EWORKSPACE, BFM_EUNSUPPORTED = range(6)
BFM_F32, BFM_F64 = 0, 1
STATUS_NAMES = {0: "BFM_OK", 1: "BFM_EINVAL", 2: "BFM_EDEVICE", 3: "BFM_ENUMERIC", 4: "BFM_EWORKSPACE",
                5: "BFM_EUNSUPPORTED"}
EXPORTED = ["bfm_params_init", "bfm_plan_create", "bfm_plan_destroy", "bfm_plan_workspace_bytes", "bfm_solve",
            "bfm_ctransform", "bfm_pushforward", "bfm_poisson_neumann", "bfm_grad", "bfm_last_error",
            "bfm_version", "bfm_ctransform_axis", "bfm_trace", "bfm_solve_batched", "bfm_autotune",
            "bfm_plan_tuning", "bfm_plan_set_tuning", "bfm_plan_set_deposit_grid", "bfm_plan_deposit_grid",
            "bfm_autotune_deposit", "bfm_ctransform_pass", "bfm_interpolate",
            "bfm_solve_noalloc", "bfm_grad_batched"]


class BFMError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), message))
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("shape", ctypes.c_int32 * 3), ("dtype", ctypes.c_int32),
                ("max_iters", ctypes.c_int32), ("tol", ctypes.c_double), ("sigma0", ctypes.c_double),
                ("sigma_min", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("alpha1", ctypes.c_double), ("alpha2", ctypes.c_double), ("check_every", ctypes.c_int32),
                ("method", ctypes.c_int32), ("power", ctypes.c_double * 3)]


METHODS = {"bfm": 0, "ga": 1}


class Result(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("status", ctypes.c_int32),
                ("sigma_floor_hits", ctypes.c_int32), ("dual", ctypes.c_double), ("primal", ctypes.c_double),
                ("gap", ctypes.c_double), ("G", ctypes.c_double), ("sigma", ctypes.c_double),
                ("mass_mu", ctypes.c_double), ("mass_nu", ctypes.c_double)]


_lib = None


def lib_path() -> str:
    return _LIB_PATH


def lib():
    """Load libbfm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError("libbfm.so is not built (%s); run `python -m paper_1905_12154_amd.build_lib`"
                               % _LIB_PATH)
        L = ctypes.CDLL(_LIB_PATH)
        vp, sz, i32, dbl = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_double
        P = ctypes.POINTER
        L.bfm_params_init.argtypes = [P(Params), i32, P(i32), i32]
        L.bfm_plan_create.argtypes = [P(Params), P(vp)]
        L.bfm_plan_destroy.argtypes = [vp]
        L.bfm_plan_destroy.restype = None
        L.bfm_plan_workspace_bytes.argtypes = [vp, P(sz)]
        L.bfm_solve.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, sz, vp, P(Result)]
        L.bfm_solve_noalloc.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, P(Result)]
        L.bfm_ctransform.argtypes = [vp, vp, vp, vp, sz, vp]
        L.bfm_pushforward.argtypes = [vp, vp, vp, vp, vp, P(dbl), vp, sz, vp]
        L.bfm_poisson_neumann.argtypes = [vp, vp, vp, P(dbl), vp, sz, vp]
        L.bfm_grad.argtypes = [vp, vp, vp, dbl, vp, vp, vp, sz, vp]
        L.bfm_ctransform_axis.argtypes = [vp, i32, i32, vp, vp, vp]
        L.bfm_autotune.argtypes = [vp, vp, vp, sz, vp]
        L.bfm_plan_tuning.argtypes = [vp, P(i32)]
        L.bfm_plan_set_tuning.argtypes = [vp, P(i32)]
        L.bfm_plan_set_deposit_grid.argtypes = [vp, i32]
        L.bfm_plan_deposit_grid.argtypes = [vp, P(i32)]
        L.bfm_autotune_deposit.argtypes = [vp, vp, vp, vp, sz, vp]
        L.bfm_ctransform_pass.argtypes = [vp, i32, vp, vp, vp, P(ctypes.c_double), vp, sz, vp]
        L.bfm_interpolate.argtypes = [vp, vp, vp, i32, P(ctypes.c_double), vp, vp, sz, vp]
        L.bfm_solve_batched.argtypes = [i32, P(vp), P(vp), P(vp), P(vp), P(vp), P(vp), P(vp), P(sz), i32, vp,
                                        P(Result)]
        L.bfm_trace.argtypes = [vp, vp, sz, P(dbl), i32, P(i32), vp]
        L.bfm_grad_batched.argtypes = [i32, P(vp), P(vp), P(vp), P(dbl), P(vp), P(vp), P(vp), P(sz), vp]
        L.bfm_last_error.argtypes = []
        L.bfm_last_error.restype = ctypes.c_char_p
        L.bfm_version.argtypes = []
        L.bfm_version.restype = ctypes.c_char_p
        for name in EXPORTED:
            if name not in ("bfm_plan_destroy", "bfm_last_error", "bfm_version"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status: int):
    if status != BFM_OK:
        raise BFMError(status, lib().bfm_last_error().decode())


def _dtype_code(dtype) -> int:
    if dtype in (torch.float32, "float32", "f32", BFM_F32):
        return BFM_F32
    if dtype in (torch.float64, "float64", "f64", BFM_F64):
        return BFM_F64
    raise ValueError("dtype must be float32 or float64")


def _torch_dtype(code: int):
    return torch.float64 if code == BFM_F64 else torch.float32


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Plan:
    """Host plan for one grid shape and dtype (``bfm_plan_create``) plus a
    cached device workspace."""

    def __init__(self, shape: Sequence[int], dtype=torch.float32, max_iters: int = 60, tol: float = 0.0,
                 sigma0: float = 0.0, sigma_min: float = 0.01, beta1: float = 0.25, beta2: float = 0.75,
                 alpha1: float = 1.25, alpha2: float = 0.8, check_every: int = 8, method: str = "bfm",
                 power: Optional[Sequence[float]] = None):
        L = lib()
        if method not in METHODS:
            raise ValueError("method must be one of %s" % sorted(METHODS))
        self.shape = tuple(int(s) for s in shape)
        self.code = _dtype_code(dtype)
        self.dtype = _torch_dtype(self.code)
        p = Params()
        shp = (ctypes.c_int32 * 3)(*(list(self.shape) + [1] * (3 - len(self.shape))))
        _check(L.bfm_params_init(ctypes.byref(p), len(self.shape), shp, self.code))
        p.max_iters, p.tol, p.sigma0, p.sigma_min = int(max_iters), float(tol), float(sigma0), float(sigma_min)
        p.beta1, p.beta2, p.alpha1, p.alpha2 = float(beta1), float(beta2), float(alpha1), float(alpha2)
        p.check_every = int(check_every)
        p.method = METHODS[method]
        self.method = method
        if power is not None:
            pw = [float(x) for x in power]
            if len(pw) != len(self.shape):
                raise ValueError("power needs one exponent per axis (%d), got %d" % (len(self.shape), len(pw)))
            for a, x in enumerate(pw):
                p.power[a] = x
        self.power = tuple(p.power[a] for a in range(len(self.shape)))
        self.params = p
        h = ctypes.c_void_p()
        _check(L.bfm_plan_create(ctypes.byref(p), ctypes.byref(h)))
        self._h = h
        nb = ctypes.c_size_t()
        _check(L.bfm_plan_workspace_bytes(h, ctypes.byref(nb)))
        self.ws_bytes = int(nb.value)
        self._ws = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.bfm_plan_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def workspace(self, device) -> torch.Tensor:
        device = torch.device(device)
        ws = self._ws.get(device)
        if ws is None:
            ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)
            self._ws[device] = ws
        off = (-ws.data_ptr()) % 256
        return ws[off:off + self.ws_bytes]

    def _field(self, t: torch.Tensor, name: str) -> torch.Tensor:
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError("%s must be a CUDA (HIP) tensor" % name)
        if tuple(t.shape) != self.shape:
            raise ValueError("%s has shape %s, plan is %s" % (name, tuple(t.shape), self.shape))
        if t.dtype != self.dtype:
            raise TypeError("%s has dtype %s, plan is %s" % (name, t.dtype, self.dtype))
        return t.contiguous()

    # -- entry points --------------------------------------------------
    def solve(self, mu, nu, phi_init=None, return_map: bool = True):
        mu = self._field(mu, "mu")
        nu = self._field(nu, "nu")
        dev = mu.device
        pi = None if phi_init is None else self._field(phi_init, "phi_init")
        phi = torch.empty_like(mu)
        psi = torch.empty_like(mu)
        T = torch.empty((len(self.shape),) + self.shape, dtype=self.dtype, device=dev) if return_map else None
        ws = self.workspace(dev)
        res = Result()
        _check(lib().bfm_solve(self._h, _ptr(mu), _ptr(nu), _ptr(pi), _ptr(phi), _ptr(psi), _ptr(T),
                               _ptr(ws), self.ws_bytes, _stream(dev), ctypes.byref(res)))
        return SolveResult(phi=phi, psi=psi, T=T, dual=res.dual, primal=res.primal, gap=res.gap, G=res.G,
                           sigma=res.sigma, iters=res.iters, converged=bool(res.converged),
                           mass_mu=res.mass_mu, mass_nu=res.mass_nu, sigma_floor_hits=res.sigma_floor_hits)

    def autotune(self, device="cuda:0", sample: Optional[torch.Tensor] = None):
        """Time the c-transform launch shapes per axis (on ``sample``, a
        potential of the plan's shape, when given) and keep the fastest."""
        if sample is not None:
            sample = self._field(sample, "sample")
            device = sample.device
        ws = self.workspace(device)
        _check(lib().bfm_autotune(self._h, _ptr(sample), _ptr(ws), self.ws_bytes, _stream(torch.device(device))))
        return self.tuning()

    def tuning(self):
        cfg = (ctypes.c_int32 * 9)()
        _check(lib().bfm_plan_tuning(self._h, cfg))
        return [(cfg[3 * a], cfg[3 * a + 1], cfg[3 * a + 2]) for a in range(len(self.shape))]

    def set_tuning(self, cfg):
        """Set the launch shapes: per axis (points per lane, lines per
        workgroup, mode), as returned by ``tuning``."""
        flat = (ctypes.c_int32 * 9)()
        for a, tri in enumerate(cfg):
            for k in range(3):
                flat[3 * a + k] = int(tri[k])
        _check(lib().bfm_plan_set_tuning(self._h, flat))

    def autotune_deposit(self, phi, mass):
        """Time the deposition's workgroup counts on phi^c of ``phi`` and the
        density ``mass`` (the problem's own: the best count depends on its
        support and map) and keep the fastest; returns the count."""
        phi = self._field(phi, "phi")
        mass = self._field(mass, "mass")
        ws = self.workspace(mass.device)
        _check(lib().bfm_autotune_deposit(self._h, _ptr(phi), _ptr(mass), _ptr(ws), self.ws_bytes,
                                          _stream(mass.device)))
        return self.deposit_grid()

    def deposit_grid(self) -> int:
        n = ctypes.c_int32()
        _check(lib().bfm_plan_deposit_grid(self._h, ctypes.byref(n)))
        return n.value

    def set_deposit_grid(self, workgroups: int):
        """Deposition workgroups: 0 (built-in) or a multiple of 8 up to 8192."""
        _check(lib().bfm_plan_set_deposit_grid(self._h, int(workgroups)))

    def interpolate(self, phi, mu, times):
        """Displacement interpolants rho_t = S_t # mu, S_t = t T + (1 - t) id,
        for each t in ``times`` (``bfm_interpolate``); T is the map of phi."""
        phi = self._field(phi, "phi")
        mu = self._field(mu, "mu")
        ts = [float(t) for t in times]
        out = torch.empty((len(ts),) + self.shape, dtype=self.dtype, device=mu.device)
        arr = (ctypes.c_double * max(1, len(ts)))(*ts)
        ws = self.workspace(mu.device)
        _check(lib().bfm_interpolate(self._h, _ptr(phi), _ptr(mu), len(ts), arr, _ptr(out), _ptr(ws), self.ws_bytes,
                                     _stream(mu.device)))
        return out

    def ctransform_pass(self, f, pass_: int, out=None, weight=None, want_sum: bool = False):
        """One pass of the column-blocked 2D transform (``bfm_ctransform_pass``):
        pass 0 maps a row-major field to the column-blocked column pass of -f,
        pass 1 a column-blocked field to the row-major transform; with
        ``weight`` and ``want_sum`` also returns sum(out * weight)."""
        f = self._field(f, "f")
        out = torch.empty_like(f) if out is None else out
        w = None if weight is None else self._field(weight, "weight")
        ws = self.workspace(f.device)
        total = ctypes.c_double()
        _check(lib().bfm_ctransform_pass(self._h, int(pass_), _ptr(f), _ptr(out), _ptr(w),
                                         ctypes.byref(total) if want_sum else None, _ptr(ws), self.ws_bytes,
                                         _stream(f.device)))
        return (out, total.value) if want_sum else out

    def ctransform_axis(self, f, axis: int, sign: int = -1, out=None):
        f = self._field(f, "f")
        out = torch.empty_like(f) if out is None else out
        _check(lib().bfm_ctransform_axis(self._h, int(axis), int(sign), _ptr(f), _ptr(out), _stream(f.device)))
        return out

    def trace(self, device) -> List[dict]:
        """Per-iteration records of the last solve on this plan's workspace."""
        ws = self.workspace(device)
        cnt = ctypes.c_int32()
        _check(lib().bfm_trace(self._h, _ptr(ws), self.ws_bytes, None, 0, ctypes.byref(cnt), _stream(device)))
        m = min(int(cnt.value), 4096)
        buf = (ctypes.c_double * (8 * max(m, 1)))()
        _check(lib().bfm_trace(self._h, _ptr(ws), self.ws_bytes, buf, m, ctypes.byref(cnt), _stream(device)))
        keys = ("iter", "dual", "primal", "G", "gap", "sigma", "J_half", "I_new")
        return [dict(zip(keys, buf[8 * r:8 * r + 8])) for r in range(m)]

    def ctransform(self, f, out=None):
        f = self._field(f, "f")
        out = torch.empty_like(f) if out is None else out
        ws = self.workspace(f.device)
        _check(lib().bfm_ctransform(self._h, _ptr(f), _ptr(out), _ptr(ws), self.ws_bytes, _stream(f.device)))
        return out

    def pushforward(self, phic, mass, return_map: bool = True):
        phic = self._field(phic, "phic")
        mass = self._field(mass, "mass")
        rho = torch.empty_like(mass)
        T = torch.empty((len(self.shape),) + self.shape, dtype=self.dtype, device=mass.device) \
            if return_map else None
        P = ctypes.c_double()
        ws = self.workspace(mass.device)
        _check(lib().bfm_pushforward(self._h, _ptr(phic), _ptr(mass), _ptr(rho), _ptr(T), ctypes.byref(P),
                                     _ptr(ws), self.ws_bytes, _stream(mass.device)))
        return rho, T, P.value

    def poisson_neumann(self, f):
        f = self._field(f, "f")
        g = torch.empty_like(f)
        G = ctypes.c_double()
        ws = self.workspace(f.device)
        _check(lib().bfm_poisson_neumann(self._h, _ptr(f), _ptr(g), ctypes.byref(G), _ptr(ws), self.ws_bytes,
                                         _stream(f.device)))
        return g, G.value

    def grad(self, phi, psi, scale: float = 1.0):
        phi = self._field(phi, "phi")
        psi = self._field(psi, "psi")
        gmu = torch.empty_like(psi)
        gnu = torch.empty_like(phi)
        ws = self.workspace(phi.device)
        _check(lib().bfm_grad(self._h, _ptr(phi), _ptr(psi), float(scale), _ptr(gmu), _ptr(gnu), _ptr(ws),
                              self.ws_bytes, _stream(phi.device)))
        return gmu, gnu


@dataclass
class SolveResult:
    phi: torch.Tensor
    psi: torch.Tensor
    T: Optional[torch.Tensor]
    dual: float
    primal: float
    gap: float
    G: float
    sigma: float
    iters: int
    converged: bool
    mass_mu: float
    mass_nu: float
    sigma_floor_hits: int = 0   # step-rule updates that left sigma at sigma_min

    @property
    def w2sq(self) -> float:
        """W2^2 = 2 C(mu, nu) for c = |x-y|^2/2."""
        return 2.0 * self.dual


_plans = {}


def plan_for(shape, dtype, **kw) -> Plan:
    kw = {k: (tuple(float(x) for x in v) if k == "power" and v is not None else v) for k, v in kw.items()}
    key = (tuple(shape), _dtype_code(dtype), tuple(sorted(kw.items())))
    p = _plans.get(key)
    if p is None:
        p = Plan(shape, dtype, **kw)
        _plans[key] = p
    return p


def solve(mu: torch.Tensor, nu: torch.Tensor, phi_init=None, return_map=True, **kw) -> SolveResult:
    """Quadratic-cost OT between grid densities: the back-and-forth iteration,
    or with ``method="ga"`` the plain H^1 gradient ascent it is compared with."""
    return plan_for(mu.shape, mu.dtype, **kw).solve(mu, nu, phi_init=phi_init, return_map=return_map)


def ctransform(f: torch.Tensor, power=None) -> torch.Tensor:
    """f^c for the quadratic cost, or the power cost of exponents ``power``."""
    return plan_for(f.shape, f.dtype, power=power).ctransform(f)


def interpolate(phi: torch.Tensor, mu: torch.Tensor, times, power=None) -> torch.Tensor:
    """Displacement interpolants between mu and the target of the map of phi."""
    return plan_for(mu.shape, mu.dtype, power=power).interpolate(phi, mu, times)


def pushforward(phic: torch.Tensor, mass: torch.Tensor, return_map=True, power=None):
    return plan_for(phic.shape, phic.dtype, power=power).pushforward(phic, mass, return_map=return_map)


def poisson_neumann(f: torch.Tensor):
    return plan_for(f.shape, f.dtype).poisson_neumann(f)


def solve_batched(mus: Sequence[torch.Tensor], nus: Sequence[torch.Tensor], max_iters: int = 100,
                  tol: float = 0.0, iters_per_graph: int = 8, return_map: bool = False,
                  workspaces: Optional[List[torch.Tensor]] = None, method: str = "bfm",
                  power: Optional[Sequence[float]] = None, aligned: bool = False) -> List[SolveResult]:
    """Solve many independent problems together (``bfm_solve_batched``): one
    HIP graph replay advances every problem by ``iters_per_graph`` iterations.
    Problems may have different shapes; all share dtype and ``max_iters``."""
    n = len(mus)
    if n != len(nus) or n == 0:
        raise ValueError("need the same positive number of mu and nu tensors")
    dev = mus[0].device
    plans = [plan_for(m.shape, m.dtype, max_iters=max_iters, tol=tol, method=method, power=power) for m in mus]
    mus = [p._field(m, "mu[%d]" % i) for i, (p, m) in enumerate(zip(plans, mus))]
    nus = [p._field(v, "nu[%d]" % i) for i, (p, v) in enumerate(zip(plans, nus))]
    phis = [torch.empty_like(m) for m in mus]
    psis = [torch.empty_like(m) for m in mus]
    Ts = [torch.empty((len(p.shape),) + p.shape, dtype=p.dtype, device=dev) for p in plans] if return_map else None
    if workspaces is None:
        ws = _aligned_workspaces(plans, dev)
    elif aligned:   # already 256-byte aligned views of ws_bytes each
        ws = list(workspaces)
    else:
        ws = []
        for p, raw in zip(plans, workspaces):
            off = (-raw.data_ptr()) % 256
            ws.append(raw[off:off + p.ws_bytes])
    VP = ctypes.c_void_p * n
    res = (Result * n)()
    _check(lib().bfm_solve_batched(
        n, VP(*[p.handle.value for p in plans]), VP(*[m.data_ptr() for m in mus]), VP(*[v.data_ptr() for v in nus]),
        VP(*[t.data_ptr() for t in phis]), VP(*[t.data_ptr() for t in psis]),
        VP(*[t.data_ptr() for t in Ts]) if Ts is not None else None, VP(*[w.data_ptr() for w in ws]),
        (ctypes.c_size_t * n)(*[p.ws_bytes for p in plans]), int(iters_per_graph), _stream(dev), res))
    out = []
    for i in range(n):
        r = res[i]
        out.append(SolveResult(phi=phis[i], psi=psis[i], T=Ts[i] if Ts is not None else None, dual=r.dual,
                               primal=r.primal, gap=r.gap, G=r.G, sigma=r.sigma, iters=r.iters,
                               converged=bool(r.converged), mass_mu=r.mass_mu, mass_nu=r.mass_nu,
                               sigma_floor_hits=r.sigma_floor_hits))
    return out


def grad_batched(plans: Sequence[Plan], phis: Sequence[torch.Tensor], psis: Sequence[torch.Tensor],
                 scales: Sequence[float], workspaces: Sequence[torch.Tensor]):
    """Gradients of W2^2 for a batch of solved pairs (``bfm_grad_batched``):
    three launches for the whole batch; returns (grad_mu list, grad_nu list)."""
    n = len(plans)
    if not (len(phis) == len(psis) == len(scales) == len(workspaces) == n) or n == 0:
        raise ValueError("need the same positive number of plans, potentials, scales and workspaces")
    phis = [p._field(t, "phi[%d]" % i) for i, (p, t) in enumerate(zip(plans, phis))]
    psis = [p._field(t, "psi[%d]" % i) for i, (p, t) in enumerate(zip(plans, psis))]
    gmus = [torch.empty_like(t) for t in psis]
    gnus = [torch.empty_like(t) for t in phis]
    VP = ctypes.c_void_p * n
    _check(lib().bfm_grad_batched(
        n, VP(*[p.handle.value for p in plans]), VP(*[t.data_ptr() for t in phis]), VP(*[t.data_ptr() for t in psis]),
        (ctypes.c_double * n)(*[float(x) for x in scales]), VP(*[t.data_ptr() for t in gmus]),
        VP(*[t.data_ptr() for t in gnus]), VP(*[w.data_ptr() for w in workspaces]),
        (ctypes.c_size_t * n)(*[p.ws_bytes for p in plans]), _stream(phis[0].device)))
    return gmus, gnus


def _aligned_workspaces(plans, dev):
    out = []
    for p in plans:
        raw = torch.empty(p.ws_bytes + 256, dtype=torch.uint8, device=dev)
        off = (-raw.data_ptr()) % 256
        out.append(raw[off:off + p.ws_bytes])
    return out


class W2LossBatched(torch.autograd.Function):
    """W2^2 of many (mu_i, nu_i) pairs from one batched solve; the backward
    pass returns each pair's mean-zeroed potentials times 2 cell_volume, for
    the whole batch at once (bfm_grad_batched) on the solve's workspaces."""

    @staticmethod
    def forward(ctx, max_iters, tol, iters_per_graph, *tensors):
        n = len(tensors) // 2
        mus, nus = tensors[:n], tensors[n:]
        dev = mus[0].device
        # the plans solve_batched looks up (same keys), so the workspaces fit them
        plans = [plan_for(m.shape, m.dtype, max_iters=max_iters, tol=tol, method="bfm", power=None) for m in mus]
        ws = _aligned_workspaces(plans, dev)
        rs = solve_batched([m.detach() for m in mus], [v.detach() for v in nus], max_iters=max_iters, tol=tol,
                           iters_per_graph=iters_per_graph, workspaces=ws, aligned=True)
        ctx.plans = plans
        ctx.workspaces = ws
        ctx.save_for_backward(*[r.phi for r in rs], *[r.psi for r in rs])
        ctx.results = [(r.iters, r.converged, r.gap) for r in rs]
        return torch.tensor([r.w2sq for r in rs], dtype=mus[0].dtype, device=dev)

    @staticmethod
    def backward(ctx, grad_out):
        saved = ctx.saved_tensors
        n = len(saved) // 2
        go = grad_out.detach().double().cpu().tolist()
        gmus, gnus = grad_batched(ctx.plans, saved[:n], saved[n:], go, ctx.workspaces)
        return (None, None, None, *gmus, *gnus)


def w2_loss_batched(mus: Sequence[torch.Tensor], nus: Sequence[torch.Tensor], max_iters: int = 200,
                    tol: float = 1e-6, iters_per_graph: int = 8) -> torch.Tensor:
    """Vector of W2^2 values, differentiable w.r.t. every mu_i and nu_i."""
    return W2LossBatched.apply(max_iters, tol, iters_per_graph, *mus, *nus)


class W2Loss(torch.autograd.Function):
    """W2^2(mu, nu) = 2 C(mu, nu) from a back-and-forth solve; the backward
    pass returns the converged Kantorovich potentials (mean-zeroed, scaled by
    2 cell_volume) as the gradients w.r.t. the grid density values."""

    @staticmethod
    def forward(ctx, mu, nu, max_iters=200, tol=1e-6):
        plan = plan_for(mu.shape, mu.dtype, max_iters=max_iters, tol=tol)
        r = plan.solve(mu.detach().contiguous(), nu.detach().contiguous(), return_map=False)
        ctx.plan = plan
        ctx.save_for_backward(r.phi, r.psi)
        return torch.tensor(r.w2sq, dtype=torch.float64, device=mu.device).to(mu.dtype)

    @staticmethod
    def backward(ctx, grad_out):
        phi, psi = ctx.saved_tensors
        gmu, gnu = ctx.plan.grad(phi, psi, float(grad_out))
        return gmu, gnu, None, None


def w2_loss(mu, nu, max_iters=200, tol=1e-6):
    return W2Loss.apply(mu, nu, max_iters, tol)
