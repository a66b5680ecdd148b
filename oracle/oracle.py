"""ctypes front end of the FP64 CPU oracle (``oracle/abc_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Arrays are numpy float64, HWC (channel fastest);
2-vector fields (v, mu, grad) are ``(H, W, 2, C)`` with index 0 along
columns (x) and 1 along rows (y); controls are ``(K, 2)`` = (eps_x, eps_c).

Each function names the passage of the paper it implements; the arithmetic
itself lives in the C file.
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ABC_ORACLE_LIB names another build of the same sources (the sanitizer build of the tests)
_LIB_PATH = os.environ.get("ABC_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
_lib = None

_dp = ct.POINTER(ct.c_double)


class _Params(ct.Structure):
    _fields_ = [
        ("K", ct.c_int), ("dt", ct.c_double), ("R", ct.c_int), ("s", ct.c_double),
        ("eps_min", ct.c_double * 2), ("eps_max", ct.c_double * 2), ("eps_init", ct.c_double),
        ("alpha", ct.c_double), ("rho", ct.c_double), ("gamma", ct.c_double),
        ("max_outer", ct.c_int), ("max_inner", ct.c_int), ("max_ls", ct.c_int),
        ("tol_alm", ct.c_double), ("tol_dal", ct.c_double),
        ("sigma0", ct.c_double), ("armijo_b", ct.c_double), ("armijo_c", ct.c_double),
        ("literal_kernel", ct.c_int), ("cost", ct.c_int), ("tol_gap", ct.c_double),
    ]


class _Energies(ct.Structure):
    _fields_ = [(n, ct.c_double) for n in
                ("TV", "fid", "K", "L", "Ltilde", "r_abs", "r_rel", "sq_vg", "sq_g", "sq_v")]


class _Stats(ct.Structure):
    _fields_ = [("status", ct.c_int), ("outer_iters", ct.c_int), ("inner_iters", ct.c_int),
                ("ls_evals", ct.c_int)] + [(n, ct.c_double) for n in
                                           ("K", "TV", "fid", "L", "Ltilde", "r_rel", "r_abs",
                                            "gap_rel", "phi_first", "phi_last")]


@dataclass
class Params:
    """Solver parameters; defaults are the paper's values (Sec. 3.2 and Sec. 4.2)."""
    K: int = 20
    dt: float = 0.25                 # Sec. 3.2
    R: int = 2
    s: float = 0.0                   # 0: 1/min(N, (2R+1)^2)
    eps_min: tuple = (2.0, 2.0)      # E = [2, 1100]^2, Sec. 3.2
    eps_max: tuple = (1100.0, 1100.0)
    eps_init: float = 57.0           # Sec. 3.2
    alpha: float = 3000.0
    rho: float = 1e-2                # Sec. 4.2
    gamma: float = 1e-2              # Sec. 4.2
    max_outer: int = 5
    max_inner: int = 50
    max_ls: int = 40
    tol_alm: float = 0.0
    tol_dal: float = 0.0
    sigma0: float = 1.0              # Sec. 3.2
    armijo_b: float = 0.5            # Sec. 3.2
    armijo_c: float = 1e-4           # Sec. 3.2
    literal_kernel: int = 0
    cost: int = 0                    # 0: TV / method of multipliers, 1: quadratic J / DAL alone
    tol_gap: float = 0.0             # stop when the relative change of L is below this
    extra: dict = field(default_factory=dict)

    def norm(self, H: int, W: int) -> float:
        if self.s > 0.0:
            return float(self.s)
        return 1.0 / min(H * W, (2 * self.R + 1) ** 2)

    def to_c(self, H: int, W: int) -> _Params:
        p = _Params()
        p.K, p.dt, p.R, p.s = self.K, self.dt, self.R, self.norm(H, W)
        p.eps_min[0], p.eps_min[1] = self.eps_min
        p.eps_max[0], p.eps_max[1] = self.eps_max
        p.eps_init = self.eps_init
        p.alpha, p.rho, p.gamma = self.alpha, self.rho, self.gamma
        p.max_outer, p.max_inner, p.max_ls = self.max_outer, self.max_inner, self.max_ls
        p.tol_alm, p.tol_dal = self.tol_alm, self.tol_dal
        p.sigma0, p.armijo_b, p.armijo_c = self.sigma0, self.armijo_b, self.armijo_c
        p.literal_kernel = self.literal_kernel
        p.cost = self.cost
        p.tol_gap = self.tol_gap
        return p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ct.CDLL(_LIB_PATH)
        for name in ("or_phi", "or_dphi", "or_phi_literal", "or_dphi_literal"):
            getattr(L, name).restype = ct.c_double
            getattr(L, name).argtypes = [ct.c_double]
        L.or_forward_step.argtypes = [_dp, _dp, ct.c_int, ct.c_int, ct.c_int, ct.POINTER(_Params),
                                      ct.c_double, ct.c_double]
        L.or_forward_step.restype = ct.c_int
        L.or_forward_sweep.argtypes = [_dp, ct.c_int, ct.c_int, ct.c_int, ct.POINTER(_Params), _dp, _dp]
        L.or_forward_sweep.restype = ct.c_int
        L.or_adjoint_step.argtypes = [_dp, _dp, _dp, ct.c_int, ct.c_int, ct.c_int, ct.POINTER(_Params),
                                      ct.c_double, ct.c_double, _dp]
        L.or_adjoint_step.restype = ct.c_int
        L.or_adjoint_sweep.argtypes = [_dp, ct.c_int, ct.c_int, ct.c_int, ct.POINTER(_Params), _dp, _dp,
                                       _dp, _dp]
        L.or_adjoint_sweep.restype = ct.c_int
        L.or_grad.argtypes = [_dp, ct.c_int, ct.c_int, ct.c_int, _dp]
        L.or_div.argtypes = [_dp, ct.c_int, ct.c_int, ct.c_int, _dp]
        L.or_energies_eval.argtypes = [_dp, _dp, _dp, _dp, ct.c_int, ct.c_int, ct.c_int,
                                       ct.POINTER(_Params), ct.POINTER(_Energies)]
        L.or_energies_eval.restype = ct.c_int
        L.or_terminal.argtypes = [_dp, _dp, _dp, _dp, ct.c_int, ct.c_int, ct.c_int, ct.POINTER(_Params),
                                  _dp, _dp]
        L.or_terminal.restype = ct.c_int
        L.or_pd_step.argtypes = [_dp, _dp, ct.c_int, ct.c_int, ct.c_int, ct.POINTER(_Params), _dp, _dp,
                                 ct.c_int, ct.POINTER(_Energies)]
        L.or_pd_step.restype = ct.c_int
        L.or_solve.argtypes = [_dp, ct.c_int, ct.c_int, ct.c_int, ct.POINTER(_Params), _dp, _dp, _dp, _dp,
                               _dp, _dp, _dp, _dp, _dp, ct.POINTER(_Stats)]
        L.or_solve.restype = ct.c_int
        _fp = ct.POINTER(ct.c_float)
        _ip = ct.POINTER(ct.c_int32)
        L.seg_relief.argtypes = [_fp, ct.c_int, ct.c_int, ct.c_int, _fp]
        L.seg_watershed.argtypes = [_fp, ct.c_int, ct.c_int, ct.c_int, ct.c_float, _ip]
        L.seg_watershed.restype = ct.c_int
        L.seg_metrics.argtypes = [_fp, _fp, _ip, ct.c_int, ct.c_int, ct.c_int, ct.c_int, _dp]
        L.seg_metrics.restype = ct.c_int
        L.or_num_threads.restype = ct.c_int
        L.or_set_num_threads.argtypes = [ct.c_int]
        _lib = L
    return _lib


def _check(rc: int, what: str) -> None:
    if rc == -4:
        raise MemoryError(f"oracle {what}: out of memory")
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def _ptr(a):
    if a is None:
        return ct.cast(None, _dp)
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return lib().or_num_threads()


def set_num_threads(n: int) -> None:
    lib().or_set_num_threads(int(n))


def phi(r: float, literal: bool = False) -> float:
    """Interaction kernel, Sec. 3.2 eq. kernel (Wendland C^2 reading)."""
    return (lib().or_phi_literal if literal else lib().or_phi)(float(r))


def dphi(r: float, literal: bool = False) -> float:
    return (lib().or_dphi_literal if literal else lib().or_dphi)(float(r))


def _eps_array(P: Params, eps):
    if eps is None:
        return np.full((P.K, 2), P.eps_init, dtype=np.float64)
    e = _f64(eps).reshape(P.K, 2)
    return e.copy()


def forward_step(c, P: Params, ex: float, ec: float):
    """One explicit Euler step of eq. MAsystem (Sec. 2, Sec. 3.2)."""
    c = _f64(c)
    H, W, C = c.shape
    out = np.empty_like(c)
    pc = P.to_c(H, W)
    _check(lib().or_forward_step(_ptr(c), _ptr(out), H, W, C, ct.byref(pc), float(ex), float(ec)),
           "forward step")
    return out


def forward_sweep(c0, P: Params, eps=None):
    """K Euler steps; returns the trajectory ``(K+1, H, W, C)``."""
    c0 = _f64(c0)
    H, W, C = c0.shape
    e = _eps_array(P, eps)
    traj = np.empty((P.K + 1, H, W, C))
    pc = P.to_c(H, W)
    _check(lib().or_forward_sweep(_ptr(c0), H, W, C, ct.byref(pc), _ptr(e), _ptr(traj)), "forward sweep")
    return traj


def adjoint_step(c, p, P: Params, ex: float, ec: float):
    """Transpose of one Euler step applied to p, plus dl/d(eps_x, eps_c) of that step (Sec. 3.1)."""
    c, p = _f64(c), _f64(p)
    H, W, C = c.shape
    out = np.empty_like(p)
    gk = np.zeros(2)
    pc = P.to_c(H, W)
    _check(lib().or_adjoint_step(_ptr(c), _ptr(p), _ptr(out), H, W, C, ct.byref(pc), float(ex), float(ec),
                                 _ptr(gk)), "adjoint step")
    return out, gk


def adjoint_sweep(traj, P: Params, pK, eps=None):
    """Discrete adjoint sweep; returns (p^0 = dl/dc^0, dl/deps ``(K, 2)``)."""
    traj = _f64(traj)
    _, H, W, C = traj.shape
    e = _eps_array(P, eps)
    pK = _f64(pK)
    p0 = np.empty((H, W, C))
    geps = np.zeros((P.K, 2))
    pc = P.to_c(H, W)
    _check(lib().or_adjoint_sweep(_ptr(traj), H, W, C, ct.byref(pc), _ptr(e), _ptr(pK), _ptr(p0), _ptr(geps)),
           "adjoint sweep")
    return p0, geps


def grad(c):
    """Discrete gradient grad# of Def. 3.1; returns ``(H, W, 2, C)``."""
    c = _f64(c)
    H, W, C = c.shape
    g = np.empty((H, W, 2, C))
    lib().or_grad(_ptr(c), H, W, C, _ptr(g))
    return g


def div(w):
    """Divergence as -grad#^T (eq. discrete_divergence away from the border)."""
    w = _f64(w)
    H, W, _, C = w.shape
    out = np.empty((H, W, C))
    lib().or_div(_ptr(w), H, W, C, _ptr(out))
    return out


def energies(c, c0, v, mu, P: Params) -> dict:
    """TV, fidelity, K (eq. cost_TV), L (eq. cost_tv_regular), L~ (eq. complete_square), residuals."""
    c, c0 = _f64(c), _f64(c0)
    H, W, C = c.shape
    v = None if v is None else _f64(v)
    mu = None if mu is None else _f64(mu)
    E = _Energies()
    pc = P.to_c(H, W)
    _check(lib().or_energies_eval(_ptr(c), _ptr(c0), _ptr(v), _ptr(mu), H, W, C, ct.byref(pc), ct.byref(E)),
           "energies")
    return {n: getattr(E, n) for n, _ in _Energies._fields_}


def terminal(cK, c0, v, mu, P: Params):
    """p^K = dL~/dc (eq. admm_terminal) and L~ (eq. complete_square)."""
    cK, c0 = _f64(cK), _f64(c0)
    H, W, C = cK.shape
    v = None if v is None else _f64(v)
    mu = None if mu is None else _f64(mu)
    pK = np.empty((H, W, C))
    Lt = ct.c_double(0.0)
    pc = P.to_c(H, W)
    _check(lib().or_terminal(_ptr(cK), _ptr(c0), _ptr(v), _ptr(mu), H, W, C, ct.byref(pc), _ptr(pK),
                             ct.cast(ct.pointer(Lt), _dp)), "terminal")
    return pK, Lt.value


def pd_step(cK, c0, v, mu, P: Params, update_mu: bool = True):
    """Shrinkage v-update (eq. soft_threshold) and dual ascent (eq. dual_ascent); returns (v, mu, energies)."""
    cK, c0 = _f64(cK), _f64(c0)
    H, W, C = cK.shape
    v = np.zeros((H, W, 2, C)) if v is None else _f64(v).copy()
    mu = np.zeros((H, W, 2, C)) if mu is None else _f64(mu).copy()
    E = _Energies()
    pc = P.to_c(H, W)
    _check(lib().or_pd_step(_ptr(cK), _ptr(c0), H, W, C, ct.byref(pc), _ptr(v), _ptr(mu), int(update_mu),
                            ct.byref(E)), "pd step")
    return v, mu, {n: getattr(E, n) for n, _ in _Energies._fields_}


def solve(c0, P: Params, eps=None, mu=None, decisions=None):
    """Method of multipliers (Alg. 2) with the DAL/Armijo control argmin (Alg. 1).

    ``decisions``: optional ``(max_outer, max_inner)`` array of accepted steps
    to replay instead of running the line search.  Returns a dict with the
    final field ``c``, ``eps``, ``v``, ``mu``, the decision log, a per-DAL
    iteration trace ``(max_outer, max_inner, 4)`` = (Phi before, Phi after,
    trials, smallest relative Armijo margin of the slot's trials), the controls after every accepted step ``eps_log`` and the
    gradient of every DAL iteration ``grad_log`` (both ``(M, P, K, 2)``) and
    stats.
    """
    c0 = _f64(c0)
    H, W, C = c0.shape
    e = _eps_array(P, eps)
    m = np.zeros((H, W, 2, C)) if mu is None else _f64(mu).copy()
    v = np.zeros((H, W, 2, C))
    cK = np.empty((H, W, C))
    dec_out = np.zeros((max(P.max_outer, 1), max(P.max_inner, 1)))
    dec_in = None if decisions is None else _f64(decisions).reshape(P.max_outer, P.max_inner).copy()
    trace = np.zeros((max(P.max_outer, 1), max(P.max_inner, 1), 4))
    eps_log = np.zeros((max(P.max_outer, 1), max(P.max_inner, 1), P.K, 2))
    grad_log = np.zeros_like(eps_log)
    st = _Stats()
    pc = P.to_c(H, W)
    _check(lib().or_solve(_ptr(c0), H, W, C, ct.byref(pc), _ptr(e), _ptr(m), _ptr(v), _ptr(cK),
                          _ptr(dec_in), _ptr(dec_out), _ptr(trace), _ptr(eps_log), _ptr(grad_log), ct.byref(st)),
           "solve")
    stats = {n: getattr(st, n) for n, _ in _Stats._fields_}
    return {"c": cK, "eps": e, "v": v, "mu": m, "decisions": dec_out, "trace": trace, "eps_log": eps_log,
            "grad_log": grad_log, "stats": stats}


# ---------------------------------------------------------------------------
# Segmentation metrics of Sec. 4.4 on a watershed labelling (seg_oracle.c).

def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def seg_relief(c):
    """FP32 relief g2 = |grad c|^2 (central differences in pixel units) of an (H, W, C) field."""
    c = _f32(c)
    H, W, C = c.shape
    g2 = np.empty((H, W), dtype=np.float32)
    lib().seg_relief(c.ctypes.data_as(ct.POINTER(ct.c_float)), H, W, C, g2.ctypes.data_as(ct.POINTER(ct.c_float)))
    return g2


def seg_watershed(c, theta: float = 0.02):
    """Marker-based watershed of an (H, W, C) field at threshold theta (Sec. 4.4):
    returns (labels (H, W) int32 in [0, k), k)."""
    c = _f32(c)
    H, W, C = c.shape
    lab = np.empty((H, W), dtype=np.int32)
    k = lib().seg_watershed(c.ctypes.data_as(ct.POINTER(ct.c_float)), H, W, C, ct.c_float(theta),
                            lab.ctypes.data_as(ct.POINTER(ct.c_int32)))
    if k < 1:
        raise RuntimeError(f"seg_watershed failed ({k})")
    return lab, k


def seg_metrics(c, c0, labels, k: int | None = None) -> dict:
    """IRV, IRC and VS (Sec. 4.4) of a labelling: c the processed field, c0 the original image."""
    c, c0 = _f32(c), _f32(c0)
    H, W, C = c.shape
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    if k is None:
        k = int(labels.max()) + 1
    out = np.empty(3)
    rc = lib().seg_metrics(c.ctypes.data_as(ct.POINTER(ct.c_float)), c0.ctypes.data_as(ct.POINTER(ct.c_float)),
                           labels.ctypes.data_as(ct.POINTER(ct.c_int32)), H, W, C, int(k), _ptr(out))
    if rc != 0:
        raise ValueError(f"seg_metrics failed ({rc})")
    return {"irv": float(out[0]), "irc": float(out[1]), "vs": float(out[2])}


def segment(c, c0, theta: float = 0.02) -> dict:
    """Watershed labels of c and their metrics against the original image c0."""
    lab, k = seg_watershed(c, theta)
    m = seg_metrics(c, c0, lab, k)
    m.update(labels=lab, k=k)
    return m
