"""Thin ctypes binding of ``libabc.so`` (declared in ``include/abc.h``).

Argument marshalling only: every step of the solver runs in the HIP library.
Tensors must be float32, contiguous and on the current HIP device; work is
ordered on torch's current stream.  The library must be built
(``python -m paper_2510_16154_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes as ct
import os
import re
from dataclasses import dataclass, fields

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libabc.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "abc.h")

ABC_OK, ABC_EINVAL, ABC_EHIP, ABC_ENONFINITE, ABC_ENOCONV = 0, -1, -2, -3, 1
ABC_WS_SOLVE, ABC_WS_FORWARD, ABC_WS_ADJOINT, ABC_WS_PD = 0, 1, 2, 3
ABC_COST_TV, ABC_COST_QUADRATIC = 0, 1
ABC_WS_TUNE = 4
ABC_FLAG_NO_GRAPHS = 1
ABC_FLAG_AUTOTUNE = 2
ABC_FLAG_PERSISTENT = 4
ABC_MAX_RADIUS = 16  # largest radius of the LDS-tiled kernels; larger ones run the direct kernels
ABC_MAX_DIRECT_RADIUS = 32767
ABC_RADIUS_SUPPORT = -1  # Params.R asking for the support radius of each image (abc_support_radius)


class AbcParams(ct.Structure):
    _fields_ = [
        ("K", ct.c_int32), ("dt", ct.c_float), ("R", ct.c_int32), ("inv_norm", ct.c_float),
        ("eps_min", ct.c_float * 2), ("eps_max", ct.c_float * 2), ("eps_init", ct.c_float),
        ("alpha", ct.c_float), ("rho", ct.c_float), ("gamma", ct.c_float),
        ("max_outer", ct.c_int32), ("max_inner", ct.c_int32), ("max_ls", ct.c_int32),
        ("tol_alm", ct.c_double), ("tol_dal", ct.c_double),
        ("sigma0", ct.c_double), ("armijo_b", ct.c_double), ("armijo_c", ct.c_double),
        ("ckpt_every", ct.c_int32), ("tile_x", ct.c_int32), ("tile_y", ct.c_int32), ("cost", ct.c_int32),
        ("adj_tile_x", ct.c_int32), ("adj_tile_y", ct.c_int32), ("flags", ct.c_int32), ("stop_K", ct.c_double),
        ("tol_gap", ct.c_double),
    ]


class AbcSolveLog(ct.Structure):
    _fields_ = [("decisions_in", ct.POINTER(ct.c_double)), ("decisions_out", ct.POINTER(ct.c_double)),
                ("eps_replay", ct.POINTER(ct.c_double)), ("grad_out", ct.POINTER(ct.c_double)),
                ("phi_out", ct.POINTER(ct.c_double)), ("outer_out", ct.POINTER(ct.c_double)),
                ("eps_out", ct.POINTER(ct.c_double))]


class AbcImage(ct.Structure):
    _fields_ = [("c0", ct.c_void_p), ("c_out", ct.c_void_p), ("eps", ct.c_void_p), ("mu", ct.c_void_p),
                ("H", ct.c_int32), ("W", ct.c_int32)]


class AbcSegStats(ct.Structure):
    _fields_ = [("k", ct.c_int32), ("nonempty", ct.c_int32), ("rounds", ct.c_int32), ("reserved", ct.c_int32),
                ("irv", ct.c_double), ("irc", ct.c_double), ("vs", ct.c_double)]


class AbcStats(ct.Structure):
    _fields_ = [("status", ct.c_int32), ("outer_iters", ct.c_int32), ("inner_iters", ct.c_int32),
                ("ls_evals", ct.c_int32)] + [(n, ct.c_double) for n in (
                    "K", "TV", "fid", "L", "Ltilde", "r_rel", "r_abs", "gap_rel", "phi_first", "phi_last",
                    "K_start", "ms_start")]


@dataclass
class Params:
    """Python mirror of ``abc_params``; defaults are the library's (``abc_default_params``)."""
    K: int = 20
    dt: float = 0.25
    R: int = 2
    inv_norm: float = 0.0
    eps_min: tuple = (2.0, 2.0)
    eps_max: tuple = (1100.0, 1100.0)
    eps_init: float = 57.0
    alpha: float = 3000.0
    rho: float = 1e-2
    gamma: float = 1e-2
    max_outer: int = 5
    max_inner: int = 50
    max_ls: int = 40
    tol_alm: float = 0.0
    tol_dal: float = 0.0
    sigma0: float = 1.0
    armijo_b: float = 0.5
    armijo_c: float = 1e-4
    ckpt_every: int = 0
    tile_x: int = 0
    tile_y: int = 0
    cost: int = 0  # ABC_COST_TV (0) or ABC_COST_QUADRATIC (1)
    adj_tile_x: int = 0
    adj_tile_y: int = 0
    flags: int = 0  # ABC_FLAG_NO_GRAPHS (1), ABC_FLAG_AUTOTUNE (2), ABC_FLAG_PERSISTENT (4); see abc.h
    stop_K: float = 0.0  # > 0: stop once the TV energy K reaches this value
    tol_gap: float = 0.0  # > 0: stop once L changes by less than this (relative) between iterations

    def __setattr__(self, name, value):
        # the converted struct (see to_c) is dropped whenever a field is assigned;
        # the two boxes are stored as tuples so that they cannot change in place
        if name in ("eps_min", "eps_max"):
            value = tuple(float(x) for x in value)
        object.__setattr__(self, name, value)
        object.__setattr__(self, "_c", None)

    def to_c(self) -> AbcParams:
        """The ``abc_params`` struct of these values, converted once and kept until
        a field is assigned (the library only reads it)."""
        c = self.__dict__.get("_c")
        if c is None:
            c = self._convert()
            object.__setattr__(self, "_c", c)
        return c

    def _convert(self) -> AbcParams:
        p = AbcParams()
        for f in fields(self):
            val = getattr(self, f.name)
            if f.name in ("eps_min", "eps_max"):
                arr = getattr(p, f.name)
                arr[0], arr[1] = float(val[0]), float(val[1])
            else:
                setattr(p, f.name, val)
        return p

    @staticmethod
    def from_c(p: AbcParams) -> "Params":
        kw = {}
        for f in fields(Params):
            v = getattr(p, f.name)
            kw[f.name] = (float(v[0]), float(v[1])) if f.name in ("eps_min", "eps_max") else v
        return Params(**kw)

    def replace(self, **kw) -> "Params":
        d = {f.name: getattr(self, f.name) for f in fields(self)}
        d.update(kw)
        return Params(**d)


class AbcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"abc error {code}: {msg}")
        self.code = code


_lib = None
_vp = ct.c_void_p


def exported_names():
    """Entry points declared in include/abc.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(abc_[a-z_]+)\s*\(", txt, re.M)))


def lib():
    """Load libabc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2510_16154_amd.build`")
    L = ct.CDLL(LIB_PATH)
    L.abc_version.restype = ct.c_int
    L.abc_last_error.restype = ct.c_char_p
    L.abc_default_params.argtypes = [ct.POINTER(AbcParams)]
    L.abc_support_radius.argtypes = [ct.c_int, ct.c_int, ct.c_float, ct.POINTER(ct.c_int32)]
    L.abc_workspace_bytes.argtypes = [ct.c_int, ct.c_int, ct.c_int, ct.c_int, ct.POINTER(AbcParams),
                                      ct.POINTER(ct.c_size_t)]
    L.abc_traj_slots.argtypes = [ct.POINTER(AbcParams), ct.POINTER(ct.c_int)]
    L.abc_forward_dynamics.argtypes = [_vp, ct.c_int, ct.c_int, ct.c_int, _vp, ct.POINTER(AbcParams), _vp, _vp,
                                       ct.c_size_t, _vp]
    L.abc_adjoint_dynamics.argtypes = [_vp, ct.c_int, ct.c_int, ct.c_int, _vp, ct.POINTER(AbcParams), _vp, _vp,
                                       _vp, _vp, ct.c_size_t, _vp]
    L.abc_adjoint_dynamics_noalloc.argtypes = [_vp, ct.c_int, ct.c_int, ct.c_int, _vp, ct.POINTER(AbcParams), _vp,
                                               _vp, _vp, _vp]
    L.abc_pd_terminal.argtypes = [_vp, _vp, _vp, _vp, ct.c_int, ct.c_int, ct.c_int, ct.POINTER(AbcParams), _vp,
                                  ct.POINTER(ct.c_double), _vp, ct.c_size_t, _vp]
    L.abc_pd_step.argtypes = [_vp, _vp, ct.c_int, ct.c_int, ct.c_int, ct.POINTER(AbcParams), _vp, _vp, ct.c_int,
                              ct.POINTER(AbcStats), _vp, ct.c_size_t, _vp]
    L.abc_solve.argtypes = [_vp, ct.c_int, ct.c_int, ct.c_int, ct.POINTER(AbcParams), _vp, _vp, _vp, _vp, _vp,
                            ct.c_size_t, _vp, ct.POINTER(AbcStats), ct.POINTER(AbcSolveLog)]
    L.abc_autotune.argtypes = [_vp, ct.c_int, ct.c_int, ct.c_int, ct.POINTER(AbcParams), ct.c_char_p, _vp,
                               ct.c_size_t, _vp, ct.POINTER(ct.c_double)]
    L.abc_workspace_bytes_batched.argtypes = [ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int32), ct.c_int, ct.c_int,
                                              ct.POINTER(AbcParams), ct.POINTER(ct.c_size_t)]
    L.abc_solve_batched.argtypes = [ct.POINTER(AbcImage), ct.c_int, ct.c_int, ct.POINTER(AbcParams), _vp,
                                    ct.c_size_t, _vp, ct.POINTER(AbcStats), ct.POINTER(ct.c_double),
                                    ct.POINTER(AbcSolveLog)]
    L.abc_segment_workspace_bytes.argtypes = [ct.c_int, ct.c_int, ct.c_int, ct.POINTER(ct.c_size_t)]
    L.abc_segment.argtypes = [_vp, _vp, ct.c_int, ct.c_int, ct.c_int, ct.c_float, _vp, _vp, ct.POINTER(AbcSegStats),
                              _vp, ct.c_size_t, _vp]
    for name in exported_names():
        if name not in ("abc_version", "abc_last_error"):
            getattr(L, name).restype = ct.c_int
    _lib = L
    return L


def _check(rc: int, allow=(ABC_OK,)):
    if rc not in allow:
        raise AbcError(rc, lib().abc_last_error().decode())
    return rc


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch.Tensor")
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("tensors must be contiguous float32 on the GPU")
    return ct.c_void_p(t.data_ptr())


def _stats_dict(s: AbcStats) -> dict:
    return {n: getattr(s, n) for n, _ in AbcStats._fields_}


def _ptr_i32(t):
    if t is None:
        return None
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dtype != torch.int32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("labels must be a contiguous int32 tensor on the GPU")
    return ct.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ host-only calls
def abc_version() -> int:
    return lib().abc_version()


def abc_support_radius(H: int, W: int, eps_x_min: float) -> int:
    """Window radius that holds the kernel's support on an H x W image for every
    eps_x >= eps_x_min (whole image when that is smaller)."""
    r = ct.c_int32(0)
    _check(lib().abc_support_radius(H, W, ct.c_float(eps_x_min), ct.byref(r)))
    return r.value


def abc_default_params() -> Params:
    p = AbcParams()
    _check(lib().abc_default_params(ct.byref(p)))
    return Params.from_c(p)


def abc_workspace_bytes(kind: int, H: int, W: int, C: int, params: Params) -> int:
    n = ct.c_size_t(0)
    p = params.to_c()
    _check(lib().abc_workspace_bytes(kind, H, W, C, ct.byref(p), ct.byref(n)))
    return n.value


def abc_traj_slots(params: Params) -> int:
    n = ct.c_int(0)
    p = params.to_c()
    _check(lib().abc_traj_slots(ct.byref(p), ct.byref(n)))
    return n.value


def _workspace(kind, H, W, C, params, device):
    torch = _torch()
    nb = abc_workspace_bytes(kind, H, W, C, params)
    return torch.empty(max(nb, 1), dtype=torch.uint8, device=device), nb


# ------------------------------------------------------------------ device calls
def abc_forward_dynamics(c0, eps, params: Params, traj=None, ws=None):
    """Trajectory ``(slots, H, W, C)`` of the agent dynamics (see abc_forward_dynamics in abc.h)."""
    torch = _torch()
    H, W, C = c0.shape
    slots = abc_traj_slots(params)
    if traj is None:
        traj = torch.empty((slots, H, W, C), dtype=torch.float32, device=c0.device)
    if ws is None:
        ws, nb = _workspace(ABC_WS_FORWARD, H, W, C, params, c0.device)
    else:
        nb = ws.numel()
    p = params.to_c()
    _check(lib().abc_forward_dynamics(_ptr(c0), H, W, C, _ptr(eps), ct.byref(p), _ptr(traj),
                                      ct.c_void_p(ws.data_ptr()), nb, _stream()))
    return traj


def abc_adjoint_dynamics(traj, eps, params: Params, gK, g0=None, geps=None, ws=None):
    """(dl/dc^0, dl/deps) from dl/dc^K by the discrete adjoint sweep (see abc.h)."""
    torch = _torch()
    H, W, C = gK.shape
    if g0 is None:
        g0 = torch.empty_like(gK)
    if geps is None:
        geps = torch.empty((params.K, 2), dtype=torch.float32, device=gK.device)
    if ws is None:
        ws, nb = _workspace(ABC_WS_ADJOINT, H, W, C, params, gK.device)
    else:
        nb = ws.numel()
    p = params.to_c()
    _check(lib().abc_adjoint_dynamics(_ptr(traj), H, W, C, _ptr(eps), ct.byref(p), _ptr(gK), _ptr(g0),
                                      _ptr(geps), ct.c_void_p(ws.data_ptr()), nb, _stream()))
    return g0, geps


def abc_adjoint_dynamics_noalloc(traj, eps, params: Params, gK, g0, geps):
    """abc_adjoint_dynamics on the library's own per-GPU scratch (see abc.h):
    the caller passes the outputs g0 (like gK) and geps (K x 2); nothing is
    allocated.  Calls that overlap on one GPU race."""
    H, W, C = gK.shape
    p = params.to_c()
    _check(lib().abc_adjoint_dynamics_noalloc(_ptr(traj), H, W, C, _ptr(eps), ct.byref(p), _ptr(gK), _ptr(g0),
                                              _ptr(geps), _stream()))
    return g0, geps


def abc_pd_terminal(cK, c0, v, mu, params: Params, want_gradient=True, want_objective=True, gK=None, ws=None):
    """(dL~/dc at cK or None, L~ or None) -- the adjoint terminal condition (see abc.h).
    ``gK`` (H x W x C) and ``ws`` (ABC_WS_PD bytes) may be passed in to avoid allocations."""
    torch = _torch()
    H, W, C = cK.shape
    if want_gradient and gK is None:
        gK = torch.empty_like(cK)
    if not want_gradient:
        gK = None
    if ws is None:
        ws, nb = _workspace(ABC_WS_PD, H, W, C, params, cK.device)
    else:
        nb = ws.numel()
    Lt = ct.c_double(0.0)
    p = params.to_c()
    _check(lib().abc_pd_terminal(_ptr(cK), _ptr(c0), _ptr(v), _ptr(mu), H, W, C, ct.byref(p), _ptr(gK),
                                 ct.byref(Lt) if want_objective else None, ct.c_void_p(ws.data_ptr()), nb,
                                 _stream()))
    return gK, (Lt.value if want_objective else None)


def abc_pd_step(cK, c0, v, mu, params: Params, update_mu=True, want_stats=True, ws=None):
    """Shrinkage of v and multiplier ascent, in place on v and mu; returns the stats dict.
    ``ws`` (ABC_WS_PD bytes) may be passed in to avoid an allocation."""
    H, W, C = cK.shape
    if ws is None:
        ws, nb = _workspace(ABC_WS_PD, H, W, C, params, cK.device)
    else:
        nb = ws.numel()
    st = AbcStats()
    p = params.to_c()
    _check(lib().abc_pd_step(_ptr(cK), _ptr(c0), H, W, C, ct.byref(p), _ptr(v), _ptr(mu), int(bool(update_mu)),
                             ct.byref(st) if want_stats else None, ct.c_void_p(ws.data_ptr()), nb, _stream()))
    return _stats_dict(st) if want_stats else None


def abc_solve(c0, params: Params, eps=None, mu=None, want_v=True, decisions=None, eps_replay=None, ws=None):
    """Full solve (see abc_solve in abc.h).  Returns a dict with the field ``c``,
    ``eps`` and ``mu`` (the tensors passed in, updated, when given), ``v``,
    ``stats``, and the logs (numpy): ``decisions`` (max_outer x max_inner),
    ``grad_log`` (M x P x K x 2), ``phi_log`` (M x P x 5: objective before and
    after the step, trials, K after the step, ms), ``outer_log``
    (M x 4: K, L, r_rel, elapsed ms after each multiplier iteration) and
    ``eps_log`` (M x P x K x 2: the projected controls of each accepted step
    from the run's own gradient).  ``decisions`` and ``eps_replay``
    (M x P x K x 2) replay a recorded control argmin."""
    import numpy as np
    torch = _torch()
    H, W, C = c0.shape
    dev = c0.device
    c_out = torch.empty_like(c0)
    v = torch.empty((H, W, 2, C), dtype=torch.float32, device=dev) if want_v else None
    if ws is None:
        ws, nb = _workspace(ABC_WS_SOLVE, H, W, C, params, dev)
    else:
        nb = ws.numel()
    M, P, K = max(params.max_outer, 1), max(params.max_inner, 1), params.K
    dp = ct.POINTER(ct.c_double)
    dec_out = np.zeros((M, P), dtype=np.float64)
    grad_log = np.zeros((M, P, K, 2), dtype=np.float64)
    phi_log = np.zeros((M, P, 5), dtype=np.float64)
    outer_log = np.zeros((M, 4), dtype=np.float64)
    eps_log = np.zeros((M, P, K, 2), dtype=np.float64)
    log = AbcSolveLog()
    keep = []
    if decisions is not None:
        dec_in = np.ascontiguousarray(np.asarray(decisions, dtype=np.float64).reshape(M, P))
        keep.append(dec_in)
        log.decisions_in = dec_in.ctypes.data_as(dp)
    if eps_replay is not None:
        er = np.ascontiguousarray(np.asarray(eps_replay, dtype=np.float64).reshape(M, P, K, 2))
        keep.append(er)
        log.eps_replay = er.ctypes.data_as(dp)
    log.decisions_out = dec_out.ctypes.data_as(dp)
    log.grad_out = grad_log.ctypes.data_as(dp)
    log.phi_out = phi_log.ctypes.data_as(dp)
    log.outer_out = outer_log.ctypes.data_as(dp)
    log.eps_out = eps_log.ctypes.data_as(dp)
    st = AbcStats()
    p = params.to_c()
    rc = lib().abc_solve(_ptr(c0), H, W, C, ct.byref(p), _ptr(eps), _ptr(mu), _ptr(v), _ptr(c_out),
                         ct.c_void_p(ws.data_ptr()), nb, _stream(), ct.byref(st), ct.byref(log))
    _check(rc, allow=(ABC_OK, ABC_ENOCONV))
    return {"c": c_out, "eps": eps, "mu": mu, "v": v, "stats": _stats_dict(st), "decisions": dec_out,
            "grad_log": grad_log, "phi_log": phi_log, "outer_log": outer_log, "eps_log": eps_log, "status": rc}


def abc_workspace_bytes_batched(shapes, C: int, params: Params) -> int:
    n = len(shapes)
    Hs = (ct.c_int32 * n)(*[int(h) for h, _ in shapes])
    Ws = (ct.c_int32 * n)(*[int(w) for _, w in shapes])
    nb = ct.c_size_t(0)
    p = params.to_c()
    _check(lib().abc_workspace_bytes_batched(Hs, Ws, n, C, ct.byref(p), ct.byref(nb)))
    return nb.value


def abc_solve_batched(images, params: Params, eps=None, mu=None, ws=None, decisions=None, eps_replay=None,
                      want_logs=False):
    """Batched solve of a list of H x W x C images (see abc_solve_batched in
    abc.h).  ``eps`` / ``mu``: optional lists of per-image tensors (in/out).
    ``decisions`` / ``eps_replay``: optional lists of per-image replay arrays
    (shapes as in abc_solve; an entry may be None).  Returns (list of final
    fields, list of stats dicts, finish times in ms), and with ``want_logs`` a
    fourth item: per image, the dict of logs abc_solve returns (decisions,
    grad_log, phi_log, outer_log, eps_log)."""
    import numpy as np
    torch = _torch()
    n = len(images)
    C = images[0].shape[2]
    outs = [torch.empty_like(x) for x in images]
    descs = (AbcImage * n)()
    for i, x in enumerate(images):
        if x.shape[2] != C:
            raise ValueError("all images must have the same channel count")
        descs[i].c0 = x.data_ptr()
        descs[i].c_out = outs[i].data_ptr()
        descs[i].eps = _ptr(eps[i]).value if eps is not None and eps[i] is not None else None
        descs[i].mu = _ptr(mu[i]).value if mu is not None and mu[i] is not None else None
        descs[i].H, descs[i].W = x.shape[0], x.shape[1]
        _ptr(x)
    if ws is None:
        nb = abc_workspace_bytes_batched([(x.shape[0], x.shape[1]) for x in images], C, params)
        ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=images[0].device)
    else:
        nb = ws.numel()
    logs_c = None
    logs = []
    keep = []
    if want_logs or decisions is not None or eps_replay is not None:
        M, P, K = max(params.max_outer, 1), max(params.max_inner, 1), params.K
        dp = ct.POINTER(ct.c_double)
        logs_c = (AbcSolveLog * n)()
        for i in range(n):
            d = {"decisions": np.zeros((M, P)), "grad_log": np.zeros((M, P, K, 2)),
                 "phi_log": np.zeros((M, P, 5)), "outer_log": np.zeros((M, 4)),
                 "eps_log": np.zeros((M, P, K, 2))}
            logs.append(d)
            lg = logs_c[i]
            lg.decisions_out = d["decisions"].ctypes.data_as(dp)
            lg.grad_out = d["grad_log"].ctypes.data_as(dp)
            lg.phi_out = d["phi_log"].ctypes.data_as(dp)
            lg.outer_out = d["outer_log"].ctypes.data_as(dp)
            lg.eps_out = d["eps_log"].ctypes.data_as(dp)
            if decisions is not None and decisions[i] is not None:
                di = np.ascontiguousarray(np.asarray(decisions[i], dtype=np.float64).reshape(M, P))
                keep.append(di)
                lg.decisions_in = di.ctypes.data_as(dp)
            if eps_replay is not None and eps_replay[i] is not None:
                er = np.ascontiguousarray(np.asarray(eps_replay[i], dtype=np.float64).reshape(M, P, K, 2))
                keep.append(er)
                lg.eps_replay = er.ctypes.data_as(dp)
    st = (AbcStats * n)()
    fin = np.zeros(n, dtype=np.float64)
    p = params.to_c()
    rc = lib().abc_solve_batched(descs, n, C, ct.byref(p), ct.c_void_p(ws.data_ptr()), nb, _stream(), st,
                                 fin.ctypes.data_as(ct.POINTER(ct.c_double)), logs_c)
    _check(rc, allow=(ABC_OK, ABC_ENOCONV))
    if want_logs:
        return outs, [_stats_dict(s) for s in st], fin, logs
    return outs, [_stats_dict(s) for s in st], fin


def abc_autotune(c0, params: Params, cache_path=None):
    """Tile shapes tuned on c0 (see abc_autotune in abc.h).  Returns (tuned Params,
    (forward us, adjoint us) -- zeros on a cache hit)."""
    torch = _torch()
    H, W, C = c0.shape
    nb = abc_workspace_bytes(ABC_WS_TUNE, H, W, C, params)
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=c0.device)
    p = params._convert()  # a fresh struct: the library writes the tuned tiles into it
    us = (ct.c_double * 2)()
    path = cache_path.encode() if cache_path else None
    _check(lib().abc_autotune(_ptr(c0), H, W, C, ct.byref(p), path, ct.c_void_p(ws.data_ptr()), nb, _stream(), us))
    return Params.from_c(p), (us[0], us[1])


# ------------------------------------------------------------------ learned warm start
def _wsnet_lib():
    L = lib()
    if not getattr(L, "_wsnet_ready", False):
        L.abc_wsnet_param_count.argtypes = [ct.c_int, ct.POINTER(ct.c_size_t)]
        L.abc_wsnet_workspace_bytes.argtypes = [ct.c_int, ct.c_int, ct.c_int, ct.c_int, ct.c_int,
                                                ct.POINTER(ct.c_size_t)]
        L.abc_wsnet_forward.argtypes = [_vp, _vp, ct.c_int, ct.c_int, ct.c_int, ct.c_int, ct.POINTER(AbcParams), _vp,
                                        _vp, _vp, ct.c_size_t, _vp]
        L.abc_wsnet_loss_grad.argtypes = [_vp, _vp, _vp, _vp, ct.c_int, ct.c_int, ct.c_int, ct.c_int,
                                          ct.POINTER(AbcParams), ct.c_float, _vp, ct.POINTER(ct.c_double), _vp,
                                          ct.c_size_t, _vp]
        L.abc_wsnet_adam.argtypes = [_vp, _vp, _vp, _vp, ct.c_size_t, ct.c_int, ct.c_float, ct.c_float, ct.c_float,
                                     ct.c_float, _vp]
        L.abc_wsnet_last_error.restype = ct.c_char_p
        L._wsnet_ready = True
    return L


def _wcheck(rc):
    if rc != ABC_OK:
        raise AbcError(rc, _wsnet_lib().abc_wsnet_last_error().decode())


def abc_wsnet_param_count(K: int) -> int:
    n = ct.c_size_t(0)
    _wcheck(_wsnet_lib().abc_wsnet_param_count(K, ct.byref(n)))
    return n.value


def abc_wsnet_forward(params, x, K: int, box: Params, ws=None):
    """(mu0 B x H x W x 6, eps0 B x K x 2) predicted for the images x (B x H x W x 3)."""
    torch = _torch()
    B, H, W, _ = x.shape
    L = _wsnet_lib()
    nb_ = ct.c_size_t(0)
    _wcheck(L.abc_wsnet_workspace_bytes(B, H, W, K, 0, ct.byref(nb_)))
    if ws is None or ws.numel() < nb_.value:
        ws = torch.empty(nb_.value, dtype=torch.uint8, device=x.device)
    mu0 = torch.empty((B, H, W, 6), dtype=torch.float32, device=x.device)
    eps0 = torch.empty((B, K, 2), dtype=torch.float32, device=x.device)
    p = box.to_c()
    _wcheck(L.abc_wsnet_forward(_ptr(params), _ptr(x), B, H, W, K, ct.byref(p), _ptr(mu0), _ptr(eps0),
                                ct.c_void_p(ws.data_ptr()), ws.numel(), _stream()))
    return mu0, eps0


def abc_wsnet_loss_grad(params, x, mu_t, eps_t, K: int, box: Params, w_eps: float, grad=None, ws=None):
    """(loss, gradient in the parameters) of the warm-start network on one batch."""
    torch = _torch()
    B, H, W, _ = x.shape
    L = _wsnet_lib()
    nb_ = ct.c_size_t(0)
    _wcheck(L.abc_wsnet_workspace_bytes(B, H, W, K, 1, ct.byref(nb_)))
    if ws is None or ws.numel() < nb_.value:
        ws = torch.empty(nb_.value, dtype=torch.uint8, device=x.device)
    if grad is None:
        grad = torch.empty_like(params)
    loss = ct.c_double(0.0)
    p = box.to_c()
    _wcheck(L.abc_wsnet_loss_grad(_ptr(params), _ptr(x), _ptr(mu_t), _ptr(eps_t), B, H, W, K, ct.byref(p),
                                  float(w_eps), _ptr(grad), ct.byref(loss), ct.c_void_p(ws.data_ptr()), ws.numel(),
                                  _stream()))
    return loss.value, grad


def abc_wsnet_adam(params, grad, m, v, t: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    _wcheck(_wsnet_lib().abc_wsnet_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), params.numel(), int(t),
                                        float(lr), float(b1), float(b2), float(eps), _stream()))


# ------------------------------------------------------------------ segmentation scores
def abc_segment_workspace_bytes(H: int, W: int, C: int) -> int:
    n = ct.c_size_t()
    _check(lib().abc_segment_workspace_bytes(H, W, C, ct.byref(n)))
    return n.value


def abc_segment(c, c0, theta: float = 0.02, labels=None, want_labels=True, ws=None):
    """Watershed labels of the processed field c (H x W x C) and the IRV / IRC / VS
    scores of Sec. 4.4 against the original image c0; with ``labels`` (int32
    H x W) those labels are scored instead.  Returns (labels or None, stats)."""
    torch = _torch()
    H, W, C = c.shape
    if tuple(c0.shape) != (H, W, C):
        raise ValueError("c and c0 must have the same shape")
    if labels is not None and tuple(labels.shape) != (H, W):
        raise ValueError("labels must be H x W")
    nb = abc_segment_workspace_bytes(H, W, C)
    if ws is None or ws.numel() < nb:
        ws = torch.empty(nb, dtype=torch.uint8, device=c.device)
    out = torch.empty((H, W), dtype=torch.int32, device=c.device) if (labels is None and want_labels) else None
    st = AbcSegStats()
    _check(lib().abc_segment(_ptr(c), _ptr(c0), H, W, C, ct.c_float(theta), _ptr_i32(labels), _ptr_i32(out),
                             ct.byref(st), ct.c_void_p(ws.data_ptr()), nb, _stream()))
    return out, {n: getattr(st, n) for n, _ in AbcSegStats._fields_ if n != "reserved"}
