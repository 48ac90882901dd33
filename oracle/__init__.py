"""Oracle for Fast and Robust ICP (arXiv 2007.07627) -- TEST INFRASTRUCTURE.

A plain, slow FP64 CPU implementation (``oracle.c``) of what the GPU path
computes, wrapped with ctypes. Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product package never
does, and the two share no code.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

P2P_L2, P2P_WELSCH, P2PL_WELSCH, P2PL_L2 = 0, 1, 2, 3
FLAG_CONVERGED, FLAG_MAX_ITER, FLAG_ZERO_WEIGHT, FLAG_DEGENERATE, FLAG_AA_SINGULAR = 1, 2, 4, 8, 16
# trace row reasons (column 2): stage start, iterate, safeguard revert, line-search trial
ROW_STAGE, ROW_ITER, ROW_REVERT, ROW_TRIAL = 1, 2, 3, 4


def build() -> str:
    """Compile oracle.c into liboracle.so (plain gcc, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-mfma",
           "-ffp-contract=off", "-o", _SO, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _SO


class Params(C.Structure):
    _fields_ = [("mode", C.c_int), ("anderson_m", C.c_int), ("nu_max", C.c_double),
                ("nu_min", C.c_double), ("eps", C.c_double), ("iter_first", C.c_int),
                ("iter_inc", C.c_int), ("iter_cap", C.c_int), ("max_total_iter", C.c_int),
                ("max_line_search", C.c_int), ("T0", C.c_double * 16)]


class Result(C.Structure):
    _fields_ = [("T", C.c_double * 16), ("energy", C.c_double), ("nu_final", C.c_double),
                ("iterations", C.c_int), ("nn_passes", C.c_int), ("evaluations", C.c_int),
                ("aa_accepted", C.c_int), ("aa_rejected", C.c_int),
                ("line_search_trials", C.c_int), ("stages", C.c_int), ("flags", C.c_uint)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_SO)
        f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        L.orc_transform_f32.argtypes = [f64p, f32p, C.c_int64, f32p]
        L.orc_nn_brute.argtypes = [f32p, C.c_int64, f32p, C.c_int64, i32p, f32p]
        L.orc_nn_query.argtypes = [f32p, C.c_int64, f32p, C.c_int64, f64p, i32p, f32p]
        L.orc_se3_exp.argtypes = [f64p, f64p]
        L.orc_se3_log.argtypes = [f64p, f64p]
        L.orc_svd3.argtypes = [f64p, f64p, f64p, f64p]
        L.orc_procrustes.argtypes = [f32p, f32p, C.c_void_p, C.c_int64, f64p]
        L.orc_procrustes.restype = C.c_uint
        L.orc_plane_residual.argtypes = [f64p, f32p, f32p, f32p]
        L.orc_plane_residual.restype = C.c_double
        L.orc_plane_gradient.argtypes = [f64p, f32p, f32p, f64p]
        L.orc_anderson_solve.argtypes = [f64p, f64p, C.c_int, C.c_int, f64p]
        L.orc_anderson_solve.restype = C.c_int
        L.orc_median.argtypes = [f64p, C.c_int64]
        L.orc_median.restype = C.c_double
        L.orc_register.argtypes = [f32p, C.c_int64, f32p, C.c_void_p, C.c_int64,
                                   C.POINTER(Params), C.POINTER(Result), C.c_void_p,
                                   C.c_int, C.POINTER(C.c_int), C.c_void_p, C.c_int,
                                   C.POINTER(C.c_int)]
        L.orc_register.restype = C.c_int
        L.orc_params_default.argtypes = [C.c_int, C.POINTER(Params)]
        L.orc_params_classical.argtypes = [C.c_int, C.POINTER(Params)]
        L.orc_params_classical.restype = C.c_int
        L.orc_eval.argtypes = [f32p, C.c_int64, f32p, C.c_void_p, C.c_int64, C.c_int, f64p,
                               C.c_double, C.POINTER(C.c_double), f64p, C.POINTER(C.c_uint)]
        L.orc_eval.restype = C.c_int
        L.orc_eval_xi.argtypes = [f32p, C.c_int64, f32p, C.c_void_p, C.c_int64, C.c_int, f64p,
                                  C.c_double, C.POINTER(C.c_double), f64p, C.POINTER(C.c_uint)]
        L.orc_eval_xi.restype = C.c_int
        L.orc_nu_min_auto.argtypes = [f32p, C.c_void_p, C.c_int64, C.c_int, C.POINTER(C.c_double),
                                      C.c_void_p]
        L.orc_nu_min_auto.restype = C.c_int
        L.orc_estimate_normals.argtypes = [f32p, C.c_int64, f32p]
        L.orc_estimate_normals.restype = C.c_int
        _lib = L
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def transform_f32(T, P):
    P = _f32(P).reshape(-1, 3)
    out = np.empty_like(P)
    lib().orc_transform_f32(_f64(T).reshape(16), P, P.shape[0], out)
    return out


def nn_brute(Pt, Q):
    Pt = _f32(Pt).reshape(-1, 3)
    Q = _f32(Q).reshape(-1, 3)
    idx = np.empty(Pt.shape[0], np.int32)
    d2 = np.empty(Pt.shape[0], np.float32)
    lib().orc_nn_brute(Pt, Pt.shape[0], Q, Q.shape[0], idx, d2)
    return idx, d2


def nn_query(P, Q, T=None):
    P = _f32(P).reshape(-1, 3)
    Q = _f32(Q).reshape(-1, 3)
    T = np.eye(4) if T is None else T
    idx = np.empty(P.shape[0], np.int32)
    d2 = np.empty(P.shape[0], np.float32)
    lib().orc_nn_query(P, P.shape[0], Q, Q.shape[0], _f64(T).reshape(16), idx, d2)
    return idx, d2


def se3_exp(xi):
    T = np.empty(16)
    lib().orc_se3_exp(_f64(xi).reshape(6), T)
    return T.reshape(4, 4)


def se3_log(T):
    xi = np.empty(6)
    lib().orc_se3_log(_f64(T).reshape(16), xi)
    return xi


def svd3(A):
    U, S, V = np.empty(9), np.empty(3), np.empty(9)
    lib().orc_svd3(_f64(A).reshape(9), U, S, V)
    return U.reshape(3, 3), S, V.reshape(3, 3)


def procrustes(P, Qh, w=None):
    P = _f32(P).reshape(-1, 3)
    Qh = _f32(Qh).reshape(-1, 3)
    T = np.empty(16)
    wp = None
    if w is not None:
        w = _f64(w)
        wp = w.ctypes.data
    flags = lib().orc_procrustes(P, Qh, wp, P.shape[0], T)
    return T.reshape(4, 4), int(flags)


def plane_residual(xi, p, q, n):
    return lib().orc_plane_residual(_f64(xi), _f32(p), _f32(q), _f32(n))


def plane_gradient(xi, p, n):
    J = np.empty(6)
    lib().orc_plane_gradient(_f64(xi), _f32(p), _f32(n), J)
    return J


def anderson_solve(dF, Fk, metric):
    dF = _f64(dF).reshape(-1, 6)
    th = np.zeros(max(dF.shape[0], 1))
    sing = lib().orc_anderson_solve(dF, _f64(Fk).reshape(6), dF.shape[0], metric, th)
    return th[: dF.shape[0]], bool(sing)


def median(v):
    v = _f64(v)
    return lib().orc_median(v, v.shape[0])


def nu_min_auto(Q, Qn, mode, per_point=False):
    """Automatic nu_min (Sec. 4.3 / Sec. 5, App. C) of a target set; with
    per_point, also the per-target medians (squared distances for
    point-to-point, tangent-plane distances for point-to-plane)."""
    Q = _f32(Q).reshape(-1, 3)
    qn = None
    if Qn is not None:
        Qn = _f32(Qn).reshape(-1, 3)
        qn = Qn.ctypes.data
    out = C.c_double(0.0)
    pp = np.zeros(Q.shape[0]) if per_point else None
    rc = lib().orc_nu_min_auto(Q, qn, Q.shape[0], int(mode), C.byref(out),
                               pp.ctypes.data if per_point else None)
    if rc != 0:
        raise ValueError("orc_nu_min_auto: invalid arguments")
    return (out.value, pp) if per_point else out.value


def estimate_normals(Q):
    """Normals from the 30 nearest points (the point included) by FP64 PCA."""
    Q = _f32(Q).reshape(-1, 3)
    out = np.zeros_like(Q)
    if lib().orc_estimate_normals(Q, Q.shape[0], out) != 0:
        raise ValueError("orc_estimate_normals: needs at least 30 points")
    return out


def eval_map(P, Q, Qn, mode, T, nu=0.0):
    """One un-accelerated map application at T: (energy, T_next, flags)."""
    P = _f32(P).reshape(-1, 3)
    Q = _f32(Q).reshape(-1, 3)
    qn = None
    if Qn is not None:
        Qn = _f32(Qn).reshape(-1, 3)
        qn = Qn.ctypes.data
    E = C.c_double(0.0)
    Tn = np.zeros(16)
    fl = C.c_uint(0)
    rc = lib().orc_eval(P, P.shape[0], Q, qn, Q.shape[0], mode, _f64(T).reshape(16), float(nu),
                        C.byref(E), Tn, C.byref(fl))
    if rc != 0:
        raise ValueError("oracle: invalid eval arguments")
    return E.value, Tn.reshape(4, 4), fl.value


def eval_map_xi(P, Q, Qn, mode, xi, nu=0.0):
    """Algorithm 2's map at the parameters xi (point-to-plane modes):
    (energy at exp(xi), Gauss-Newton candidate xi* linearised at xi, flags)."""
    P = _f32(P).reshape(-1, 3)
    Q = _f32(Q).reshape(-1, 3)
    Qn = _f32(Qn).reshape(-1, 3)
    E = C.c_double(0.0)
    xo = np.zeros(6)
    fl = C.c_uint(0)
    rc = lib().orc_eval_xi(P, P.shape[0], Q, Qn.ctypes.data, Q.shape[0], mode, _f64(xi).reshape(6),
                           float(nu), C.byref(E), xo, C.byref(fl))
    if rc != 0:
        raise ValueError("oracle: invalid eval arguments")
    return E.value, xo, fl.value


def default_params(mode):
    p = Params()
    lib().orc_params_default(mode, C.byref(p))
    return p


def classical_params(mode):
    """ICP (P2P_L2) or ICP-l (P2PL_L2) with the comparison methods' settings:
    no mixing, no line search, 1000 iterations, ||dT||_F^2 < 1e-5."""
    p = Params()
    if lib().orc_params_classical(mode, C.byref(p)) != 0:
        raise ValueError("oracle: classical settings exist for P2P_L2 and P2PL_L2 only")
    return p


def register(P, Q, Qn=None, params=None, trace_cap=0, etrace_cap=0, **overrides):
    """Run the full registration; returns a dict (T as 4x4) and, if
    trace_cap > 0, the transforms at which correspondences were computed; if
    etrace_cap > 0, (stage, accepted energy) per inner iteration."""
    P = _f32(P).reshape(-1, 3)
    Q = _f32(Q).reshape(-1, 3)
    if params is None:
        params = default_params(overrides.pop("mode", P2P_WELSCH))
    for k, v in overrides.items():
        if k == "T0":
            params.T0[:] = list(np.asarray(v, dtype=np.float64).reshape(16))
        else:
            setattr(params, k, v)
    qn = None
    if Qn is not None:
        Qn = _f32(Qn).reshape(-1, 3)
        qn = Qn.ctypes.data
    res = Result()
    tr = None
    tl = C.c_int(0)
    if trace_cap > 0:
        tr = np.zeros(20 * trace_cap)
    et = None
    el = C.c_int(0)
    if etrace_cap > 0:
        et = np.zeros(2 * etrace_cap)
    rc = lib().orc_register(P, P.shape[0], Q, qn, Q.shape[0], C.byref(params), C.byref(res),
                            None if tr is None else tr.ctypes.data, trace_cap, C.byref(tl),
                            None if et is None else et.ctypes.data, etrace_cap, C.byref(el))
    if rc != 0:
        raise ValueError("oracle: invalid registration arguments")
    out = {f: getattr(res, f) for f, _ in Result._fields_ if f != "T"}
    out["T"] = np.array(res.T[:]).reshape(4, 4)
    if tr is not None:
        out["trace"] = tr[: 20 * tl.value].reshape(-1, 20)
    if et is not None:
        out["etrace"] = et[: 2 * el.value].reshape(-1, 2)
    return out
