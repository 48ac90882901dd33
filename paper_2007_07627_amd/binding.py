"""Thin ctypes binding of libicp (include/icp.h). Argument marshalling only:
every step of the registration runs in the HIP library. Function names are
those of the C ABI. Raises if the compiled library is missing -- there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libicp.so")

ICP_OK, ICP_ERR_INVALID_ARG, ICP_ERR_NONFINITE, ICP_ERR_NO_NORMALS, ICP_ERR_OOM = 0, 1, 2, 3, 4
ICP_ERR_DEVICE, ICP_ERR_NOT_READY, ICP_ERR_UNKNOWN_TICKET, ICP_ERR_QUEUE_FULL = 5, 6, 7, 8
ICP_P2P_L2, ICP_P2P_WELSCH, ICP_P2PL_WELSCH, ICP_P2PL_L2 = 0, 1, 2, 3
ICP_NN_AUTO, ICP_NN_BRUTE, ICP_NN_CLUSTER = 0, 1, 2
ICP_ENGINE_GRAPH, ICP_ENGINE_PLAIN = 0, 1
ICP_FLAG_CONVERGED, ICP_FLAG_MAX_ITER, ICP_FLAG_ZERO_WEIGHT = 1, 2, 4
ICP_FLAG_DEGENERATE, ICP_FLAG_AA_SINGULAR = 8, 16
ICP_TRACE_ROW = 36

EXPORTED = ["icp_create", "icp_destroy", "icp_params_default", "icp_params_classical", "icp_register", "icp_register_trace",
            "icp_eval", "icp_trace_items",
            "icp_register_dev",
            "icp_nn_query", "icp_nn_query_dev", "icp_nn_query_dev_noalloc", "icp_nu_min_auto", "icp_estimate_normals", "icp_batch_submit", "icp_batch_submit_dev", "icp_poll",
            "icp_batch_wait_all", "icp_batch_config", "icp_profile", "icp_profile_read",
            "icp_tuning_default", "icp_tuning_lookup", "icp_tuning_set", "icp_tuning_entries",
            "icp_autotune", "icp_device_arch", "icp_tuning_file_write", "icp_tuning_file_read",
            "icp_status_str"]


class icp_params(C.Structure):
    _fields_ = [("mode", C.c_int), ("anderson_m", C.c_int), ("nu_max", C.c_double),
                ("nu_min", C.c_double), ("eps", C.c_double), ("iter_first", C.c_int),
                ("iter_inc", C.c_int), ("iter_cap", C.c_int), ("max_total_iter", C.c_int),
                ("max_line_search", C.c_int), ("nn", C.c_int), ("engine", C.c_int),
                ("T0", C.c_double * 16)]


class icp_result(C.Structure):
    _fields_ = [("T", C.c_double * 16), ("energy", C.c_double), ("nu_final", C.c_double),
                ("iterations", C.c_int), ("nn_passes", C.c_int), ("evaluations", C.c_int),
                ("aa_accepted", C.c_int), ("aa_rejected", C.c_int),
                ("line_search_trials", C.c_int), ("stages", C.c_int),
                ("status_flags", C.c_uint), ("latency_ms", C.c_double),
                ("nn_pairs", C.c_double), ("nn_exact_pairs", C.c_double)]


class icp_profile_stats(C.Structure):
    _fields_ = [("nn_ms", C.c_double), ("reduce_ms", C.c_double), ("solve_ms", C.c_double),
                ("passes", C.c_longlong)]


class icp_tuning(C.Structure):
    _fields_ = [("slice_min", C.c_int), ("list_margin", C.c_float), ("brute_clusters", C.c_int),
                ("brute_items", C.c_int), ("grid_per_cu", C.c_int)]


class icp_tuning_entry(C.Structure):
    _fields_ = [("m_bucket", C.c_int), ("n_bucket", C.c_int), ("mode", C.c_int), ("method", C.c_int),
                ("batch", C.c_int), ("tuning", icp_tuning), ("ms", C.c_double)]


class icp_request(C.Structure):
    _fields_ = [("P", C.c_void_p), ("M", C.c_int64), ("Q", C.c_void_p), ("Qn", C.c_void_p),
                ("N", C.c_int64), ("params", icp_params)]


class ICPError(RuntimeError):
    def __init__(self, status, where):
        super().__init__(f"{where}: {icp_status_str(status)} ({status})")
        self.status = status


_lib = None


def lib():
    """Load libicp.so (built by paper_2007_07627_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libicp.so not found at {LIB_PATH}: build it first "
                               "(python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32 = C.c_void_p, C.c_int64, C.c_int
        L.icp_create.argtypes = [i32, C.c_size_t, C.POINTER(vp)]
        L.icp_destroy.argtypes = [vp]
        L.icp_params_default.argtypes = [i32, C.POINTER(icp_params)]
        L.icp_params_classical.argtypes = [i32, C.POINTER(icp_params)]
        L.icp_register.argtypes = [vp, vp, i64, vp, vp, i64, C.POINTER(icp_params), C.POINTER(icp_result)]
        L.icp_register_trace.argtypes = [vp, vp, i64, vp, vp, i64, C.POINTER(icp_params),
                                         C.POINTER(icp_result), vp, i32, C.POINTER(C.c_int)]
        L.icp_eval.argtypes = [vp, vp, i64, vp, vp, i64, i32, vp, C.c_double,
                               C.POINTER(C.c_double), vp, C.POINTER(C.c_uint)]
        L.icp_trace_items.argtypes = [vp, vp, i32, C.POINTER(C.c_int)]
        L.icp_register_dev.argtypes = [vp, vp, i64, vp, vp, i64, C.POINTER(icp_params),
                                       C.POINTER(icp_result), vp]
        L.icp_nn_query.argtypes = [vp, vp, i64, vp, i64, vp, i32, vp, vp]
        L.icp_nn_query_dev.argtypes = [vp, vp, i64, vp, i64, vp, i32, vp, vp, vp]
        L.icp_nn_query_dev_noalloc.argtypes = [vp, i64, vp, i64, vp, i32, vp, vp, vp]
        L.icp_batch_submit.argtypes = [vp, C.POINTER(icp_request), i32, C.POINTER(C.c_uint64)]
        L.icp_batch_submit_dev.argtypes = [vp, C.POINTER(icp_request), i32, C.POINTER(C.c_uint64), vp]
        L.icp_poll.argtypes = [vp, C.c_uint64, C.POINTER(icp_result)]
        L.icp_nu_min_auto.argtypes = [vp, vp, vp, C.c_int64, i32, C.POINTER(C.c_double)]
        L.icp_estimate_normals.argtypes = [vp, vp, C.c_int64, vp]
        L.icp_batch_wait_all.argtypes = [vp]
        L.icp_batch_config.argtypes = [vp, i32, i32]
        L.icp_profile.argtypes = [vp, i32]
        L.icp_profile_read.argtypes = [vp, C.POINTER(icp_profile_stats)]
        L.icp_tuning_default.argtypes = [C.POINTER(icp_tuning)]
        L.icp_tuning_lookup.argtypes = [vp, i64, i64, i32, i32, i32, C.POINTER(icp_tuning), C.POINTER(C.c_int)]
        L.icp_tuning_set.argtypes = [vp, C.POINTER(icp_tuning_entry)]
        L.icp_tuning_entries.argtypes = [vp, C.POINTER(icp_tuning_entry), i32, C.POINTER(C.c_int)]
        L.icp_autotune.argtypes = [vp, i64, i64, i32, i32, i32, C.POINTER(icp_tuning_entry)]
        L.icp_device_arch.argtypes = [i32, C.c_char_p, i32]
        L.icp_tuning_file_write.argtypes = [C.c_char_p, C.c_char_p, C.POINTER(icp_tuning_entry), i32]
        L.icp_tuning_file_read.argtypes = [C.c_char_p, C.c_char_p, C.POINTER(icp_tuning_entry), i32,
                                           C.POINTER(C.c_int)]
        L.icp_status_str.argtypes = [i32]
        L.icp_status_str.restype = C.c_char_p
        for n in EXPORTED:
            if n != "icp_status_str":
                getattr(L, n).restype = C.c_int
        _lib = L
    return _lib


def icp_status_str(status: int) -> str:
    return lib().icp_status_str(int(status)).decode()


def _check(rc, where):
    if rc != ICP_OK:
        raise ICPError(rc, where)


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32).reshape(-1, 3))


def _ptr(a):
    return None if a is None else a.ctypes.data


def result_dict(r: icp_result) -> dict:
    d = {f: getattr(r, f) for f, _ in icp_result._fields_ if f != "T"}
    d["T"] = np.array(r.T[:], dtype=np.float64).reshape(4, 4)
    return d


# ------------------------------------------------------------------ C ABI wrappers

def icp_create(device: int = 0, hbm_budget_bytes: int = 0):
    h = C.c_void_p()
    _check(lib().icp_create(device, hbm_budget_bytes, C.byref(h)), "icp_create")
    return h


def icp_destroy(ctx):
    _check(lib().icp_destroy(ctx), "icp_destroy")


def icp_params_default(mode: int = ICP_P2P_WELSCH, **overrides) -> icp_params:
    p = icp_params()
    _check(lib().icp_params_default(mode, C.byref(p)), "icp_params_default")
    for k, v in overrides.items():
        if k == "T0":
            p.T0[:] = list(np.asarray(v, dtype=np.float64).reshape(16))
        else:
            setattr(p, k, v)
    return p


def icp_params_classical(mode: int = ICP_P2P_L2, **overrides) -> icp_params:
    """ICP (ICP_P2P_L2) or ICP-l (ICP_P2PL_L2) with the comparison methods'
    settings: no mixing, no line search, 1000 iterations, ||dT||_F^2 < 1e-5."""
    p = icp_params()
    _check(lib().icp_params_classical(mode, C.byref(p)), "icp_params_classical")
    for k, v in overrides.items():
        if k == "T0":
            p.T0[:] = list(np.asarray(v, dtype=np.float64).reshape(16))
        else:
            setattr(p, k, v)
    return p


def icp_register(ctx, P, Q, Qn=None, params: icp_params | None = None, raw=False):
    P, Q = _f32(P), _f32(Q)
    Qn = None if Qn is None else _f32(Qn)
    params = params or icp_params_default()
    r = icp_result()
    rc = lib().icp_register(ctx, _ptr(P), P.shape[0], _ptr(Q), _ptr(Qn), Q.shape[0],
                            C.byref(params), C.byref(r))
    if raw:
        return rc, r
    _check(rc, "icp_register")
    return result_dict(r)


def icp_register_trace(ctx, P, Q, Qn=None, params: icp_params | None = None, cap: int = 100000):
    """Registration plus the per-pass trace: rows [E, nu, state, reuse, T(16),
    update(16)] (ICP_TRACE_ROW doubles)."""
    P, Q = _f32(P), _f32(Q)
    Qn = None if Qn is None else _f32(Qn)
    params = params or icp_params_default()
    r = icp_result()
    tr = np.zeros((cap, ICP_TRACE_ROW))
    n = C.c_int(0)
    rc = lib().icp_register_trace(ctx, _ptr(P), P.shape[0], _ptr(Q), _ptr(Qn), Q.shape[0],
                                  C.byref(params), C.byref(r), tr.ctypes.data, cap, C.byref(n))
    _check(rc, "icp_register_trace")
    d = result_dict(r)
    d["trace"] = tr[: n.value].copy()
    return d


def icp_eval(ctx, P, Q, Qn, mode, T, nu=0.0, raw=False):
    """One un-accelerated map application at T: returns (energy, T_next, flags)."""
    P, Q = _f32(P), _f32(Q)
    Qn = None if Qn is None else _f32(Qn)
    T = np.ascontiguousarray(np.asarray(T, np.float64).reshape(4, 4))
    E = C.c_double(0.0)
    Tn = np.zeros((4, 4))
    fl = C.c_uint(0)
    rc = lib().icp_eval(ctx, _ptr(P), P.shape[0], _ptr(Q), _ptr(Qn), Q.shape[0], mode,
                        T.ctypes.data, float(nu), C.byref(E), Tn.ctypes.data, C.byref(fl))
    if raw:
        return rc
    _check(rc, "icp_eval")
    return E.value, Tn, fl.value


def icp_trace_items(ctx, cap: int = 1 << 20):
    """Per-work-item diagnostics of the last traced registration's last pass."""
    out = np.zeros((cap, 8), np.int32)
    n = C.c_int(0)
    _check(lib().icp_trace_items(ctx, out.ctypes.data, cap, C.byref(n)), "icp_trace_items")
    return out[: min(n.value, cap)].copy()


def icp_register_dev(ctx, P_t, Q_t, Qn_t=None, params: icp_params | None = None, stream=None):
    """Device variant: torch tensors (contiguous float32, shape (n, 3)) in HBM."""
    params = params or icp_params_default()
    r = icp_result()
    st = None if stream is None else int(stream.cuda_stream)
    rc = lib().icp_register_dev(ctx, P_t.data_ptr(), P_t.shape[0], Q_t.data_ptr(),
                                None if Qn_t is None else Qn_t.data_ptr(), Q_t.shape[0],
                                C.byref(params), C.byref(r), st)
    _check(rc, "icp_register_dev")
    return result_dict(r)


def icp_estimate_normals(ctx, Q, raw=False):
    """Normals from the 30 nearest points (the point included), FP64 PCA."""
    Q = _f32(Q)
    out = np.zeros_like(Q)
    rc = lib().icp_estimate_normals(ctx, _ptr(Q), Q.shape[0], _ptr(out))
    if raw:
        return rc, out
    _check(rc, "icp_estimate_normals")
    return out


def icp_nu_min_auto(ctx, Q, Qn=None, mode: int = ICP_P2P_WELSCH, raw=False):
    """Automatic nu_min of a target set (the value params.nu_min <= 0 selects)."""
    Q = _f32(Q)
    Qn = None if Qn is None else _f32(Qn)
    out = C.c_double(0.0)
    rc = lib().icp_nu_min_auto(ctx, _ptr(Q), _ptr(Qn), Q.shape[0], int(mode), C.byref(out))
    if raw:
        return rc, out.value
    _check(rc, "icp_nu_min_auto")
    return out.value


def icp_nn_query(ctx, P, Q, T=None, method: int = ICP_NN_AUTO, raw=False):
    P, Q = _f32(P), _f32(Q)
    T = np.ascontiguousarray(np.eye(4) if T is None else np.asarray(T, np.float64).reshape(4, 4))
    idx = np.empty(P.shape[0], np.int32)
    d2 = np.empty(P.shape[0], np.float32)
    rc = lib().icp_nn_query(ctx, _ptr(P) if P.shape[0] else None, P.shape[0], _ptr(Q), Q.shape[0],
                            T.ctypes.data, method, _ptr(idx) if P.shape[0] else None,
                            _ptr(d2) if P.shape[0] else None)
    if raw:
        return rc, idx, d2
    _check(rc, "icp_nn_query")
    return idx, d2


def icp_nn_query_dev(ctx, P_t, Q_t, T, method, idx_t, d2_t, stream=None):
    T = np.ascontiguousarray(np.asarray(T, np.float64).reshape(4, 4))
    st = None if stream is None else int(stream.cuda_stream)
    rc = lib().icp_nn_query_dev(ctx, P_t.data_ptr(), P_t.shape[0], Q_t.data_ptr(), Q_t.shape[0],
                                T.ctypes.data, method, idx_t.data_ptr(), d2_t.data_ptr(), st)
    _check(rc, "icp_nn_query_dev")


def icp_nn_query_dev_noalloc(P_t, Q_t, T, method, idx_t, d2_t, stream=None, raw=False):
    """Allocation-free closest-point query on the current device (no context):
    enqueued on `stream`, outputs ready when the stream reaches that point."""
    T = np.ascontiguousarray(np.asarray(T, np.float64).reshape(4, 4))
    st = None if stream is None else int(stream.cuda_stream)
    rc = lib().icp_nn_query_dev_noalloc(P_t.data_ptr(), P_t.shape[0], Q_t.data_ptr(), Q_t.shape[0],
                                        T.ctypes.data, method, idx_t.data_ptr(), d2_t.data_ptr(), st)
    if raw:
        return rc
    _check(rc, "icp_nn_query_dev_noalloc")


def icp_batch_submit(ctx, requests):
    """requests: iterable of (P, Q, Qn_or_None, icp_params). Returns tickets."""
    keep = []
    arr = (icp_request * len(requests))()
    for i, (P, Q, Qn, prm) in enumerate(requests):
        P, Q = _f32(P), _f32(Q)
        Qn = None if Qn is None else _f32(Qn)
        keep.append((P, Q, Qn))
        arr[i].P = _ptr(P)
        arr[i].M = P.shape[0]
        arr[i].Q = _ptr(Q)
        arr[i].Qn = _ptr(Qn)
        arr[i].N = Q.shape[0]
        arr[i].params = prm
    t = (C.c_uint64 * len(requests))()
    _check(lib().icp_batch_submit(ctx, arr, len(requests), t), "icp_batch_submit")
    return list(t)


def icp_batch_submit_dev(ctx, requests, stream=None, raw=False):
    """requests: iterable of (P_t, Q_t, Qn_t_or_None, icp_params) with torch
    tensors in HBM (contiguous float32, shape (n, 3)), kept alive by the
    caller until their results are polled. Returns tickets."""
    arr = (icp_request * len(requests))()
    for i, (P, Q, Qn, prm) in enumerate(requests):
        arr[i].P = P.data_ptr()
        arr[i].M = P.shape[0]
        arr[i].Q = Q.data_ptr()
        arr[i].Qn = None if Qn is None else Qn.data_ptr()
        arr[i].N = Q.shape[0]
        arr[i].params = prm
    t = (C.c_uint64 * len(requests))()
    st = None if stream is None else int(stream.cuda_stream)
    rc = lib().icp_batch_submit_dev(ctx, arr, len(requests), t, st)
    if raw:
        return rc, list(t)
    _check(rc, "icp_batch_submit_dev")
    return list(t)


def icp_poll(ctx, ticket):
    """Returns (status, result dict or None)."""
    r = icp_result()
    rc = lib().icp_poll(ctx, C.c_uint64(ticket), C.byref(r))
    return rc, (result_dict(r) if rc == ICP_OK else None)


def icp_batch_wait_all(ctx):
    _check(lib().icp_batch_wait_all(ctx), "icp_batch_wait_all")


def icp_batch_config(ctx, passes_per_replay: int, max_slots: int):
    _check(lib().icp_batch_config(ctx, passes_per_replay, max_slots), "icp_batch_config")


def tuning_dict(t: icp_tuning) -> dict:
    return {f: getattr(t, f) for f, _ in icp_tuning._fields_}


def entry_dict(e: icp_tuning_entry) -> dict:
    d = {f: getattr(e, f) for f in ("m_bucket", "n_bucket", "mode", "method", "batch", "ms")}
    d["tuning"] = tuning_dict(e.tuning)
    return d


def make_entry(m_bucket, n_bucket, mode, method, ms=0.0, batch=0, **tuning) -> icp_tuning_entry:
    e = icp_tuning_entry()
    e.m_bucket, e.n_bucket, e.mode, e.method, e.ms, e.batch = m_bucket, n_bucket, mode, method, ms, batch
    t = icp_tuning()
    _check(lib().icp_tuning_default(C.byref(t)), "icp_tuning_default")
    for k, v in tuning.items():
        setattr(t, k, v)
    e.tuning = t
    return e


def icp_tuning_default() -> dict:
    t = icp_tuning()
    _check(lib().icp_tuning_default(C.byref(t)), "icp_tuning_default")
    return tuning_dict(t)


def icp_tuning_lookup(ctx, M, N, mode, method, batch=0):
    """(tuning dict, found: 2 exact bucket, 1 nearby, 0 defaults) for the
    synchronous calls (batch=0) or the batch engine (batch=1)."""
    t = icp_tuning()
    f = C.c_int(0)
    _check(lib().icp_tuning_lookup(ctx, M, N, mode, method, batch, C.byref(t), C.byref(f)),
           "icp_tuning_lookup")
    return tuning_dict(t), f.value


def icp_tuning_set(ctx, entry: icp_tuning_entry, raw=False):
    rc = lib().icp_tuning_set(ctx, C.byref(entry))
    if raw:
        return rc
    _check(rc, "icp_tuning_set")


def icp_tuning_entries(ctx, cap=4096):
    arr = (icp_tuning_entry * cap)()
    n = C.c_int(0)
    _check(lib().icp_tuning_entries(ctx, arr, cap, C.byref(n)), "icp_tuning_entries")
    return [arr[i] for i in range(min(cap, n.value))]


def icp_autotune(ctx, M, N, mode, method, batch=0) -> icp_tuning_entry:
    e = icp_tuning_entry()
    _check(lib().icp_autotune(ctx, M, N, mode, method, batch, C.byref(e)), "icp_autotune")
    return e


def icp_device_arch(device=0) -> str:
    buf = C.create_string_buffer(64)
    _check(lib().icp_device_arch(device, buf, 64), "icp_device_arch")
    return buf.value.decode()


def icp_tuning_file_write(path, arch, entries, raw=False):
    arr = (icp_tuning_entry * max(1, len(entries)))(*entries)
    rc = lib().icp_tuning_file_write(path.encode(), arch.encode(), arr, len(entries))
    if raw:
        return rc
    _check(rc, "icp_tuning_file_write")


def icp_tuning_file_read(path, arch=None, cap=4096, raw=False):
    arr = (icp_tuning_entry * cap)()
    n = C.c_int(0)
    rc = lib().icp_tuning_file_read(path.encode(), None if arch is None else arch.encode(), arr, cap,
                                    C.byref(n))
    if raw:
        return rc, [arr[i] for i in range(min(cap, n.value))]
    _check(rc, "icp_tuning_file_read")
    return [arr[i] for i in range(min(cap, n.value))]


def icp_profile(ctx, enable: bool):
    _check(lib().icp_profile(ctx, 1 if enable else 0), "icp_profile")


def icp_profile_read(ctx) -> dict:
    st = icp_profile_stats()
    _check(lib().icp_profile_read(ctx, C.byref(st)), "icp_profile_read")
    return {f: getattr(st, f) for f, _ in icp_profile_stats._fields_}
