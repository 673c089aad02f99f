"""ctypes binding of librkkt.so (include/rkkt.h).  Argument marshalling only:
every computation runs in the library's HIP kernels.

Device arrays are torch tensors (float64, contiguous, on the GPU); their
``data_ptr()`` is passed.  Host arrays (the network, the initial loads) are
numpy arrays.  Functions keep the C names; errors raise ``RkktError``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librkkt.so")

c_int_p = ctypes.POINTER(ctypes.c_int)
c_dbl_p = ctypes.POINTER(ctypes.c_double)

RKKT_OK = 0
ERRORS = {-1: "RKKT_ERR_ARG", -2: "RKKT_ERR_HIP", -3: "RKKT_ERR_SINGULAR_GX",
          -4: "RKKT_ERR_NOT_PD", -5: "RKKT_ERR_NONFINITE", -6: "RKKT_ERR_NOMEM"}
EXPORTS = ("rkkt_create", "rkkt_analyze", "rkkt_set_loads", "rkkt_dims_get", "rkkt_evaluate",
           "rkkt_condense", "rkkt_factor", "rkkt_step", "rkkt_status", "rkkt_destroy",
           "rkkt_last_error", "rkkt_profile_begin", "rkkt_profile_end", "rkkt_solve",
           "rkkt_iterate", "rkkt_graph_capture", "rkkt_graph_launch", "rkkt_batch_create",
           "rkkt_batch_launch", "rkkt_batch_destroy", "rkkt_autotune", "rkkt_analyze_lu",
           "rkkt_analyze_schedule", "rkkt_set_line_status", "rkkt_solve_warm", "rkkt_multi_create",
           "rkkt_multi_iterate", "rkkt_multi_capture", "rkkt_multi_launch", "rkkt_multi_launches",
           "rkkt_multi_destroy", "rkkt_multi_last_error", "rkkt_probe_peaks")
MLP_EXPORTS = ("rkkt_mlp_create", "rkkt_mlp_destroy", "rkkt_mlp_last_error", "rkkt_mlp_n_params",
               "rkkt_mlp_set_params", "rkkt_mlp_get_params", "rkkt_mlp_forward", "rkkt_mlp_gradients",
               "rkkt_mlp_train_step", "rkkt_mlp_forward_static")
IPM_STATUS = {0: "converged", 1: "max_iter", 2: "line_search_failed",
              3: "inertia_correction_failed", 4: "device_error"}
STAGES = ("evaluate", "condense_values", "refactor", "reduce", "scenario_sum", "factor",
          "step_rhs", "reduced_solve", "step_recover", "stacked_product")


class RkktError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Network(ctypes.Structure):
    _fields_ = [("n_bus", ctypes.c_int), ("n_line", ctypes.c_int), ("n_gen", ctypes.c_int),
                ("n_load", ctypes.c_int), ("ref_bus", ctypes.c_int),
                ("line_from", c_int_p), ("line_to", c_int_p),
                ("r", c_dbl_p), ("x", c_dbl_p), ("b", c_dbl_p), ("rate", c_dbl_p),
                ("gen_bus", c_int_p),
                ("pmin", c_dbl_p), ("pmax", c_dbl_p), ("qmin", c_dbl_p), ("qmax", c_dbl_p),
                ("c2", c_dbl_p), ("c1", c_dbl_p), ("c0", c_dbl_p),
                ("vmin", c_dbl_p), ("vmax", c_dbl_p), ("load_bus", c_int_p)]


class Options(ctypes.Structure):
    _fields_ = [("col_tile", ctypes.c_int), ("device", ctypes.c_int), ("variant", ctypes.c_int),
                ("scen_per_group", ctypes.c_int), ("chain_rows", ctypes.c_int),
                ("sweep_form", ctypes.c_int)]


class Dims(ctypes.Structure):
    _fields_ = [("n_x", ctypes.c_int), ("n_u", ctypes.c_int), ("m", ctypes.c_int),
                ("n_scen", ctypes.c_int), ("n_bus", ctypes.c_int), ("n_line", ctypes.c_int),
                ("n_gen", ctypes.c_int),
                ("nnz_gx", ctypes.c_longlong), ("nnz_gu", ctypes.c_longlong),
                ("nnz_h", ctypes.c_longlong), ("nnz_k", ctypes.c_longlong),
                ("nnz_lu", ctypes.c_longlong), ("lu_update_flops", ctypes.c_longlong),
                ("nnz_kx", ctypes.c_longlong), ("n_ev", ctypes.c_longlong),
                ("n_trip", ctypes.c_longlong),
                ("levels_up", ctypes.c_int), ("levels_down", ctypes.c_int),
                ("col_tile", ctypes.c_int), ("workspace_bytes", ctypes.c_longlong),
                ("variant", ctypes.c_int), ("lds_reduce", ctypes.c_int),
                ("lds_group", ctypes.c_int), ("scen_per_group", ctypes.c_int),
                ("lds_step", ctypes.c_int), ("chain_rows", ctypes.c_int),
                ("nnz_kxx", ctypes.c_longlong), ("nnz_kxu", ctypes.c_longlong),
                ("nnz_kuu", ctypes.c_longlong), ("idx_bytes", ctypes.c_longlong),
                ("n_load", ctypes.c_int), ("sweep_form", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_ITER_FIELDS = ("x", "u", "y", "z", "obj_weight", "f", "grad_x", "grad_u", "g", "h", "sigma_x",
                "sigma_u", "sigma_s", "delta_w", "khat", "chol", "info", "r1x", "r1u", "r2", "r3",
                "r4", "px", "pu", "ps", "py", "pz")


class Iteration(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double if n in ("obj_weight", "delta_w") else ctypes.c_void_p)
                for n in _ITER_FIELDS]


class IpmOptions(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("mu0", ctypes.c_double),
                ("verbose", ctypes.c_int), ("warm_duals", ctypes.c_int)]


class IpmResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("obj", ctypes.c_double),
                ("kkt_error", ctypes.c_double), ("mu", ctypes.c_double),
                ("obj_weight", ctypes.c_double), ("factorizations", ctypes.c_int)]


_lib = None


def lib():
    """Load librkkt.so (built in place by paper_2301_04869_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2301_04869_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    L.rkkt_create.argtypes = [ctypes.POINTER(Network), ctypes.c_int, c_dbl_p, c_dbl_p,
                              ctypes.POINTER(Options), ctypes.POINTER(vp)]
    L.rkkt_analyze.argtypes = [ctypes.POINTER(Network), ctypes.c_int, ctypes.POINTER(Options),
                               ctypes.POINTER(Dims)]
    L.rkkt_set_loads.argtypes = [vp, vp, vp, vp]
    L.rkkt_set_line_status.argtypes = [vp, vp, vp]
    L.rkkt_dims_get.argtypes = [vp, ctypes.POINTER(Dims)]
    L.rkkt_evaluate.argtypes = [vp, vp, vp, vp, vp, ctypes.c_double, vp, vp, vp, vp, vp, vp]
    L.rkkt_condense.argtypes = [vp, vp, vp, vp, ctypes.c_double, vp, vp]
    L.rkkt_factor.argtypes = [vp, vp, vp, vp]
    L.rkkt_step.argtypes = [vp] + [vp] * 12 + [vp]
    L.rkkt_status.argtypes = [vp, vp, c_int_p, c_int_p]
    L.rkkt_destroy.argtypes = [vp]
    L.rkkt_profile_begin.argtypes = [vp, ctypes.c_int]
    L.rkkt_probe_peaks.argtypes = [ctypes.c_int] + [ctypes.POINTER(ctypes.c_double)] * 3
    L.rkkt_profile_end.argtypes = [vp, vp, c_dbl_p, c_int_p]
    L.rkkt_solve.argtypes = [vp, ctypes.POINTER(IpmOptions), vp, vp, vp, vp, vp,
                             ctypes.POINTER(IpmResult), vp]
    L.rkkt_solve_warm.argtypes = [vp, ctypes.POINTER(IpmOptions), vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                  ctypes.POINTER(IpmResult), vp]
    L.rkkt_iterate.argtypes = [vp, ctypes.POINTER(Iteration), vp]
    L.rkkt_graph_capture.argtypes = [vp, ctypes.POINTER(Iteration)]
    L.rkkt_graph_launch.argtypes = [vp, vp]
    L.rkkt_multi_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Iteration), ctypes.c_int,
                                    ctypes.POINTER(vp)]
    L.rkkt_multi_iterate.argtypes = [vp, vp]
    L.rkkt_multi_capture.argtypes = [vp]
    L.rkkt_multi_launch.argtypes = [vp, vp]
    L.rkkt_multi_launches.argtypes = [vp]
    L.rkkt_multi_destroy.argtypes = [vp]
    L.rkkt_multi_last_error.argtypes = [vp]
    L.rkkt_multi_last_error.restype = ctypes.c_char_p
    L.rkkt_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Iteration), ctypes.c_int,
                                    ctypes.POINTER(vp)]
    L.rkkt_batch_launch.argtypes = [vp, vp]
    L.rkkt_batch_destroy.argtypes = [vp]
    L.rkkt_autotune.argtypes = [ctypes.POINTER(Network), ctypes.c_int, c_dbl_p, c_dbl_p,
                                ctypes.POINTER(Options), ctypes.c_int, ctypes.POINTER(Options),
                                c_dbl_p]
    L.rkkt_analyze_lu.argtypes = [ctypes.POINTER(Network), ctypes.c_int, ctypes.POINTER(Options),
                                  c_int_p, c_int_p, c_int_p]
    L.rkkt_analyze_schedule.argtypes = [ctypes.POINTER(Network), ctypes.c_int, ctypes.POINTER(Options),
                                        ctypes.c_int] + [c_int_p] * 9
    L.rkkt_last_error.argtypes = [vp]
    L.rkkt_last_error.restype = ctypes.c_char_p
    L.rkkt_mlp_create.argtypes = [c_int_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(vp)]
    L.rkkt_mlp_destroy.argtypes = [vp]
    L.rkkt_mlp_last_error.argtypes = [vp]
    L.rkkt_mlp_last_error.restype = ctypes.c_char_p
    L.rkkt_mlp_n_params.argtypes = [vp]
    L.rkkt_mlp_n_params.restype = ctypes.c_longlong
    L.rkkt_mlp_set_params.argtypes = [vp, vp, vp]
    L.rkkt_mlp_get_params.argtypes = [vp, vp, vp]
    L.rkkt_mlp_forward.argtypes = [vp, vp, ctypes.c_int, vp, vp]
    L.rkkt_mlp_forward_static.argtypes = [vp, vp, ctypes.c_int, vp, vp]
    L.rkkt_mlp_gradients.argtypes = [vp, vp, vp, ctypes.c_int, vp, vp, vp]
    L.rkkt_mlp_train_step.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_float, vp, vp]
    for name in ("rkkt_mlp_create", "rkkt_mlp_destroy", "rkkt_mlp_set_params", "rkkt_mlp_get_params",
                 "rkkt_mlp_forward", "rkkt_mlp_gradients", "rkkt_mlp_train_step", "rkkt_mlp_forward_static"):
        getattr(L, name).restype = ctypes.c_int
    for name in EXPORTS:
        if not name.endswith("last_error"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc, handle=None):
    if rc != RKKT_OK:
        msg = lib().rkkt_last_error(handle).decode()
        raise RkktError(rc, msg)


def _host_network(net):
    """Build the C struct from an object with the synthgrid.Network fields.
    Returns (struct, keepalive list)."""
    keep = []

    def ia(a):
        a = np.ascontiguousarray(a, dtype=np.int32)
        keep.append(a)
        return a.ctypes.data_as(c_int_p)

    def da(a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        keep.append(a)
        return a.ctypes.data_as(c_dbl_p)
    s = Network(int(net.n_bus), int(net.n_line), int(net.n_gen), int(len(net.load_bus)),
                int(net.ref_bus), ia(net.line_from), ia(net.line_to), da(net.r), da(net.x),
                da(net.b), da(net.rate), ia(net.gen_bus), da(net.pmin), da(net.pmax),
                da(net.qmin), da(net.qmax), da(net.c2), da(net.c1), da(net.c0),
                da(net.vmin), da(net.vmax), ia(net.load_bus))
    return s, keep


def _ptr(t, name, numel=None):
    if t is None:
        raise ValueError(f"{name} is None")
    if not (t.is_cuda and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous device tensor")
    if str(t.dtype) != "torch.float64":
        raise ValueError(f"{name} must be float64")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(getattr(stream, "cuda_stream", stream))


class Handle:
    """An rkkt_problem* with its dimensions; destroyed with the object."""

    def __init__(self, ptr, dims):
        self.ptr = ptr
        self.dims = dims

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.rkkt_destroy(self.ptr)
            self.ptr = None


def rkkt_analyze(net, n_scen, col_tile=0, variant=0, scen_per_group=0, chain_rows=0, sweep_form=0):
    s, keep = _host_network(net)
    d = Dims()
    _check(lib().rkkt_analyze(ctypes.byref(s), int(n_scen),
                              ctypes.byref(Options(col_tile, 0, variant, scen_per_group, chain_rows,
                                                   sweep_form)),
                              ctypes.byref(d)))
    return d.as_dict()


def rkkt_create(net, pd, qd, col_tile=0, device=0, variant=0, scen_per_group=0, chain_rows=0, sweep_form=0):
    """pd, qd: host [N][n_load] arrays (scenario-major); the launch-shape
    options of rkkt_options (0 = automatic)."""
    s, keep = _host_network(net)
    pd = np.ascontiguousarray(pd, dtype=np.float64)
    qd = np.ascontiguousarray(qd, dtype=np.float64)
    if pd.ndim != 2 or pd.shape != qd.shape or pd.shape[1] != len(net.load_bus):
        raise ValueError("pd, qd must be [N][n_load]")
    h = ctypes.c_void_p()
    _check(lib().rkkt_create(ctypes.byref(s), pd.shape[0], pd.ctypes.data_as(c_dbl_p),
                             qd.ctypes.data_as(c_dbl_p),
                             ctypes.byref(Options(col_tile, device, variant, scen_per_group,
                                                  chain_rows, sweep_form)),
                             ctypes.byref(h)))
    d = Dims()
    _check(lib().rkkt_dims_get(h, ctypes.byref(d)), h)
    return Handle(h, d.as_dict())


def rkkt_analyze_lu(net, n_scen, col_tile=0):
    """Returns (perm, f_ptr, f_col) numpy int32 arrays of the filled LU pattern."""
    d = rkkt_analyze(net, n_scen, col_tile)
    s, keep = _host_network(net)
    perm = np.zeros(d["n_x"], dtype=np.int32)
    fp = np.zeros(d["n_x"] + 1, dtype=np.int32)
    fc = np.zeros(d["nnz_lu"], dtype=np.int32)
    _check(lib().rkkt_analyze_lu(ctypes.byref(s), int(n_scen), ctypes.byref(Options(col_tile, 0)),
                                 perm.ctypes.data_as(c_int_p), fp.ctypes.data_as(c_int_p),
                                 fc.ctypes.data_as(c_int_p)))
    return perm, fp, fc


SCHEDULES = ("reduce_up", "reduce_down", "step_up", "step_down", "refactor")


def rkkt_analyze_schedule(net, n_scen, which, col_tile=0, variant=0, scen_per_group=0, chain_rows=0,
                          sweep_form=0):
    """Host-only export of a level-sliced schedule: dict with nphase, slots,
    ptr [nphase*slots+1], ent [n_ent][4], chain_rows, chain_pos [t][t]."""
    s, keep = _host_network(net)
    w = SCHEDULES.index(which) if isinstance(which, str) else int(which)
    o = Options(col_tile, 0, variant, scen_per_group, chain_rows, sweep_form)
    nph, sl, ne, ct, nu_ = (ctypes.c_int() for _ in range(5))
    L = lib()
    _check(L.rkkt_analyze_schedule(ctypes.byref(s), int(n_scen), ctypes.byref(o), w, ctypes.byref(nph),
                                   ctypes.byref(sl), ctypes.byref(ne), ctypes.byref(ct), None, None, None,
                                   ctypes.byref(nu_), None))
    ptr = np.zeros(nph.value * sl.value + 1, dtype=np.int32)
    ent = np.zeros((ne.value, 4), dtype=np.int32)
    cp = np.zeros((ct.value, ct.value), dtype=np.int32)
    upd = np.zeros(max(nu_.value, 1), dtype=np.int32)
    _check(L.rkkt_analyze_schedule(ctypes.byref(s), int(n_scen), ctypes.byref(o), w, ctypes.byref(nph),
                                   ctypes.byref(sl), ctypes.byref(ne), ctypes.byref(ct),
                                   ptr.ctypes.data_as(c_int_p), ent.ctypes.data_as(c_int_p),
                                   cp.ctypes.data_as(c_int_p), ctypes.byref(nu_),
                                   upd.ctypes.data_as(c_int_p)))
    return {"nphase": nph.value, "slots": sl.value, "ptr": ptr, "ent": ent, "chain_rows": ct.value,
            "chain_pos": cp, "upd": upd[:nu_.value]}


def rkkt_autotune(net, pd, qd, reps=5, device=0):
    """Returns (the fastest launch shape as rkkt_create keyword arguments,
    its mean time of one hot-path pass in ms)."""
    s, keep = _host_network(net)
    pd = np.ascontiguousarray(pd, dtype=np.float64)
    qd = np.ascontiguousarray(qd, dtype=np.float64)
    best = Options()
    ms = ctypes.c_double()
    _check(lib().rkkt_autotune(ctypes.byref(s), pd.shape[0], pd.ctypes.data_as(c_dbl_p),
                               qd.ctypes.data_as(c_dbl_p), ctypes.byref(Options(0, device, 0)),
                               int(reps), ctypes.byref(best), ctypes.byref(ms)))
    return ({"col_tile": best.col_tile, "variant": best.variant, "scen_per_group": best.scen_per_group,
             "chain_rows": best.chain_rows, "sweep_form": best.sweep_form}, ms.value)


def rkkt_dims_get(p):
    d = Dims()
    _check(lib().rkkt_dims_get(p.ptr, ctypes.byref(d)), p.ptr)
    return d.as_dict()


def rkkt_set_loads(p, pd, qd, stream=None):
    """pd, qd: device [N][n_load] tensors."""
    _check(lib().rkkt_set_loads(p.ptr, _ptr(pd, "pd"), _ptr(qd, "qd"), _stream(stream)), p.ptr)


def rkkt_set_line_status(p, status, stream=None):
    """status: device [N][n_line] float64 tensor, 1 in service, 0 tripped."""
    d = p.dims
    if tuple(status.shape) != (d["n_scen"], d["n_line"]):
        raise ValueError("status must be [N][n_line]")
    _check(lib().rkkt_set_line_status(p.ptr, _ptr(status, "status"), _stream(stream)), p.ptr)


def rkkt_evaluate(p, x, u, y, z, obj_weight, f, grad_x, grad_u, g, h, stream=None):
    d = p.dims
    N, nx, nu, m = d["n_scen"], d["n_x"], d["n_u"], d["m"]
    _check(lib().rkkt_evaluate(p.ptr, _ptr(x, "x", N * nx), _ptr(u, "u", nu), _ptr(y, "y", N * nx),
                               _ptr(z, "z", N * m), float(obj_weight), _ptr(f, "f", N),
                               _ptr(grad_x, "grad_x", N * nx), _ptr(grad_u, "grad_u", N * nu),
                               _ptr(g, "g", N * nx), _ptr(h, "h", N * m), _stream(stream)), p.ptr)


def rkkt_condense(p, sigma_x, sigma_u, sigma_s, delta_w, khat, stream=None):
    d = p.dims
    N, nx, nu, m = d["n_scen"], d["n_x"], d["n_u"], d["m"]
    _check(lib().rkkt_condense(p.ptr, _ptr(sigma_x, "sigma_x", N * nx), _ptr(sigma_u, "sigma_u", nu),
                               _ptr(sigma_s, "sigma_s", N * m), float(delta_w),
                               _ptr(khat, "khat", nu * nu), _stream(stream)), p.ptr)


def rkkt_factor(p, khat, info, stream=None):
    nu = p.dims["n_u"]
    if not (info.is_cuda and str(info.dtype) == "torch.int32" and info.numel() >= 1):
        raise ValueError("info must be a device int32 tensor")
    _check(lib().rkkt_factor(p.ptr, _ptr(khat, "khat", nu * nu), ctypes.c_void_p(info.data_ptr()),
                             _stream(stream)), p.ptr)


def rkkt_step(p, r1x, r1u, r2, r3, r4, sigma_s, chol, px, pu, ps, py, pz, stream=None):
    d = p.dims
    N, nx, nu, m = d["n_scen"], d["n_x"], d["n_u"], d["m"]
    _check(lib().rkkt_step(p.ptr, _ptr(r1x, "r1x", N * nx), _ptr(r1u, "r1u", nu),
                           _ptr(r2, "r2", N * m), _ptr(r3, "r3", N * nx), _ptr(r4, "r4", N * m),
                           _ptr(sigma_s, "sigma_s", N * m), _ptr(chol, "chol", nu * nu),
                           _ptr(px, "px", N * nx), _ptr(pu, "pu", nu), _ptr(ps, "ps", N * m),
                           _ptr(py, "py", N * nx), _ptr(pz, "pz", N * m), _stream(stream)), p.ptr)


def rkkt_status(p, stream=None):
    code = ctypes.c_int()
    scen = ctypes.c_int()
    _check(lib().rkkt_status(p.ptr, _stream(stream), ctypes.byref(code), ctypes.byref(scen)), p.ptr)
    return code.value, scen.value


def rkkt_profile_begin(p, max_records):
    _check(lib().rkkt_profile_begin(p.ptr, int(max_records)), p.ptr)


def rkkt_profile_end(p, stream=None):
    """Returns {stage: (total ms, records)}."""
    ms = (ctypes.c_double * len(STAGES))()
    cnt = (ctypes.c_int * len(STAGES))()
    _check(lib().rkkt_profile_end(p.ptr, _stream(stream), ms, cnt), p.ptr)
    return {s: (ms[i], cnt[i]) for i, s in enumerate(STAGES)}


def rkkt_probe_peaks(device=0):
    """Measured machine balance: {"hbm_gbs", "fp64_vec_tfs", "fp64_mfma_tfs"}
    (copy, FP64 multiply-add and FP64 matrix-core probes)."""
    out = [ctypes.c_double() for _ in range(3)]
    _check(lib().rkkt_probe_peaks(int(device), *[ctypes.byref(v) for v in out]))
    return {"hbm_gbs": out[0].value, "fp64_vec_tfs": out[1].value, "fp64_mfma_tfs": out[2].value}


def rkkt_solve(p, x=None, u=None, y=None, z=None, s=None, tol=0.0, max_iter=-1, mu0=0.0,
               verbose=False, stream=None):
    """Device interior-point solve; optional device outputs x, u, y, z, s.
    Returns the result fields as a dict (status as text)."""
    d = p.dims
    N, nx, nu, m = d["n_scen"], d["n_x"], d["n_u"], d["m"]

    def opt(t, name, n):
        return ctypes.c_void_p(None) if t is None else _ptr(t, name, n)
    r = IpmResult()
    _check(lib().rkkt_solve(p.ptr, ctypes.byref(IpmOptions(tol, max_iter, mu0, int(verbose), 0)),
                            opt(x, "x", N * nx), opt(u, "u", nu), opt(y, "y", N * nx),
                            opt(z, "z", N * m), opt(s, "s", N * m), ctypes.byref(r),
                            _stream(stream)), p.ptr)
    out = {k: getattr(r, k) for k, _ in r._fields_}
    out["status"] = IPM_STATUS.get(out["status"], out["status"])
    return out


def rkkt_solve_warm(p, x0, u0, y0, z0, x=None, u=None, y=None, z=None, s=None, tol=0.0, max_iter=-1,
                    mu0=0.0, verbose=False, warm_duals=0, stream=None):
    """Device interior-point solve from a start point (device float64 x0
    [N][n_x], u0 [n_u], y0 [N][n_x], z0 [N][m]; multipliers for the objective
    weighted 1/N).  Returns the result fields as a dict."""
    d = p.dims
    N, nx, nu, m = d["n_scen"], d["n_x"], d["n_u"], d["m"]

    def opt(t, name, n):
        return ctypes.c_void_p(None) if t is None else _ptr(t, name, n)
    r = IpmResult()
    _check(lib().rkkt_solve_warm(p.ptr, ctypes.byref(IpmOptions(tol, max_iter, mu0, int(verbose),
                                                                int(warm_duals))),
                                 _ptr(x0, "x0", N * nx), _ptr(u0, "u0", nu), _ptr(y0, "y0", N * nx),
                                 _ptr(z0, "z0", N * m), opt(x, "x", N * nx), opt(u, "u", nu),
                                 opt(y, "y", N * nx), opt(z, "z", N * m), opt(s, "s", N * m),
                                 ctypes.byref(r), _stream(stream)), p.ptr)
    out = {k: getattr(r, k) for k, _ in r._fields_}
    out["status"] = IPM_STATUS.get(out["status"], out["status"])
    return out


def _iteration(p, a):
    """Marshal a dict of tensors / scalars into the rkkt_iteration struct."""
    d = p.dims
    N, nx, nu, m = d["n_scen"], d["n_x"], d["n_u"], d["m"]
    sizes = dict(x=N * nx, u=nu, y=N * nx, z=N * m, f=N, grad_x=N * nx, grad_u=N * nu, g=N * nx,
                 h=N * m, sigma_x=N * nx, sigma_u=nu, sigma_s=N * m, khat=nu * nu, chol=nu * nu,
                 r1x=N * nx, r1u=nu, r2=N * m, r3=N * nx, r4=N * m, px=N * nx, pu=nu, ps=N * m,
                 py=N * nx, pz=N * m)
    vals = []
    for n in _ITER_FIELDS:
        if n in ("obj_weight", "delta_w"):
            vals.append(float(a[n]))
        elif n == "info":
            t = a[n]
            if not (t.is_cuda and str(t.dtype) == "torch.int32"):
                raise ValueError("info must be a device int32 tensor")
            vals.append(ctypes.c_void_p(t.data_ptr()))
        else:
            vals.append(_ptr(a[n], n, sizes[n]))
    return Iteration(*vals)


def rkkt_iterate(p, args, stream=None):
    it = _iteration(p, args)
    _check(lib().rkkt_iterate(p.ptr, ctypes.byref(it), _stream(stream)), p.ptr)


def rkkt_graph_capture(p, args):
    it = _iteration(p, args)
    _check(lib().rkkt_graph_capture(p.ptr, ctypes.byref(it)), p.ptr)


def rkkt_graph_launch(p, stream=None):
    _check(lib().rkkt_graph_launch(p.ptr, _stream(stream)), p.ptr)


class Multi:
    """An rkkt_multi* (independent instances, one launch per kernel
    configuration) with the handles and buffers it uses (kept alive with it)."""

    def __init__(self, handles, args_list):
        n = len(handles)
        arr = (ctypes.c_void_p * n)(*[h.ptr for h in handles])
        its = (Iteration * n)(*[_iteration(h, a) for h, a in zip(handles, args_list)])
        ptr = ctypes.c_void_p()
        rc = lib().rkkt_multi_create(arr, its, n, ctypes.byref(ptr))
        if rc != RKKT_OK:
            raise RkktError(rc, lib().rkkt_multi_last_error(None).decode())
        self.ptr = ptr
        self.handles = list(handles)
        self.args = list(args_list)

    def _check(self, rc):
        if rc != RKKT_OK:
            raise RkktError(rc, lib().rkkt_multi_last_error(self.ptr).decode())

    def iterate(self, stream=None):
        self._check(lib().rkkt_multi_iterate(self.ptr, _stream(stream)))

    def capture(self):
        self._check(lib().rkkt_multi_capture(self.ptr))

    def launch(self, stream=None):
        self._check(lib().rkkt_multi_launch(self.ptr, _stream(stream)))

    @property
    def n_launches(self):
        return int(lib().rkkt_multi_launches(self.ptr))

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.rkkt_multi_destroy(self.ptr)
            self.ptr = None


class Batch:
    """An rkkt_batch* with the handles it captured (kept alive with it)."""

    def __init__(self, ptr, handles):
        self.ptr = ptr
        self.handles = handles

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.rkkt_batch_destroy(self.ptr)
            self.ptr = None


def rkkt_batch_create(handles, args_list):
    n = len(handles)
    arr = (ctypes.c_void_p * n)(*[h.ptr for h in handles])
    its = (Iteration * n)(*[_iteration(h, a) for h, a in zip(handles, args_list)])
    b = ctypes.c_void_p()
    _check(lib().rkkt_batch_create(arr, its, n, ctypes.byref(b)))
    return Batch(b, list(handles))


def rkkt_batch_launch(b, stream=None):
    _check(lib().rkkt_batch_launch(b.ptr, _stream(stream)))


def rkkt_batch_destroy(b):
    if b.ptr:
        lib().rkkt_batch_destroy(b.ptr)
        b.ptr = None


def rkkt_destroy(p):
    if p.ptr:
        lib().rkkt_destroy(p.ptr)
        p.ptr = None


def rkkt_last_error(p=None):
    return lib().rkkt_last_error(p.ptr if p is not None else None).decode()


# ------------------------------------------------------------ warm-start MLP
def _fptr(t, name, numel=None):
    if t is None:
        raise ValueError(f"{name} is None")
    if not (t.is_cuda and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous device tensor")
    if str(t.dtype) != "torch.float32":
        raise ValueError(f"{name} must be float32")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


class Mlp:
    """An rkkt_mlp* (rkkt_mlp.h); destroyed with the object."""

    def __init__(self, sizes, batch_max):
        sizes = np.ascontiguousarray(sizes, dtype=np.int32)
        h = ctypes.c_void_p()
        rc = lib().rkkt_mlp_create(sizes.ctypes.data_as(c_int_p), len(sizes) - 1, int(batch_max),
                                   ctypes.byref(h))
        if rc != RKKT_OK:
            raise RkktError(rc, lib().rkkt_mlp_last_error(None).decode())
        self.ptr = h
        self.sizes = [int(v) for v in sizes]
        self.batch_max = int(batch_max)
        self.n_params = int(lib().rkkt_mlp_n_params(h))

    def _check(self, rc):
        if rc != RKKT_OK:
            raise RkktError(rc, lib().rkkt_mlp_last_error(self.ptr).decode())

    def set_params(self, params, stream=None):
        self._check(lib().rkkt_mlp_set_params(self.ptr, _fptr(params, "params", self.n_params), _stream(stream)))

    def get_params(self, params, stream=None):
        self._check(lib().rkkt_mlp_get_params(self.ptr, _fptr(params, "params", self.n_params), _stream(stream)))

    def forward(self, x, y, stream=None):
        b = x.shape[0]
        self._check(lib().rkkt_mlp_forward(self.ptr, _fptr(x, "x", b * self.sizes[0]), b,
                                           _fptr(y, "y", b * self.sizes[-1]), _stream(stream)))

    def forward_static(self, x, y, stream=None):
        """rkkt_mlp_forward_static: the forward pass in the library's static
        workspace (no allocation; batch limited by that workspace)."""
        b = x.shape[0]
        self._check(lib().rkkt_mlp_forward_static(self.ptr, _fptr(x, "x", b * self.sizes[0]), b,
                                                  _fptr(y, "y", b * self.sizes[-1]), _stream(stream)))

    def gradients(self, x, t, grads, loss, stream=None):
        b = x.shape[0]
        g = _fptr(grads, "grads", self.n_params) if grads is not None else None
        self._check(lib().rkkt_mlp_gradients(self.ptr, _fptr(x, "x", b * self.sizes[0]),
                                             _fptr(t, "t", b * self.sizes[-1]), b, g,
                                             _fptr(loss, "loss", 1), _stream(stream)))

    def train_step(self, x, t, lr, loss, stream=None):
        b = x.shape[0]
        self._check(lib().rkkt_mlp_train_step(self.ptr, _fptr(x, "x", b * self.sizes[0]),
                                              _fptr(t, "t", b * self.sizes[-1]), b, float(lr),
                                              _fptr(loss, "loss", 1), _stream(stream)))

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.rkkt_mlp_destroy(self.ptr)
            self.ptr = None


def mlp_layout(sizes):
    """(offset of W_l, offset of b_l) per layer in the parameter vector."""
    out, off = [], 0
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        out.append((off, off + fi * fo))
        off += fi * fo + fo
    return out

